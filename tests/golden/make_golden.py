"""Writes tdes_ecb_vectors.txt from the oracle only.

The paper prints no worked example (its figures and kernel are not given), so
these vectors are the oracle's own output on seeded inputs; test_golden.py
checks them against OpenSSL, which pins them to an outside implementation, and
against the current oracle, which catches drift.

Each line: keying k1 k2 k3 plaintext ciphertext (hex; 4 blocks per line).
Run from the repository root: python tests/golden/make_golden.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1305_4376_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tdes_ecb_vectors.txt")


def main():
    lines = ["# Triple-DES EDE, ECB: keying k1 k2 k3 plaintext ciphertext (hex, 4 blocks)",
             "# EDE order and its inverse: Section II.A; blocks independent: Abstract.",
             "# Written by make_golden.py from the oracle; pinned to OpenSSL by test_golden.py."]
    for i in range(24):
        keying = (3, 2, 1)[i % 3]
        k = inputs.key_triple(0x601D + i, keying)
        pt = inputs.message(0x601D0 + i, 4)
        ct = oracle.tdes_ecb(*k, pt)
        lines.append(" ".join([str(keying), k[0].hex(), k[1].hex(), k[2].hex(), pt.tobytes().hex(), ct.tobytes().hex()]))
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
