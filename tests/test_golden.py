"""Stored EDE vectors (tests/golden/tdes_ecb_vectors.txt): oracle drift and an outside pin."""
import os

import numpy as np
import pytest

import oracle
from tests import _openssl

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tdes_ecb_vectors.txt")


def load_vectors():
    out = []
    for line in open(PATH):
        if line.startswith("#") or not line.strip():
            continue
        keying, k1, k2, k3, pt, ct = line.split()
        out.append((int(keying), bytes.fromhex(k1), bytes.fromhex(k2), bytes.fromhex(k3),
                    np.frombuffer(bytes.fromhex(pt), np.uint8), np.frombuffer(bytes.fromhex(ct), np.uint8)))
    return out


def test_vectors_present():
    v = load_vectors()
    assert len(v) == 24 and {x[0] for x in v} == {1, 2, 3}


def test_oracle_reproduces_vectors():
    for _, k1, k2, k3, pt, ct in load_vectors():
        assert np.array_equal(oracle.tdes_ecb(k1, k2, k3, pt), ct)
        assert np.array_equal(oracle.tdes_ecb(k1, k2, k3, ct, decrypt=True), pt)


@pytest.mark.skipif(not _openssl.available(), reason="libcrypto not loadable")
def test_vectors_match_openssl():
    for _, k1, k2, k3, pt, ct in load_vectors():
        assert np.array_equal(_openssl.tdes_ecb(k1, k2, k3, pt), ct)
