"""Structural pins on the oracle's DES tables (the standard's tables, which the paper names but does not print).

Each check is a property the standard's tables must have, stated independently
of how the oracle uses them, so that a transcription slip (a swapped or retyped
entry) fails at least one of them.  The end-to-end comparison with OpenSSL in
test_oracle_openssl.py pins every entry exactly.
"""
import itertools

import oracle


def test_ip_fp_are_inverse_permutations():
    ip, fp = oracle.table("IP"), oracle.table("FP")
    assert sorted(ip) == list(range(1, 65))
    assert sorted(fp) == list(range(1, 65))
    # FP[IP] and IP[FP] are the identity: FP = IP^-1.
    assert [ip[fp[i] - 1] for i in range(64)] == list(range(1, 65))
    assert [fp[ip[i] - 1] for i in range(64)] == list(range(1, 65))


def test_ip_is_a_transposed_bit_matrix():
    # IP reads the even bit positions (2,4,6,8) of the eight bytes, then the odd ones,
    # taking bytes last-to-first: output row r is byte position q(r) of bytes 8..1.
    ip = oracle.table("IP")
    order = [2, 4, 6, 8, 1, 3, 5, 7]
    for r in range(8):
        row = ip[8 * r: 8 * r + 8]
        assert row == [8 * (7 - j) + order[r] for j in range(8)]


def test_expansion_structure():
    e = oracle.table("E")
    counts = {b: e.count(b) for b in range(1, 33)}
    assert all(c in (1, 2) for c in counts.values())
    assert sum(1 for c in counts.values() if c == 2) == 16
    # Box s reads the six consecutive bits 4s .. 4s+5 of R (cyclically, 1-based, with bit 0 = bit 32).
    for s in range(8):
        assert e[6 * s: 6 * s + 6] == [((4 * s + j - 1) % 32) + 1 for j in range(6)]


def test_p_is_a_permutation_spreading_boxes():
    p = oracle.table("P")
    assert sorted(p) == list(range(1, 33))
    # Design properties of P (published with the S-box criteria): through E, the four
    # outputs of a box reach six different boxes of the next round, no two outputs the
    # same box, two of them as end bits (read by two boxes) and two as middle bits, and
    # never the box itself.
    e = oracle.table("E")
    for box in range(8):
        outs = [p.index(4 * box + j + 1) + 1 for j in range(4)]  # positions in f(R)
        reached = [{i // 6 for i, x in enumerate(e) if x == b} for b in outs]
        union = set().union(*reached)
        assert len(union) == 6 and sum(len(r) for r in reached) == 6
        assert sorted(len(r) for r in reached) == [1, 1, 2, 2]
        assert box not in union


def test_key_schedule_tables():
    pc1, pc2, shifts = oracle.table("PC1"), oracle.table("PC2"), oracle.table("SHIFTS")
    assert len(set(pc1)) == 56 and all(1 <= b <= 64 and b % 8 != 0 for b in pc1)
    assert len(set(pc2)) == 48 and all(1 <= b <= 56 for b in pc2)
    # The first 24 subkey bits come from C, the last 24 from D.
    assert all(b <= 28 for b in pc2[:24]) and all(b > 28 for b in pc2[24:])
    assert sum(shifts) == 28
    assert shifts.count(1) == 4 and shifts.count(2) == 12
    assert [i for i, s in enumerate(shifts) if s == 1] == [0, 1, 8, 15]


def _sbox(s):
    flat = oracle.table("SBOX")
    tab = flat[64 * s: 64 * s + 64]

    def f(x):  # x: 6-bit input b1..b6 with b1 the MSB
        row = ((x >> 4) & 2) | (x & 1)
        col = (x >> 1) & 15
        return tab[16 * row + col]
    return tab, f


def test_sbox_rows_are_permutations():
    for s in range(8):
        tab, _ = _sbox(s)
        for r in range(4):
            assert sorted(tab[16 * r: 16 * r + 16]) == list(range(16))


def test_sbox_design_criteria():
    """The S-box design criteria published by the standard's designers (Coppersmith, 1994).

    S-4: inputs differing in one bit give outputs differing in at least two bits.
    S-5: inputs differing exactly in the two middle bits give outputs differing in at least two bits.
    S-6: inputs differing in the first two bits and agreeing in the last two never give equal outputs.
    S-7: for a fixed nonzero input difference, at most 8 of the 32 input pairs share an output difference.
    """
    for s in range(8):
        _, f = _sbox(s)
        for x in range(64):
            for bit in range(6):
                assert bin(f(x) ^ f(x ^ (1 << bit))).count("1") >= 2, (s, x, bit)
            assert bin(f(x) ^ f(x ^ 0b001100)).count("1") >= 2, (s, x)
            for e, ff in itertools.product((0, 1), repeat=2):
                d = 0b110000 | (e << 3) | (ff << 2)
                assert f(x) != f(x ^ d), (s, x, d)
        for d in range(1, 64):
            hist = {}
            for x in range(64):
                od = f(x) ^ f(x ^ d)
                hist[od] = hist.get(od, 0) + 1
            # Each unordered pair is counted twice above: at most 8 pairs = 16 ordered inputs.
            assert max(hist.values()) <= 16, (s, d)
