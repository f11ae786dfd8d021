"""Pin the oracle to an outside implementation: OpenSSL's single DES and DES-EDE3-ECB.

This fixes every table entry, the bit and byte order of a block (the standard's:
bit 1 is the most significant bit of byte 0), the key-parity handling and the
EDE wiring of the three keys (Section II.A: encrypt K1, decrypt K2, encrypt K3;
decryption in reverse).  Skipped where libcrypto cannot be loaded.
"""
import numpy as np
import pytest

import oracle
from paper_1305_4376_amd import inputs
from tests import _openssl

pytestmark = pytest.mark.skipif(not _openssl.available(), reason="libcrypto not loadable")


@pytest.mark.parametrize("keying", [3, 2, 1])
@pytest.mark.parametrize("decrypt", [False, True])
def test_tdes_ecb_matches_openssl(keying, decrypt):
    k = inputs.key_triple(inputs.KEY_SEED_BASE + 100 + keying, keying)
    n = 1 << 15
    data = inputs.message(inputs.DATA_SEED_BASE + 100 + keying, n)
    want = _openssl.tdes_ecb(*k, data, decrypt=decrypt)
    got = oracle.tdes_ecb(*k, data, decrypt=decrypt, threads=8)
    assert np.array_equal(got, want)


def test_tdes_ecb_many_keys_matches_openssl():
    # Many independent key triples, few blocks each: exercises the key schedule broadly.
    triples = inputs.key_triples(0x51, 256)
    for t in range(triples.shape[0]):
        k1, k2, k3 = (triples[t, 8 * i: 8 * i + 8].tobytes() for i in range(3))
        data = inputs.message(0x52 + t, 16)
        assert np.array_equal(oracle.tdes_ecb(k1, k2, k3, data), _openssl.tdes_ecb(k1, k2, k3, data))
        assert np.array_equal(oracle.tdes_ecb(k1, k2, k3, data, decrypt=True),
                              _openssl.tdes_ecb(k1, k2, k3, data, decrypt=True))


def test_single_des_matches_openssl():
    words = inputs.splitmix64(0x53, 0, 2 * 2000).astype("<u8").view(np.uint8).reshape(2000, 16)
    for row in words:
        key, block = row[:8].tobytes(), row[8:].tobytes()
        for dec in (False, True):
            assert oracle.des_block(key, block, dec) == _openssl.des_block(key, block, dec)


def test_special_blocks_match_openssl():
    # All-zero and all-one blocks and keys, and unparitied keys.
    k = inputs.key_triple(0x54)
    for data in (np.zeros(64, np.uint8), np.full(64, 0xFF, np.uint8)):
        for key in (k, (b"\x00" * 8,) * 3, (b"\xff" * 8,) * 3, (b"\x00" * 8, b"\xff" * 8, b"\x00" * 8)):
            assert np.array_equal(oracle.tdes_ecb(*key, data), _openssl.tdes_ecb(*key, data))
