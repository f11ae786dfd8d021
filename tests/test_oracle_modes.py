"""Pin the oracle's CBC and CTR modes (SP 800-38A, with TDEA as the block cipher) to outside facts.

The paper is ECB only (Abstract); these modes reuse its cipher unchanged.  Pins:
- CBC, both directions: OpenSSL's DES-EDE3-CBC on the same keys, IV and data;
- CTR: OpenSSL's DES-EDE3-ECB applied to counter blocks that this test builds
  on its own (IV + j modulo 2^64, big-endian), XORed into the data -- the
  mode's definition with an outside cipher, including the wrap past 2^64 - 1;
- invariants: CTR is its own inverse; CBC decrypt inverts CBC encrypt; CBC's
  first block under a zero IV is ECB's; a one-block change in CBC ciphertext
  changes exactly two plaintext blocks (decryption's error propagation).
"""
import numpy as np
import pytest

import oracle
from paper_1305_4376_amd import inputs
from tests import _openssl

needs_openssl = pytest.mark.skipif(not _openssl.available(), reason="libcrypto not loadable")


def _iv(seed: int) -> bytes:
    return inputs.splitmix64(seed, 0, 1).astype("<u8").tobytes()


@needs_openssl
@pytest.mark.parametrize("keying", [3, 2, 1])
@pytest.mark.parametrize("n", [1, 2, 33, 4097])
def test_cbc_matches_openssl(keying, n):
    k = inputs.key_triple(inputs.KEY_SEED_BASE + 200 + keying, keying)
    iv = _iv(0xC0 + n)
    data = inputs.message(inputs.DATA_SEED_BASE + 200 + n, n)
    assert np.array_equal(oracle.tdes_cbc(*k, iv, data), _openssl.tdes_cbc(*k, iv, data))
    assert np.array_equal(oracle.tdes_cbc(*k, iv, data, decrypt=True), _openssl.tdes_cbc(*k, iv, data, decrypt=True))


def _counter_blocks(iv: bytes, n: int) -> np.ndarray:
    """IV + j (mod 2^64) for j < n, each as 8 big-endian bytes, built with Python integers."""
    t0 = int.from_bytes(iv, "big")
    return np.frombuffer(b"".join(((t0 + j) % (1 << 64)).to_bytes(8, "big") for j in range(n)), dtype=np.uint8)


@needs_openssl
@pytest.mark.parametrize("iv", [bytes(8), b"\xff" * 7 + b"\xfd", b"\x00\x00\x00\x00\xff\xff\xff\xfe",
                                 bytes.fromhex("0123456789abcdef")])
def test_ctr_matches_definition_with_openssl_cipher(iv):
    k = inputs.key_triple(inputs.KEY_SEED_BASE + 210)
    n = 1000
    data = inputs.message(inputs.DATA_SEED_BASE + 210, n)
    keystream = _openssl.tdes_ecb(*k, _counter_blocks(iv, n))
    assert np.array_equal(oracle.tdes_ctr(*k, iv, data), data ^ keystream)


def test_ctr_is_its_own_inverse_and_in_place_safe():
    k = inputs.key_triple(inputs.KEY_SEED_BASE + 211)
    iv = _iv(0xC1)
    data = inputs.message(inputs.DATA_SEED_BASE + 211, 777)
    once = oracle.tdes_ctr(*k, iv, data)
    assert not np.array_equal(once, data)
    assert np.array_equal(oracle.tdes_ctr(*k, iv, once), data)


def test_cbc_structure():
    k = inputs.key_triple(inputs.KEY_SEED_BASE + 212)
    iv = _iv(0xC2)
    data = inputs.message(inputs.DATA_SEED_BASE + 212, 64)
    ct = oracle.tdes_cbc(*k, iv, data)
    assert np.array_equal(oracle.tdes_cbc(*k, iv, ct, decrypt=True), data)
    # Zero IV: the first block is plain ECB.
    assert np.array_equal(oracle.tdes_cbc(*k, bytes(8), data[:8]), oracle.tdes_ecb(*k, data[:8]))
    # Block j of the ciphertext is ECB of (P_j xor C_{j-1}).
    prev = np.concatenate([np.frombuffer(iv, np.uint8), ct[:-8]])
    assert np.array_equal(ct, oracle.tdes_ecb(*k, data ^ prev))
    # Decryption: flipping a bit of C_5 garbles P_5 and flips the same bit of P_6 only.
    bad = ct.copy()
    bad[8 * 5 + 3] ^= 0x10
    pt = oracle.tdes_cbc(*k, iv, bad, decrypt=True)
    diff = (pt != data).reshape(-1, 8).any(axis=1)
    assert list(np.nonzero(diff)[0]) == [5, 6]
    assert np.array_equal(pt[48:56] ^ data[48:56], np.eye(1, 8, 3, dtype=np.uint8)[0] * 0x10)
