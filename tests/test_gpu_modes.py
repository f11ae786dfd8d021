"""GPU parity of the CTR and CBC-decrypt modes on the bitsliced core (beyond the paper, which is ECB only).

The oracle computes the modes from their definitions in NIST SP 800-38A
(oracle/des_oracle.c), pinned to OpenSSL in test_oracle_modes.py.  Here the
library's output must equal the oracle's bit for bit: over whole messages at
sizes that span several 2048-block tiles and a ragged tail, with 16-byte and
8-byte aligned buffers, IVs whose counter wraps past 2^64 - 1 inside the
message, and at the full 1 GiB size on sampled blocks (block j of CTR is the
one-block CTR at IV + j; block j of CBC decryption is the one-block CBC
decryption with IV = ciphertext block j - 1).  Tolerance: 0 bits.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1305_4376_amd as td
from paper_1305_4376_amd import inputs
from tests import _gpu

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 31, 2047, 2048, 2049, 4133, 3 * 2048, 9000]
IVS = [bytes(8), bytes.fromhex("0123456789abcdef"), b"\xff" * 7 + b"\xf0", b"\x00\x00\x00\x00\xff\xff\xff\xf8"]


def _setup(seed, n, offset=0):
    keys = inputs.key_triple(inputs.KEY_SEED_BASE + seed)
    host = inputs.message(inputs.DATA_SEED_BASE + seed, n)
    return keys, _gpu.device_sched(*keys), host, _gpu.to_device(host, offset), _gpu.empty_like_dev(8 * n, offset)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("offset", [0, 8])
def test_ctr_matches_oracle(n, offset):
    keys, sched, host, src, dst = _setup(300 + n % 97, n, offset)
    for iv in IVS:
        print(f"[modes] ctr n={n} offset={offset} iv={iv.hex()}", flush=True)
        td.tdes_ctr_crypt(sched, iv, src, dst, n)
        torch.cuda.synchronize()
        assert np.array_equal(dst.cpu().numpy(), oracle.tdes_ctr(*keys, iv, host)), iv.hex()


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("offset", [0, 8])
def test_cbc_decrypt_matches_oracle(n, offset):
    keys, sched, host, src, dst = _setup(400 + n % 89, n, offset)
    for iv in IVS[:2]:
        print(f"[modes] cbc n={n} offset={offset} iv={iv.hex()}", flush=True)
        td.tdes_cbc_decrypt(sched, iv, src, dst, n)
        torch.cuda.synchronize()
        assert np.array_equal(dst.cpu().numpy(), oracle.tdes_cbc(*keys, iv, host, decrypt=True)), iv.hex()


def test_ctr_in_place_and_round_trip():
    n = 5000
    keys, sched, host, src, dst = _setup(501, n)
    iv = IVS[2]
    td.tdes_ctr_crypt(sched, iv, src, src, n)          # in place
    torch.cuda.synchronize()
    assert np.array_equal(src.cpu().numpy(), oracle.tdes_ctr(*keys, iv, host))
    td.tdes_ctr_crypt(sched, iv, src, dst, n)          # decrypts
    torch.cuda.synchronize()
    assert np.array_equal(dst.cpu().numpy(), host)


def test_cbc_decrypt_inverts_oracle_encryption():
    n = 4133
    keys = inputs.key_triple(inputs.KEY_SEED_BASE + 502, 2)
    iv = IVS[1]
    plain = inputs.message(inputs.DATA_SEED_BASE + 502, n)
    ct = oracle.tdes_cbc(*keys, iv, plain)
    sched = _gpu.device_sched(*keys)
    src, dst = _gpu.to_device(ct), _gpu.empty_like_dev(8 * n)
    td.tdes_cbc_decrypt(sched, iv, src, dst, n)
    torch.cuda.synchronize()
    assert np.array_equal(dst.cpu().numpy(), plain)


def test_mode_argument_errors():
    keys, sched, host, src, dst = _setup(503, 64)

    def code(fn, *args):
        with pytest.raises(td.TdesError) as e:
            fn(*args)
        return e.value.code

    assert code(td.tdes_cbc_decrypt, sched, bytes(8), src, src, 64) == -3      # in place
    assert code(td.tdes_cbc_decrypt, sched, bytes(8), src[:256], src[8:264], 32) == -3
    assert code(td.tdes_ctr_crypt, sched, bytes(8), src[:256], src[8:264], 32) == -3
    assert code(td.tdes_ctr_crypt, sched, None, src, dst, 64) == -1
    assert code(td.tdes_cbc_decrypt, sched, None, src, dst, 64) == -1
    assert code(td.tdes_ctr_crypt, sched, bytes(8), src[4:], dst[4:], 8) == -2
    td.tdes_ctr_crypt(sched, bytes(8), src, dst, 0)                         # zero blocks: nothing to do
    td.tdes_cbc_decrypt(sched, bytes(8), src, src, 0)


@pytest.mark.parametrize("mode", ["ctr", "cbc"])
def test_one_gib_sampled(mode):
    """The 1 GiB message (2^27 blocks) in the launch configuration the benchmark times; sampled blocks."""
    n = 1 << 27
    keys = inputs.key_triple(inputs.KEY_SEED_BASE + 2)
    sched = _gpu.device_sched(*keys)
    seed = inputs.DATA_SEED_BASE + 2
    src = _gpu.device_message(seed, n)
    dst = torch.empty_like(src)
    iv = b"\xff\xff\xff\xff\xf8\x00\x00\x00"                               # the counter's low word wraps mid-message
    print(f"[modes] 1 GiB {mode}", flush=True)
    if mode == "ctr":
        td.tdes_ctr_crypt(sched, iv, src, dst, n)
    else:
        td.tdes_cbc_decrypt(sched, iv, src, dst, n)
    torch.cuda.synchronize()
    idx = _gpu.sample_indices(n, 4096, 3, boundaries=[k << 21 for k in range(1, 64, 5)])
    got = _gpu.gather_blocks(dst, idx).reshape(-1, 8)
    data = inputs.blocks_at(seed, idx).reshape(-1, 8)
    t0 = int.from_bytes(iv, "big")
    for r, j in enumerate(idx.tolist()):
        if mode == "ctr":
            want = oracle.tdes_ctr(*keys, ((t0 + j) % (1 << 64)).to_bytes(8, "big"), data[r])
        else:
            prev = iv if j == 0 else inputs.blocks_at(seed, np.array([j - 1])).tobytes()
            want = oracle.tdes_cbc(*keys, prev, data[r], decrypt=True)
        assert np.array_equal(got[r], want), f"block {j}"
