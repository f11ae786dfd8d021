"""Unit tests of the bitsliced core's pieces, run on the device (kernels in tests/units/k_units.hip).

These localise a failure that the end-to-end parity tests would only report
as a wrong block:
- every S-box circuit on all 64 inputs, plain and with a key mask of 0 and
  ~0, against the oracle's S-box table (FIPS 46-3);
- the 32x32 bit transpose against a transpose computed here;
- the per-lane-key rounds, round by round, against the oracle's (L_i, R_i)
  trace of single DES;
- each folded DES stage (the one-key-per-wave path, with the schedule's
  folded words) against the oracle's L16 R16 for that stage's key and
  direction.
Tolerance: 0 bits.
"""
import ctypes
import os

import numpy as np
import pytest
import torch

import oracle
import paper_1305_4376_amd as td
from paper_1305_4376_amd import inputs
from tests._gpu import DEV

pytestmark = pytest.mark.gpu

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "units", "libtdes_units.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        raise ImportError(f"{LIB} is missing: build with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB)
    vp = ctypes.c_void_p
    lib.units_sbox.argtypes = [vp]
    lib.units_transpose.argtypes = [vp, vp]
    lib.units_rounds.argtypes = [vp, vp, ctypes.c_int, vp]
    lib.units_folded_stage.argtypes = [vp, vp, ctypes.c_int, vp]
    return lib


def _words(n):
    return torch.zeros(n, dtype=torch.int32, device=DEV)


def _host_u32(t):
    return t.cpu().numpy().view(np.uint32)


def test_sbox_circuits_on_device(lib):
    out = _words(8 * 3 * 2 * 4)
    assert lib.units_sbox(out.data_ptr()) == 0
    got = _host_u32(out).reshape(8, 3, 2, 4)
    table = np.frombuffer(bytes(oracle.table("SBOX")), dtype=np.uint8).reshape(8, 4, 16)
    for b in range(8):
        for p in range(64):
            row, col = ((p >> 5) & 1) * 2 + (p & 1), (p >> 1) & 15
            s = int(table[b, row, col])
            for variant in range(3):
                for j in range(4):
                    want = ((s >> (3 - j)) & 1) ^ (1 if variant == 2 else 0)
                    assert (int(got[b, variant, p // 32, j]) >> (p % 32)) & 1 == want, (b, variant, p, j)


def test_transpose_on_device(lib):
    w = inputs.splitmix64(0xA1, 0, 32).astype(np.uint32)
    src = torch.from_numpy(w.view(np.int32).copy()).to(DEV)
    out = _words(32)
    assert lib.units_transpose(src.data_ptr(), out.data_ptr()) == 0
    got = _host_u32(out)
    bits = (w[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1   # bits[row, col]
    want = (bits.T.astype(np.uint64) << np.arange(32, dtype=np.uint64)[None, :]).sum(axis=1).astype(np.uint32)
    assert np.array_equal(got, want)


def _blocks(seed):
    data = inputs.message(seed, 32)
    return data, torch.from_numpy(data.view(np.int32).copy()).to(DEV)


def _value(planes, j):
    """Bit j of 32 planes, plane k as bit 31 - k (bit 1 of the half is the most significant)."""
    v = 0
    for k in range(32):
        v |= ((int(planes[k]) >> j) & 1) << (31 - k)
    return v


@pytest.mark.parametrize("keying", [3, 1])
def test_rounds_match_oracle_trace(lib, keying):
    k1, k2, k3 = inputs.key_triple(inputs.KEY_SEED_BASE + 300 + keying, keying)
    data, blocks = _blocks(inputs.DATA_SEED_BASE + 300)
    words = td.tdes_expand_key(k1, k2, k3).view("<u4")
    ks = torch.from_numpy(words[:32].view(np.int32).copy()).to(DEV)   # the first stage: K1's 16 rounds
    out = _words(17 * 64)
    assert lib.units_rounds(blocks.data_ptr(), ks.data_ptr(), 16, out.data_ptr()) == 0
    planes = _host_u32(out).reshape(17, 64)
    for j in range(32):
        trace = oracle.des_trace(k1, data[8 * j: 8 * j + 8].tobytes())
        for i in range(17):
            x, y = planes[i, :32], planes[i, 32:]
            lo, hi = (y, x) if i % 2 else (x, y)           # in place: the halves trade roles each round
            got = (_value(lo, j) << 32) | _value(hi, j)
            assert got == trace[i], f"block {j} after round {i}"


@pytest.mark.parametrize("direction", [td.TDES_ENCRYPT, td.TDES_DECRYPT])
def test_folded_stages_match_oracle(lib, direction):
    k1, k2, k3 = inputs.key_triple(inputs.KEY_SEED_BASE + 310)
    data, blocks = _blocks(inputs.DATA_SEED_BASE + 310)
    sched = td.tdes_expand_key(k1, k2, k3)
    dir_words = torch.from_numpy(sched.view(np.int32)[direction * (td.TDES_SCHED_BYTES // 8):].copy()).to(DEV)
    stages = [(k1, False), (k2, True), (k3, False)] if direction == td.TDES_ENCRYPT else \
             [(k3, True), (k2, False), (k1, True)]
    for stage, (key, decrypt) in enumerate(stages):
        out = _words(64)
        assert lib.units_folded_stage(blocks.data_ptr(), dir_words.data_ptr(), stage, out.data_ptr()) == 0
        planes = _host_u32(out)
        for j in range(32):
            want = oracle.des_trace(key, data[8 * j: 8 * j + 8].tobytes(), decrypt)[16]
            got = (_value(planes[:32], j) << 32) | _value(planes[32:], j)
            assert got == want, f"stage {stage} block {j}"
