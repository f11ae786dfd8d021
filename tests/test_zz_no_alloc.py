"""GPU test of tdes_ecb_batch_static, the batched entry point that allocates nothing.

Its output must equal tdes_ecb_batch's on the same jobs, bit for bit (each
message ECB-EDE'd on its own: Abstract, Section II.A), on two calls in a row
with the second one smaller (the library's one scratch array per GPU keeps the
first call's plan and must not leak it into the second), and jobs that the
kernels refuse must leave their output untouched and be counted.
"""
import numpy as np
import pytest
import torch

import paper_1305_4376_amd as td
from paper_1305_4376_amd import inputs
from tests import _gpu
from tests._gpu import DEV

pytestmark = pytest.mark.gpu

EDGE = [0, 1, 2, 31, 32, 33, 2047, 2048, 2049, 4095, 4096, 4097, 6000]


def _table(n_keys, seed):
    keys = inputs.key_triples(seed, n_keys)
    host = np.concatenate([td.tdes_expand_key(k[:8].tobytes(), k[8:16].tobytes(), k[16:].tobytes()) for k in keys])
    dev = torch.empty(host.size, dtype=torch.uint8, device=DEV)
    td.tdes_sched_upload(host, dev)
    return keys, dev


def _jobs(lengths, n_keys, seed):
    """Inputs packed first, outputs after them; every third message in place; both directions."""
    lengths = np.asarray(lengths, dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(lengths)[:-1]]) * 8
    total = int(lengths.sum()) * 8
    jobs = np.zeros(lengths.size, dtype=td.JOB_DTYPE)
    jobs["in_off"], jobs["out_off"], jobs["n_blocks"] = starts, starts + total, lengths
    sel = np.arange(lengths.size) % 3 == 1
    jobs["out_off"][sel] = starts[sel]
    rng = np.random.default_rng(seed)
    jobs["sched_idx"] = rng.integers(0, n_keys, lengths.size)
    jobs["direction"] = rng.integers(0, 2, lengths.size)
    return jobs, total


def _run_both(jobs, total, table, n_keys, seed):
    """The same jobs through tdes_ecb_batch and tdes_ecb_batch_static; returns both buffers and the refused count."""
    ref = torch.empty(2 * total + 64, dtype=torch.uint8, device=DEV)
    td.tdes_fill_splitmix64(ref, ref.numel() // 8, seed, 0)
    got = ref.clone()
    ctx = td.tdes_ctx_create()
    try:
        td.tdes_ecb_batch(ctx, jobs, table, n_keys, ref)
        torch.cuda.synchronize()
    finally:
        td.tdes_ctx_destroy(ctx)
    dev_jobs = torch.from_numpy(jobs.view(np.uint8).copy()).to(DEV)
    rejected = torch.full((1,), 0xFFFF, dtype=torch.int32, device=DEV)
    td.tdes_ecb_batch_static(dev_jobs, jobs.size, table, n_keys, got, dev_rejected=rejected)
    torch.cuda.synchronize()
    return ref, got, int(rejected.item())


def _check_oracle(jobs, keys, buf, seed, per_job=64):
    host = buf.cpu().numpy()
    words = inputs.message(seed, host.size // 8)
    for j, job in enumerate(jobs):
        n = int(job["n_blocks"])
        if n == 0:
            continue
        idx = np.unique(np.concatenate([[0, n - 1], np.random.default_rng(j).integers(0, n, per_job)]))
        k = keys[job["sched_idx"]]
        src = words[int(job["in_off"]):int(job["in_off"]) + 8 * n].reshape(-1, 8)[idx].reshape(-1)
        want = _gpu.oracle_on_blocks((k[:8].tobytes(), k[8:16].tobytes(), k[16:].tobytes()), src,
                                     decrypt=bool(job["direction"]))
        out = host[int(job["out_off"]):int(job["out_off"]) + 8 * n].reshape(-1, 8)[idx].reshape(-1)
        assert np.array_equal(out, want), f"job {j}: {n} blocks, direction {int(job['direction'])}"


def test_static_batch_equals_batch_twice():
    n_keys = 97
    keys, table = _table(n_keys, 0x57A1)
    # first call: 1500 messages, log-uniform lengths up to 2^15 blocks, plus the edge lengths
    lengths = np.concatenate([inputs.log_uniform_lengths(0x57A2, 1500, 1 << 15), EDGE])
    jobs, total = _jobs(lengths, n_keys, 0x57A3)
    print(f"[static] call 1: {jobs.size} jobs, {total // 8} blocks", flush=True)
    ref, got, rejected = _run_both(jobs, total, table, n_keys, 0x57A4)
    assert rejected == 0
    assert torch.equal(ref, got), "static batch differs from tdes_ecb_batch (call 1)"
    _check_oracle(jobs, keys, got, 0x57A4)
    # second call, smaller: fewer and shorter messages
    lengths = np.concatenate([inputs.log_uniform_lengths(0x57A5, 40, 5000), EDGE[:6]])
    jobs, total = _jobs(lengths, n_keys, 0x57A6)
    print(f"[static] call 2: {jobs.size} jobs, {total // 8} blocks", flush=True)
    ref, got, rejected = _run_both(jobs, total, table, n_keys, 0x57A7)
    assert rejected == 0
    assert torch.equal(ref, got), "static batch differs from tdes_ecb_batch (call 2)"
    _check_oracle(jobs, keys, got, 0x57A7)


def test_static_batch_refuses_malformed_jobs():
    n_keys = 5
    keys, table = _table(n_keys, 0x57B1)
    lengths = [3000, 100, 2048, 77, 5000, 64]
    jobs, total = _jobs(lengths, n_keys, 0x57B2)
    buf_bytes = 2 * total + 64 + 8192          # an unused tail after the outputs
    bad = jobs.copy()
    bad["sched_idx"][1] = n_keys               # no such schedule
    bad["direction"][3] = 2                    # no such direction
    bad["out_off"][4] = 2 * total + 64         # 5000 blocks from the unused tail: past the buffer
    seed = 0x57B3
    buf = torch.empty(buf_bytes, dtype=torch.uint8, device=DEV)
    td.tdes_fill_splitmix64(buf, buf_bytes // 8, seed, 0)
    before = buf.cpu().numpy()
    dev_jobs = torch.from_numpy(bad.view(np.uint8).copy()).to(DEV)
    rejected = torch.zeros(1, dtype=torch.int32, device=DEV)
    print("[static] malformed jobs", flush=True)
    td.tdes_ecb_batch_static(dev_jobs, bad.size, table, n_keys, buf, dev_rejected=rejected)
    torch.cuda.synchronize()
    assert int(rejected.item()) == 3
    after = buf.cpu().numpy()
    for j in (1, 3):  # refused: output bytes unchanged
        lo, hi = int(bad["out_off"][j]), int(bad["out_off"][j]) + 8 * int(bad["n_blocks"][j])
        assert np.array_equal(after[lo:hi], before[lo:hi]), f"refused job {j} wrote its output"
    lo = int(bad["out_off"][4])
    assert np.array_equal(after[lo:], before[lo:]), "refused job 4 wrote into the tail"
    good = np.array([0, 2, 5])
    _check_oracle(bad[good], keys, torch.from_numpy(after), seed, per_job=4096)
    with pytest.raises(td.TdesError) as e:
        td.tdes_ecb_batch_static(dev_jobs.data_ptr(), td.TDES_STATIC_MAX_JOBS + 1, table, n_keys, buf,
                                 base_bytes=buf_bytes)
    assert e.value.code == -4
