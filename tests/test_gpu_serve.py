"""GPU tests of the serving engine (continuous batching over resident key schedules).

The pin: every request's output is ECB-EDE of its own payload under its own
key (Abstract, Section II.A), the same bit for bit whether it runs alone or in
a mix of overlapping requests, and equal to the oracle on every block.  One
test runs the serving workload's own shape (65536 resident triples, requests
of 512 B .. 16 MiB, 2^24-block steps, three steps in flight, a 64 GiB budget).
Admission is checked against the device-memory budget.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_1305_4376_amd as td
from paper_1305_4376_amd import inputs
from tests import _gpu
from tests._gpu import DEV

pytestmark = pytest.mark.gpu

N_KEYS = 512


@pytest.fixture(scope="module")
def table():
    keys = inputs.key_triples(0x5E01, N_KEYS)
    host = np.concatenate([td.tdes_expand_key(k[:8].tobytes(), k[8:16].tobytes(), k[16:].tobytes()) for k in keys])
    dev = torch.empty(host.size, dtype=torch.uint8, device=DEV)
    td.tdes_sched_upload(host, dev)
    return keys, dev


def _requests(n, seed, max_blocks=1 << 15):
    rng = np.random.default_rng(seed)
    reqs = np.zeros(n, dtype=td.REQUEST_DTYPE)
    reqs["n_blocks"] = inputs.log_uniform_lengths(seed, n, max_blocks)
    reqs["key_id"] = rng.integers(0, N_KEYS, n)
    reqs["direction"] = rng.integers(0, 2, n)
    reqs["seed"] = seed * 1000003 + np.arange(n)
    reqs["user_tag"] = np.arange(n)
    return reqs


def _outputs_by_tag(server, completions, reqs):
    """Copies each kept output to the host (device-to-device through a tensor), then releases it."""
    res = {}
    for c in completions:
        assert c["status"] == 0, c
        n = int(reqs[c["user_tag"]]["n_blocks"])
        buf = torch.empty(8 * n, dtype=torch.uint8, device=DEV)
        _copy_dev(buf.data_ptr(), int(c["dev_out"]), 8 * n)
        torch.cuda.synchronize()
        res[int(c["user_tag"])] = buf.cpu().numpy()
        td.tdes_server_release(server, int(c["id"]))
    return res


_hip = None


def _copy_dev(dst, src, nbytes):
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    assert _hip.hipMemcpy(dst, src, nbytes, 3) == 0  # hipMemcpyDeviceToDevice


def _check_oracle(keys, req, out):
    """Every block of a request's output against the oracle on its payload (generated from the request's seed)."""
    n = int(req["n_blocks"])
    k = keys[req["key_id"]]
    src = inputs.payload(int(req["seed"]), n)
    want = _gpu.oracle_on_blocks((k[:8].tobytes(), k[8:16].tobytes(), k[16:].tobytes()), src,
                                 decrypt=bool(req["direction"]))
    assert out.size == want.size
    if not np.array_equal(out, want):
        bad = np.flatnonzero((out != want).reshape(-1, 8).any(1))
        raise AssertionError(f"request tag {int(req['user_tag'])} (key {int(req['key_id'])}, {n} blocks): "
                             f"{bad.size} blocks differ from the oracle, first {bad[0]}")


def test_alone_equals_in_the_mix(table):
    keys, dev_table = table
    reqs = _requests(200, 0x5E02)
    probe = [3, 50, 77, 150, 199]
    # Alone: one request at a time through its own server.
    server = td.tdes_server_create(dev_table, N_KEYS, 1 << 30, max_inflight=2, keep_outputs=True)
    try:
        alone = {}
        for i in probe:
            td.tdes_server_submit(server, reqs[i])
            td.tdes_server_wait_idle(server, 60)
            alone.update(_outputs_by_tag(server, td.tdes_server_poll(server), reqs))
        assert td.tdes_server_stats(server)["pool_bytes_in_use"] == 0
    finally:
        td.tdes_server_destroy(server)
    # In the mix: all 200 arrive over ~20 ms and overlap on the device.
    server = td.tdes_server_create(dev_table, N_KEYS, 1 << 30, max_inflight=3, max_step_jobs=64, keep_outputs=True)
    try:
        arrival = np.sort(np.random.default_rng(7).uniform(0, 0.02, reqs.size))
        done = td.tdes_server_run_trace(server, reqs, arrival)
        assert (done["status"] == 0).all()
        assert (done["t_complete"] >= done["t_launch"]).all() and (done["t_launch"] >= done["t_admit"]).all()
        assert (done["t_admit"] >= done["t_arrival"] - 1e-9).all()
        stats = td.tdes_server_stats(server)
        assert stats["steps"] > 1 and stats["completed"] == reqs.size
        mixed = _outputs_by_tag(server, done, reqs)
        assert td.tdes_server_stats(server)["pool_bytes_in_use"] == 0
    finally:
        td.tdes_server_destroy(server)
    for i in probe:
        assert np.array_equal(alone[i], mixed[i]), f"request {i} differs alone and in the mix"
    for i in range(reqs.size):
        _check_oracle(keys, reqs[i], mixed[i])


def test_tuned_steps_every_block(table):
    """Steps under a non-default batch shape (128 threads, 8 groups per CU, every remainder as a
    wave tile below 1024 blocks, two tiles per draw): every block of every request against the oracle."""
    keys, dev_table = table
    reqs = _requests(160, 0x5E1F, max_blocks=1 << 16)
    server = td.tdes_server_create(dev_table, N_KEYS, 1 << 30, max_inflight=3, max_step_jobs=48,
                                   keep_outputs=True, tuning=(128, 8, 1024, 2))
    try:
        arrival = np.sort(np.random.default_rng(16).uniform(0, 0.01, reqs.size))
        print(f"[serve] tuned steps: {reqs.size} requests", flush=True)
        done = td.tdes_server_run_trace(server, reqs, arrival)
        assert (done["status"] == 0).all()
        assert td.tdes_server_stats(server)["steps"] > 1
        mixed = _outputs_by_tag(server, done, reqs)
    finally:
        td.tdes_server_destroy(server)
    for i in range(reqs.size):
        _check_oracle(keys, reqs[i], mixed[i])


def test_backlog_steps_every_block(table):
    """A long queue served in larger steps (backlog_step_blocks): fewer steps than with the fixed step
    cap on the same trace, and every block of every request still equal to the oracle and to the
    fixed-cap run."""
    keys, dev_table = table
    reqs = _requests(160, 0x5E2B, max_blocks=1 << 16)
    arrival = np.zeros(reqs.size)
    outs, steps = [], []
    for backlog in (0, 1 << 20):
        server = td.tdes_server_create(dev_table, N_KEYS, 1 << 30, max_inflight=2, max_step_jobs=4096,
                                       max_step_blocks=1 << 16, keep_outputs=True, backlog_step_blocks=backlog)
        try:
            print(f"[serve] backlog steps: cap {backlog}, {reqs.size} requests at once", flush=True)
            done = td.tdes_server_run_trace(server, reqs, arrival)
            assert (done["status"] == 0).all()
            steps.append(td.tdes_server_stats(server)["steps"])
            outs.append(_outputs_by_tag(server, done, reqs))
        finally:
            td.tdes_server_destroy(server)
    assert steps[1] < steps[0], steps
    for i in range(reqs.size):
        assert np.array_equal(outs[0][i], outs[1][i]), i
        _check_oracle(keys, reqs[i], outs[1][i])


def test_server_rejects_bad_tuning(table):
    _, dev_table = table
    for kw in ({"tuning": (96, 4, 0, 0)}, {"tuning": (256, 4, 4096, 0)}, {"tuning": (256, 4, 0, 17)}):
        with pytest.raises(td.TdesError) as e:
            td.tdes_server_create(dev_table, N_KEYS, 1 << 20, **kw)
        assert e.value.code == -7, kw


def test_budget_admission_and_cancel(table):
    keys, dev_table = table
    budget = 64 << 20
    reqs = _requests(120, 0x5E03, max_blocks=1 << 19)   # up to 4 MiB each: many will not fit at once
    server = td.tdes_server_create(dev_table, N_KEYS, budget, max_inflight=2, max_step_jobs=16)
    try:
        big = np.zeros(1, dtype=td.REQUEST_DTYPE)
        big["n_blocks"] = (budget // 16) + 1                 # input + output just over the budget
        with pytest.raises(td.TdesError) as e:
            td.tdes_server_submit(server, big)
        assert e.value.code == -10
        bad = reqs[:1].copy()
        bad["key_id"] = N_KEYS
        with pytest.raises(td.TdesError) as e:
            td.tdes_server_submit(server, bad)
        assert e.value.code == -4
        done = td.tdes_server_run_trace(server, reqs, np.zeros(reqs.size))
        assert (done["status"] == 0).all()
        stats = td.tdes_server_stats(server)
        assert stats["peak_pool_bytes"] <= budget
        assert stats["completed"] == reqs.size and stats["pool_bytes_in_use"] == 0
        assert stats["bytes"] == int(reqs["n_blocks"].sum()) * 8
        # Cancel: fill the budget with one request, queue two more, cancel the last while it waits.
        fill = np.zeros(1, dtype=td.REQUEST_DTYPE)
        fill["n_blocks"] = budget // 16 - 4096
        ids = [td.tdes_server_submit(server, fill), td.tdes_server_submit(server, reqs[0]),
               td.tdes_server_submit(server, reqs[1])]
        canceled = True
        try:
            td.tdes_server_cancel(server, ids[2])
        except td.TdesError as err:       # it may already have been admitted
            assert err.code == -11
            canceled = False
        td.tdes_server_wait_idle(server, 60)
        got = {int(c["id"]): int(c["status"]) for c in td.tdes_server_poll(server)}
        assert got[ids[0]] == 0 and got[ids[1]] == 0
        assert got[ids[2]] == (-11 if canceled else 0)
    finally:
        td.tdes_server_destroy(server)


def test_host_payloads(table):
    keys, dev_table = table
    server = td.tdes_server_create(dev_table, N_KEYS, 1 << 28, max_inflight=2)
    try:
        n = 5000
        host_in = inputs.message(0x5E04, n)
        host_out = np.zeros_like(host_in)
        req = np.zeros(1, dtype=td.REQUEST_DTYPE)
        req["n_blocks"] = n
        req["key_id"] = 9
        req["direction"] = 1
        req["host_in"] = host_in.ctypes.data
        req["host_out"] = host_out.ctypes.data
        td.tdes_server_submit(server, req)
        td.tdes_server_wait_idle(server, 60)
        (c,) = td.tdes_server_poll(server)
        assert c["status"] == 0 and c["dev_out"] == 0
        k = keys[9]
        want = _gpu.oracle_on_blocks((k[:8].tobytes(), k[8:16].tobytes(), k[16:].tobytes()), host_in, decrypt=True)
        assert np.array_equal(host_out, want)
    finally:
        td.tdes_server_destroy(server)


SERVE_KEYS = 65536


def test_serving_workload_shape_every_block():
    """The serving workload's shape: 65536 resident three-key triples (schedule offsets up to
    ~100 MiB into the table), requests log-uniform from 64 to 2^21 blocks (512 B .. 16 MiB) including
    one of exactly 2^21 blocks and key ids at the top of the table, 50/50 directions, a 64 GiB budget,
    three steps in flight of at most 2^24 blocks, outputs kept on the device.  Every block of every
    request is compared with the oracle, and 24 requests (the largest among them) are also run alone
    and compared with their result in the mix."""
    keys = inputs.key_triples(0x5E10, SERVE_KEYS)
    host = np.concatenate([td.tdes_expand_key(k[:8].tobytes(), k[8:16].tobytes(), k[16:].tobytes()) for k in keys])
    dev_table = torch.empty(host.size, dtype=torch.uint8, device=DEV)
    td.tdes_sched_upload(host, dev_table)
    del host
    n = 96
    rng = np.random.default_rng(0x5E11)
    reqs = np.zeros(n, dtype=td.REQUEST_DTYPE)
    u = rng.random(n)
    reqs["n_blocks"] = np.floor(np.exp(np.log(64) + u * (np.log(2 ** 21) - np.log(64)))).astype(np.int64)
    reqs["n_blocks"][[5, 60]] = [1 << 21, 64]
    reqs["key_id"] = rng.integers(0, SERVE_KEYS, n)
    reqs["key_id"][[1, 2, 3, 5, 90]] = [SERVE_KEYS - 1, SERVE_KEYS - 2, 0, SERVE_KEYS - 1, SERVE_KEYS - 3]
    reqs["direction"] = rng.integers(0, 2, n)
    reqs["seed"] = 0x5E120000 + np.arange(n)
    reqs["user_tag"] = np.arange(n)
    probe = sorted(set([5, 1, 2, 3, 60, 90] + rng.choice(n, 24, replace=False).tolist()))[:24]
    if 5 not in probe:
        probe[-1] = 5
    print(f"[serve] {n} requests, {int(reqs['n_blocks'].sum())} blocks, mixed run", flush=True)
    server = td.tdes_server_create(dev_table, SERVE_KEYS, 64 << 30, max_inflight=3, max_step_jobs=4096,
                                   max_step_blocks=1 << 24, keep_outputs=True)
    try:
        arrival = np.cumsum(rng.exponential(0.0002, n))
        done = td.tdes_server_run_trace(server, reqs, arrival)
        assert (done["status"] == 0).all()
        stats = td.tdes_server_stats(server)
        assert stats["completed"] == n and stats["steps"] > 1
        mixed = _outputs_by_tag(server, done, reqs)
        assert td.tdes_server_stats(server)["pool_bytes_in_use"] == 0
    finally:
        td.tdes_server_destroy(server)
    print(f"[serve] oracle on every block ({stats['steps']} steps)", flush=True)
    for i in range(n):
        _check_oracle(keys, reqs[i], mixed[i])
    print(f"[serve] {len(probe)} requests alone", flush=True)
    server = td.tdes_server_create(dev_table, SERVE_KEYS, 64 << 30, max_inflight=3, max_step_jobs=4096,
                                   max_step_blocks=1 << 24, keep_outputs=True)
    try:
        for i in probe:
            td.tdes_server_submit(server, reqs[i])
            td.tdes_server_wait_idle(server, 120)
            alone = _outputs_by_tag(server, td.tdes_server_poll(server), reqs)
            assert np.array_equal(alone[i], mixed[i]), f"request {i} differs alone and in the mix"
    finally:
        td.tdes_server_destroy(server)
