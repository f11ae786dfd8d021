"""GPU parity of the batched path: many messages, each with its own key triple and direction.

Each message must come out exactly as the oracle's ECB over that message alone
(blocks independent, EDE and its reverse: Abstract, Section II.A), whether the
batch runs as one persistent launch (graph or direct) or as one plain launch
per message.  Tolerance: 0 bits.
"""
import numpy as np
import pytest
import torch

import paper_1305_4376_amd as td
from paper_1305_4376_amd import inputs
from tests import _gpu
from tests._gpu import DEV

pytestmark = pytest.mark.gpu

EDGE_LENGTHS = [0, 1, 2, 31, 32, 33, 63, 64, 65, 1799, 1800, 1801, 2047, 2048, 2049, 4095, 4096, 4097, 6000]


def _table(n_keys, seed):
    keys = inputs.key_triples(seed, n_keys)
    host = np.concatenate([td.tdes_expand_key(k[:8].tobytes(), k[8:16].tobytes(), k[16:].tobytes()) for k in keys])
    dev = torch.empty(host.size, dtype=torch.uint8, device=DEV)
    td.tdes_sched_upload(host, dev)
    return keys, dev


def _layout(lengths, seed, in_place_every=0):
    """Jobs over one buffer: all inputs first, then all outputs (or in place)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    starts = np.concatenate([[0], np.cumsum(lengths)[:-1]]) * 8
    total = int(lengths.sum()) * 8
    buf = torch.empty(2 * total + 64, dtype=torch.uint8, device=DEV)
    td.tdes_fill_splitmix64(buf, total // 8, seed, 0)
    jobs = np.zeros(len(lengths), dtype=td.JOB_DTYPE)
    jobs["in_off"] = starts
    jobs["out_off"] = starts + total
    if in_place_every:
        sel = np.arange(len(lengths)) % in_place_every == 0
        jobs["out_off"][sel] = starts[sel]
    jobs["n_blocks"] = lengths
    torch.cuda.synchronize()
    return jobs, buf, total


def _check_jobs(jobs, keys, buf, seed, sample_per_job=None):
    host = buf.cpu().numpy()
    for j, job in enumerate(jobs):
        n = int(job["n_blocks"])
        if n == 0:
            continue
        k = keys[job["sched_idx"]]
        k1, k2, k3 = k[:8].tobytes(), k[8:16].tobytes(), k[16:].tobytes()
        first = int(job["in_off"]) // 8
        if sample_per_job is None or n <= sample_per_job:
            idx = np.arange(n)
        else:
            rng = np.random.default_rng(j)
            idx = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, sample_per_job)]))
        src = inputs.blocks_at(seed, first + idx)
        want = _gpu.oracle_on_blocks((k1, k2, k3), src, decrypt=bool(job["direction"]))
        out = host[int(job["out_off"]):int(job["out_off"]) + 8 * n].reshape(-1, 8)[idx].reshape(-1)
        assert np.array_equal(out, want), f"job {j}: n={n} dir={job['direction']}"


@pytest.mark.parametrize("flags", [0, td.TDES_BATCH_NO_GRAPH, td.TDES_BATCH_PER_MESSAGE])
def test_batch_edge_lengths(flags):
    keys, table = _table(7, 0xB01)
    lengths = EDGE_LENGTHS * 3
    jobs, buf, _ = _layout(lengths, 0xB02, in_place_every=5)
    jobs["sched_idx"] = np.arange(len(lengths)) % 7          # keys shared between messages
    jobs["direction"] = (np.arange(len(lengths)) // 2) % 2    # both directions mixed
    ctx = td.tdes_ctx_create()
    try:
        print(f"[batch] edge lengths flags={flags}", flush=True)
        td.tdes_ecb_batch(ctx, jobs, table, 7, buf, flags)
        torch.cuda.synchronize()
        _check_jobs(jobs, keys, buf, 0xB02)
        if flags != td.TDES_BATCH_PER_MESSAGE:
            info = td.tdes_ctx_get_info(ctx)
            assert info["blocks"] == sum(lengths)
            assert info["lane_tiles"] > 0 and info["wave_tiles"] > 0
    finally:
        td.tdes_ctx_destroy(ctx)


def test_graph_replays_match_eager():
    keys, table = _table(32, 0xB11)
    lengths = inputs.log_uniform_lengths(0xB12, 300, 20000)
    jobs, buf, total = _layout(lengths, 0xB13)
    jobs["sched_idx"] = np.arange(len(lengths)) % 32
    jobs["direction"] = np.arange(len(lengths)) % 2
    ctx = td.tdes_ctx_create()
    try:
        td.tdes_ecb_batch(ctx, jobs, table, 32, buf, td.TDES_BATCH_NO_GRAPH)
        torch.cuda.synchronize()
        eager = buf[total:2 * total].clone()
        _check_jobs(jobs, keys, buf, 0xB13, sample_per_job=64)
        for rep in range(4):
            buf[total:2 * total].zero_()
            torch.cuda.synchronize()
            if rep == 0:
                td.tdes_ecb_batch(ctx, jobs, table, 32, buf, 0)   # plans and captures
            else:
                td.tdes_ecb_batch_replay(ctx, 0)                  # graph replay only
            torch.cuda.synchronize()
            assert torch.equal(buf[total:2 * total], eager), f"replay {rep}"
            # eager work between replays
            scratch = torch.randn(1 << 16, device=DEV)
            float(scratch.sum())
        assert td.tdes_ctx_get_info(ctx)["graph_captures"] == 1
        # A different batch on the same buffers reuses the captured graph.
        jobs2 = jobs[::-1].copy()
        jobs2["direction"] ^= 1
        td.tdes_ecb_batch(ctx, jobs2, table, 32, buf, 0)
        torch.cuda.synchronize()
        assert td.tdes_ctx_get_info(ctx)["graph_captures"] == 1
        _check_jobs(jobs2, keys, buf, 0xB13, sample_per_job=64)
    finally:
        td.tdes_ctx_destroy(ctx)


def test_c4_batch_equals_per_message():
    """The batched workload: 4096 messages of log-uniform length 1..131072 blocks, each under its own
    three-key triple; one persistent launch equals 4096 plain launches, and every block equals the oracle."""
    n_msgs = 4096
    seed = inputs.DATA_SEED_BASE + 4
    keys, table = _table(n_msgs, inputs.KEY_SEED_BASE + 4)
    lengths = inputs.log_uniform_lengths(seed, n_msgs, 131072)
    jobs, buf, total = _layout(lengths, seed)
    jobs["sched_idx"] = np.arange(n_msgs)
    ctx = td.tdes_ctx_create()
    try:
        print("[batch] C4 4096 messages", flush=True)
        td.tdes_ecb_batch(ctx, jobs, table, n_msgs, buf, 0)
        torch.cuda.synchronize()
        batched = buf[total:2 * total].clone()
        buf[total:2 * total].zero_()
        td.tdes_ecb_batch(ctx, jobs, table, n_msgs, buf, td.TDES_BATCH_PER_MESSAGE)
        torch.cuda.synchronize()
        assert torch.equal(buf[total:2 * total], batched)
        _check_jobs(jobs, keys, buf, seed)          # every block of every message
        info = td.tdes_ctx_get_info(ctx)
        assert info["blocks"] == int(lengths.sum())
        assert info["padded_blocks"] < 1.05 * info["blocks"]
    finally:
        td.tdes_ctx_destroy(ctx)


def test_batch_rejects_bad_jobs():
    keys, table = _table(2, 0xB21)
    jobs, buf, total = _layout([100, 200, 300], 0xB22)
    ctx = td.tdes_ctx_create()

    def expect(code, j, n_scheds=2, flags=0):
        with pytest.raises(td.TdesError) as e:
            td.tdes_ecb_batch(ctx, j, table, n_scheds, buf, flags)
        assert e.value.code == code

    try:
        bad = jobs.copy(); bad["direction"][1] = 2
        expect(-7, bad)
        bad = jobs.copy(); bad["sched_idx"][2] = 2
        expect(-4, bad)
        bad = jobs.copy(); bad["in_off"][0] += 4
        expect(-2, bad)
        bad = jobs.copy(); bad["out_off"][1] = bad["out_off"][0] + 8   # two outputs overlap
        expect(-3, bad)
        bad = jobs.copy(); bad["out_off"][1] = bad["in_off"][0]        # writes another job's input
        expect(-3, bad)
        bad = jobs.copy(); bad["out_off"][0] = bad["in_off"][0] + 8    # partial self overlap
        expect(-3, bad)
        expect(-3, bad, flags=td.TDES_BATCH_PER_MESSAGE)
        with pytest.raises(td.TdesError) as e:
            td.tdes_ecb_batch_replay(ctx)
        assert e.value.code == -11                                    # nothing planned yet
        ok = jobs.copy(); ok["out_off"] = ok["in_off"]                  # in place is fine
        td.tdes_ecb_batch(ctx, ok, table, 2, buf, 0)
        torch.cuda.synchronize()
        for bad_shape in ((96, 2), (64, 1, 2049), (64, 1, 0, 17)):
            with pytest.raises(td.TdesError) as e:
                td.tdes_ctx_set_tuning(ctx, *bad_shape)
            assert e.value.code == -7
    finally:
        td.tdes_ctx_destroy(ctx)


@pytest.mark.parametrize("per_draw", [1, 3])
def test_replays_with_more_tiles_than_waves(per_draw):
    """A small grid (one 64-thread workgroup per CU) takes most tiles from the work counter, one or
    three per draw, so each replay relies on the previous launch having left the counter at zero."""
    keys, table = _table(16, 0xB21)
    lengths = inputs.log_uniform_lengths(0xB22, 400, 40000)
    jobs, buf, total = _layout(lengths, 0xB23)
    jobs["sched_idx"] = np.arange(len(lengths)) % 16
    ctx = td.tdes_ctx_create()
    try:
        td.tdes_ctx_set_tuning(ctx, 64, 1, 0, per_draw)
        td.tdes_ecb_batch(ctx, jobs, table, 16, buf, td.TDES_BATCH_NO_GRAPH)
        torch.cuda.synchronize()
        info = td.tdes_ctx_get_info(ctx)
        n_waves = torch.cuda.get_device_properties(0).multi_processor_count
        assert info["tiles"] > 2 * n_waves, (info["tiles"], n_waves)
        eager = buf[total:2 * total].clone()
        _check_jobs(jobs, keys, buf, 0xB23, sample_per_job=32)
        for rep in range(4):
            print(f"[batch] replay {rep} with {info['tiles']} tiles on {n_waves} waves", flush=True)
            buf[total:2 * total].zero_()
            torch.cuda.synchronize()
            if rep == 0:
                td.tdes_ecb_batch(ctx, jobs, table, 16, buf, 0)
            else:
                td.tdes_ecb_batch_replay(ctx, td.TDES_BATCH_NO_GRAPH if rep == 3 else 0)
            torch.cuda.synchronize()
            assert torch.equal(buf[total:2 * total], eager), f"replay {rep}"
    finally:
        td.tdes_ctx_destroy(ctx)


@pytest.mark.parametrize("shape", [(64, 1, 0, 0), (128, 2, 1, 3), (256, 1, 2048, 2), (256, 6, 512, 16),
                                   (192, 3, 1800, 1)])
def test_batch_tuning_shapes(shape):
    """Launch shapes and tilings (threads, workgroups per CU, wave/lane cut-over, tiles per draw):
    every message still matches the oracle."""
    keys, table = _table(5, 0xB31)
    lengths = inputs.log_uniform_lengths(0xB32, 200, 10000)
    jobs, buf, total = _layout(lengths, 0xB33)
    jobs["sched_idx"] = np.arange(len(lengths)) % 5
    ctx = td.tdes_ctx_create()
    try:
        td.tdes_ctx_set_tuning(ctx, *shape)
        td.tdes_ecb_batch(ctx, jobs, table, 5, buf, 0)
        torch.cuda.synchronize()
        info = td.tdes_ctx_get_info(ctx)
        assert (info["threads"], info["groups_per_cu"]) == shape[:2]
        assert info["wave_remainder"] == (shape[2] or 1800) and info["tiles_per_draw"] == (shape[3] or 1)
        _check_jobs(jobs, keys, buf, 0xB33, sample_per_job=48)
        buf[total:2 * total].zero_()
        torch.cuda.synchronize()
        td.tdes_ecb_batch_replay(ctx, 0)  # graph replay under the same tuning
        torch.cuda.synchronize()
        _check_jobs(jobs, keys, buf, 0xB33, sample_per_job=48)
    finally:
        td.tdes_ctx_destroy(ctx)


def test_plan_growth_after_graph_capture():
    """A batch larger than the context's plan buffers reallocates them after a graph was captured;
    the next launch must use a graph captured for the new buffers (the slot array's offset moves
    with the capacity even when the allocator returns the same address)."""
    keys, table = _table(16, 0xB41)
    big = inputs.log_uniform_lengths(0xB42, 3000, 131072)
    jobs_big, buf, _ = _layout(big, 0xB43)
    jobs_big["sched_idx"] = np.arange(big.size) % 16
    small = jobs_big[:3].copy()
    ctx = td.tdes_ctx_create()
    try:
        td.tdes_ecb_batch(ctx, small, table, 16, buf, 0)    # small plan, graph captured
        torch.cuda.synchronize()
        captures = td.tdes_ctx_get_info(ctx)["graph_captures"]
        td.tdes_ecb_batch(ctx, jobs_big, table, 16, buf, 0)  # grows the plan buffers
        torch.cuda.synchronize()
        assert td.tdes_ctx_get_info(ctx)["graph_captures"] == captures + 1
        _check_jobs(jobs_big, keys, buf, 0xB43, sample_per_job=8)
    finally:
        td.tdes_ctx_destroy(ctx)
