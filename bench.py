"""Benchmark: Triple-DES (EDE) ECB on one MI355X.

Timed step (the line's `value`): encrypt one 1 GiB message (2^27 blocks of
seeded random bytes, resident in HBM) under a random three-key triple, then
decrypt the ciphertext -- one launch each, kernel-only as in the paper (inputs
already on the device; transfers excluded).  value = plaintext bytes processed
per second over the timed steps (GB = 1e9 bytes), with the shipped kernel.

The same JSON line also carries
  roofline      the shipped kernel against the 32-bit integer ALU peak;
  variants      GB/s of the table and bitsliced kernels on the same message;
  batched       4096 messages of log-uniform length, each under its own key:
                one persistent graph launch against 4096 plain launches;
  serving       Poisson arrivals of mixed requests at three offered loads:
                delivered GB/s, p50 / p99 latency;
  cpu_baseline  the CPU oracle on this host's cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "3DES-ECB GB/s on 1 MI355X (plain vs batched); serving p50/p99 latency"
N_BLOCKS = 1 << 27
DATA_SEED = 0x3DE50000 + 1
KEY_SEED = 0x4B455900 + 1

# MI355X integer ALU peak: 256 CUs x 128 32-bit lane-operations per clock x 2.4 GHz
# (the lane rate behind the published 157.3 TFLOP/s FP32 vector figure, which counts an FMA as 2).
ALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
PKG = os.path.join(ROOT, "paper_1305_4376_amd")
KERNEL_SOURCES = ["csrc/bitslice_core.h", "csrc/k_bitslice.hip", "csrc/sbox_circuits.inc", "csrc/rounds_asm.inc"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "tdes_bitslice_kernel_1GiB_traffic.md")


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--cpu-sample-blocks", type=int, default=1 << 23)
    ap.add_argument("--cpu-one-thread-blocks", type=int, default=1 << 20)
    ap.add_argument("--serve-seconds", type=float, default=1.0, help="trace length per offered load")
    ap.add_argument("--no-host-path", action="store_true")
    ap.add_argument("--no-paper-ablation", action="store_true",
                    help="skip the paper's launch scheme: a 512 MiB message cut into launches of "
                         "128 .. 2^26 blocks (the analogue of Table II)")
    ap.add_argument("--plain-only", action="store_true",
                    help="only the timed encrypt + decrypt steps of the 1 GiB message (for profiling them alone)")
    ap.add_argument("--no-c1", action="store_true", help="skip the 1 MiB message row")
    ap.add_argument("--c1-only", action="store_true", help="only the 1 MiB message row (for profiling it alone)")
    ap.add_argument("--tuning-cache", default=None,
                    help="also record the batch and serving tunings chosen here in this autotuner cache file")
    ap.add_argument("--no-c3", action="store_true", help="skip the keying x size x direction sweep")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 1 GiB elementwise XOR kernel (1 GiB read + 1 GiB written), the known-size "
                         "reference that scales the profiler's FETCH_SIZE / WRITE_SIZE counters")
    return ap.parse_args()


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(PKG, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the shipped kernel from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m_hash = re.search(r"kernel source hash:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"HBM bytes per launch:\s*([0-9.e+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_hash():
        return None
    return float(m_bytes.group(1))


COUNTERS_FILE = os.path.join(ROOT, "profiles", "tdes_ecb_kernels_1GiB_counters.md")


def measured_issued_ops():
    """VALU lane-operations per block that the shipped kernel issues, from the committed SQ counter
    summary, if it was taken on the current kernel source; else None."""
    try:
        text = open(COUNTERS_FILE).read()
    except OSError:
        return None
    m_hash = re.search(r"kernel source hash:\s*([0-9a-f]+)", text)
    m_ops = re.search(r"issued VALU lane-ops per block:\s*([0-9.]+)", text)
    if not m_hash or not m_ops or m_hash.group(1) != kernel_hash():
        return None
    return float(m_ops.group(1))


def circuit_gates() -> int:
    """Gates in the shipped S-box circuits (sum over the eight boxes)."""
    text = open(os.path.join(PKG, "gen", "sbox_circuits.txt")).read()
    return sum(int(g) for g in re.findall(r"^gates (\d+)", text, flags=re.M))


def time_plain(td, torch, sched, src, ct, pt, variant, steps, warmup):
    """Wall time of `steps` encrypt+decrypt steps and per-launch HIP-event durations (same stream)."""
    for _ in range(warmup):
        td.tdes_ecb_run(sched, src, ct, N_BLOCKS, td.TDES_ENCRYPT, variant)
        td.tdes_ecb_run(sched, ct, pt, N_BLOCKS, td.TDES_DECRYPT, variant)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(2 * steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[2 * i][0].record()
        td.tdes_ecb_run(sched, src, ct, N_BLOCKS, td.TDES_ENCRYPT, variant)
        ev[2 * i][1].record()
        ev[2 * i + 1][0].record()
        td.tdes_ecb_run(sched, ct, pt, N_BLOCKS, td.TDES_DECRYPT, variant)
        ev[2 * i + 1][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [a.elapsed_time(b) for a, b in ev]


def key_table(td, torch, inputs, seed, count, dev):
    keys = inputs.key_triples(seed, count)
    import numpy as np
    host = np.empty(count * td.TDES_SCHED_BYTES, dtype=np.uint8)
    for i in range(count):
        k = keys[i]
        host[i * td.TDES_SCHED_BYTES:(i + 1) * td.TDES_SCHED_BYTES] = td.tdes_expand_key(k[:8].tobytes(), k[8:16].tobytes(), k[16:].tobytes())
    table = torch.empty(host.size, dtype=torch.uint8, device=dev)
    td.tdes_sched_upload(host, table)
    return table


def bench_batched(td, torch, inputs, dev, reps=10, cache=None):
    """C4: 4096 messages, log-uniform 1..131072 blocks, own three-key triple each, encrypt."""
    import numpy as np
    n_msgs = 4096
    seed = inputs.DATA_SEED_BASE + 4
    table = key_table(td, torch, inputs, inputs.KEY_SEED_BASE + 4, n_msgs, dev)
    lengths = inputs.log_uniform_lengths(seed, n_msgs, 131072)
    starts = np.concatenate([[0], np.cumsum(lengths)[:-1]]) * 8
    total = int(lengths.sum()) * 8
    buf = torch.empty(2 * total, dtype=torch.uint8, device=dev)
    td.tdes_fill_splitmix64(buf, total // 8, seed, 0)
    jobs = np.zeros(n_msgs, dtype=td.JOB_DTYPE)
    jobs["in_off"], jobs["out_off"], jobs["n_blocks"] = starts, starts + total, lengths
    jobs["sched_idx"] = np.arange(n_msgs)
    from paper_1305_4376_amd import autotune
    ctx = td.tdes_ctx_create()
    try:
        tuned = autotune.tune_batch(ctx, jobs, table, n_msgs, buf, reps=3, path=cache)

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps
        t_plan = timed(lambda: td.tdes_ecb_batch(ctx, jobs, table, n_msgs, buf, 0))
        t_replay = timed(lambda: td.tdes_ecb_batch_replay(ctx, 0))
        t_direct = timed(lambda: td.tdes_ecb_batch_replay(ctx, td.TDES_BATCH_NO_GRAPH))
        out_batched = buf[total:].clone()
        t_plain = timed(lambda: td.tdes_ecb_batch(ctx, jobs, table, n_msgs, buf, td.TDES_BATCH_PER_MESSAGE))
        same = bool(torch.equal(buf[total:], out_batched))
        info = td.tdes_ctx_get_info(ctx)
    finally:
        td.tdes_ctx_destroy(ctx)
    gbs = lambda t: round(total / t / 1e9, 3)
    return {
        "workload": "4096 messages, lengths log-uniform 1..131072 blocks, own 3-key triple each, encrypt",
        "bytes": total,
        "graph_replay_gbs": gbs(t_replay), "graph_replay_ms": round(t_replay * 1e3, 4),
        "direct_launch_gbs": gbs(t_direct),
        "plan_upload_launch_gbs": gbs(t_plan),
        "per_message_plain_gbs": gbs(t_plain), "per_message_plain_ms": round(t_plain * 1e3, 4),
        "speedup_vs_per_message": round(t_plain / t_replay, 2),
        "identical_to_per_message": same,
        "tiles": info["tiles"], "lane_tiles": info["lane_tiles"],
        "padding_frac": round(info["padded_blocks"] / info["blocks"] - 1, 4),
        "tuning": {k: info[k] for k in ("threads", "groups_per_cu", "wave_remainder", "tiles_per_draw")},
        "autotune_best_ms": {"x".join(str(v) for v in c[1:]): c[0] for c in tuned["candidates"][:6]},
        "autotune_candidates": len(tuned["candidates"]),
    }, total / t_replay, tuple(info[k] for k in ("threads", "groups_per_cu", "wave_remainder", "tiles_per_draw"))


def bench_serving(td, torch, inputs, dev, batch_capacity_bps, seconds, tuning=None, cache=None, step_blocks=1 << 24,
                  backlog_step_blocks=1 << 25, in_flight=3):
    """C5: Poisson arrivals, sizes log-uniform 512 B .. 16 MiB, 50/50 directions, 65536 resident triples,
    64 GiB admission budget.  The batch shape of the server's steps is chosen by its saturated
    throughput (every request of a trace arriving at once).  Offered loads: 0.5 / 0.8 / 0.95 of the batched workload's capacity (graph
    replay), and the same fractions of the server's own saturated throughput."""
    import numpy as np
    n_keys = 65536
    table = key_table(td, torch, inputs, inputs.KEY_SEED_BASE + 5, n_keys, dev)
    mean_bytes = 8 * (2 ** 21 - 64) / np.log(2 ** 21 / 64)  # mean of the log-uniform size law

    def trace(seed, n, lam):
        rng = np.random.default_rng(seed)
        u = rng.random(n)
        reqs = np.zeros(n, dtype=td.REQUEST_DTYPE)
        reqs["n_blocks"] = np.floor(np.exp(np.log(64) + u * (np.log(2 ** 21) - np.log(64)))).astype(np.int64)
        reqs["key_id"] = rng.integers(0, n_keys, n)
        reqs["direction"] = rng.integers(0, 2, n)
        reqs["seed"] = (0x5E000000 + (seed & 0xFF) * 10000000) + np.arange(n)
        arrival = np.cumsum(rng.exponential(1.0 / lam, n)) if lam else np.zeros(n)
        return reqs, arrival

    def run(reqs, arrival, shape=None):
        server = td.tdes_server_create(table, n_keys, 64 << 30, max_inflight=in_flight, max_step_jobs=4096,
                                       max_step_blocks=step_blocks, tuning=shape,
                                       backlog_step_blocks=backlog_step_blocks)
        try:
            # Warm-up: the first 5% of the trace (graph captures, plan buffers, first allocations), not measured.
            n_warm = max(200, len(reqs) // 20)
            td.tdes_server_run_trace(server, reqs[:n_warm], arrival[:n_warm] - arrival[0])
            td.tdes_server_wait_idle(server, 60)
            done = td.tdes_server_run_trace(server, reqs, arrival)
            stats = td.tdes_server_stats(server)
        finally:
            td.tdes_server_destroy(server)
        ok = done["status"] == 0
        lat = (done["t_complete"] - done["t_arrival"])[ok]
        span = done["t_complete"].max() - done["t_arrival"].min()
        wait = (done["t_admit"] - done["t_arrival"])[ok]
        half = len(lat) // 2
        return {"requests": len(reqs), "delivered_gbs": round(float(reqs["n_blocks"][ok].sum() * 8) / span / 1e9, 2),
                "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                # queue growth: admission wait in the second half of the trace against the first
                "admit_wait_ms_first_half": round(float(np.mean(wait[:half])) * 1e3, 3),
                "admit_wait_ms_second_half": round(float(np.mean(wait[half:])) * 1e3, 3),
                "failed": int((~ok).sum()), "steps": stats["steps"],
                "peak_pool_gib": round(stats["peak_pool_bytes"] / 2 ** 30, 3)}

    # Saturation: 100000 requests (about 157 GB of payload, long enough that filling and draining the
    # step pipeline weigh little) all arriving at t = 0, for each batch shape of the server's steps
    # (the library's default and the one tuned on the batched workload); the fastest is kept for the
    # loads.
    from paper_1305_4376_amd import autotune
    sat_trace = trace(0x5E50, 100000, 0.0)
    candidates = {}

    def saturated(sh):
        candidates[sh] = run(*sat_trace, shape=sh)
        return candidates[sh]["delivered_gbs"]
    shape = autotune.tune_serving(saturated, [None] + ([tuple(tuning)] if tuning else []), step_blocks,
                                  path=cache)["shape"]
    sat = candidates[shape]
    capacity_bps = sat["delivered_gbs"] * 1e9
    by_batch, by_server = [], []
    for rows, base_bps, tag in ((by_batch, batch_capacity_bps, 0), (by_server, capacity_bps, 8)):
        for li, load in enumerate((0.5, 0.8, 0.95)):
            lam = load * base_bps / mean_bytes
            n = int(max(2000, min(400000, lam * seconds)))
            r = run(*trace(0x5E5E + tag + li, n, lam), shape=shape)
            rows.append({"load": load, "offered_gbs": round(lam * mean_bytes / 1e9, 2), **r})
    return {"workload": "Poisson arrivals, 512 B..16 MiB log-uniform, 50/50 encrypt/decrypt, 65536 resident "
                        "3-key triples, 64 GiB budget, payloads generated on the device at admission; latency = "
                        "host-observed completion - scheduled arrival; each trace after a warm-up of 5% of it",
            "steps": {"in_flight": in_flight, "max_step_blocks": step_blocks, "backlog_step_blocks": backlog_step_blocks},
            "tuning": list(shape) if shape else "default",
            "saturated_gbs_by_shape": {("x".join(map(str, sh)) if sh else "default"): r["delivered_gbs"]
                                       for sh, r in candidates.items()},
            "capacity_gbs": round(capacity_bps / 1e9, 2), "batch_capacity_gbs": round(batch_capacity_bps / 1e9, 2),
            "saturation": sat,
            "loads": by_batch, "loads_basis": "fractions of the batched workload's capacity (graph replay)",
            "loads_vs_server": by_server, "loads_vs_server_basis": "fractions of the server's saturated throughput"}


def bench_host_path(td, torch, sched, dev, reps=3):
    """A 1 GiB message in pinned host memory: copies in, kernel and copies out overlapped in 32 MiB
    chunks (the best of a 16..256 MiB sweep).  PCIe-inclusive; reported beside the kernel-only value,
    never as it."""
    n = N_BLOCKS
    host = torch.empty(n * 8, dtype=torch.uint8).pin_memory()
    dev_msg = torch.empty(n * 8, dtype=torch.uint8, device=dev)
    td.tdes_fill_splitmix64(dev_msg, n, DATA_SEED, 0)
    host.copy_(dev_msg)
    out = torch.empty_like(host).pin_memory()
    del dev_msg
    td.tdes_ecb_host(sched, host, out, n, td.TDES_ENCRYPT, chunk_blocks=1 << 22)
    t0 = time.perf_counter()
    for _ in range(reps):
        td.tdes_ecb_host(sched, host, out, n, td.TDES_ENCRYPT, chunk_blocks=1 << 22)
    dt = (time.perf_counter() - t0) / reps
    return {"workload": "the 1 GiB message in pinned host memory, encrypt, 32 MiB chunks through 3 device "
                        "slots (H2D, kernel, D2H on separate streams)", "gbs": round(n * 8 / dt / 1e9, 3),
            "ms": round(dt * 1e3, 3)}


def bench_sizes(td, torch, sched, dev):
    """Kernel time of one launch against message size, both variants (HIP events, mean of repeats):
    where the bitsliced kernel's fixed per-tile latency stops mattering."""
    out = []
    buf = torch.empty((1 << 24) * 8, dtype=torch.uint8, device=dev)
    td.tdes_fill_splitmix64(buf, 1 << 24, DATA_SEED, 0)
    dst = torch.empty_like(buf)
    for log_n in range(8, 25, 2):
        n = 1 << log_n
        row = {"blocks": n}
        for name, v in (("table", td.TDES_VARIANT_TABLE), ("bitslice", td.TDES_VARIANT_BITSLICE)):
            reps = 20
            for _ in range(3):
                td.tdes_ecb_run(sched, buf, dst, n, td.TDES_ENCRYPT, v)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            for a, b in ev:
                a.record()
                td.tdes_ecb_run(sched, buf, dst, n, td.TDES_ENCRYPT, v)
                b.record()
            torch.cuda.synchronize()
            us = sum(a.elapsed_time(b) for a, b in ev) / reps * 1e3
            row[name + "_us"] = round(us, 2)
            row[name + "_gbs"] = round(n * 8 / us / 1e3, 3)
        out.append(row)
    return out


def bench_paper_scheme(td, torch, sched, dev):
    """The paper's host loop (Listing 1.1): one launch per chunk of a 512 MiB message, swept over the
    chunk size as in Table II, issued by the library (tdes_ecb_chunked, the kernel chosen by chunk size).  Sizes that need more than
    16384 launches are timed on their first 16384 chunks and scaled to the message (extrapolated)."""
    total = 1 << 26  # 512 MiB
    msg = torch.empty(total * 8, dtype=torch.uint8, device=dev)
    td.tdes_fill_splitmix64(msg, total, DATA_SEED, 0)
    rows = []
    for chunk in (128, 512, 2048, 8192, 32768, 131072, 524288, 1 << 21, 1 << 23, 1 << 26):
        launches = total // chunk
        timed = min(launches, 16384)
        td.tdes_ecb_chunked(sched, msg, msg, chunk, min(timed, 64) * chunk)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        td.tdes_ecb_chunked(sched, msg, msg, chunk, timed * chunk)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) * launches / timed
        rows.append({"blocks_per_launch": chunk, "launches": launches, "seconds": round(dt, 5),
                     "gbs": round(total * 8 / dt / 1e9, 3), "extrapolated": timed < launches})
    return {"workload": "512 MiB message, in place, one launch per chunk (Listing 1.1's loop, issued by "
                        "tdes_ecb_chunked; table kernel below 2^20 blocks per chunk, bitsliced from there)",
            "rows": rows}


_SLEEP_S_PER_CYCLE = []


def _hold_stream(torch, seconds):
    """Keeps torch's current stream busy for about `seconds` (a spin kernel), so that what the host
    enqueues meanwhile starts on the GPU back to back, not when the host gets to it."""
    if not _SLEEP_S_PER_CYCLE:
        torch.cuda._sleep(1 << 20)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        torch.cuda._sleep(1 << 22)
        b.record()
        torch.cuda.synchronize()
        _SLEEP_S_PER_CYCLE.append(max(a.elapsed_time(b) / 1e3 / (1 << 22), 1e-12))
    torch.cuda._sleep(min(int(seconds / _SLEEP_S_PER_CYCLE[0]), 1 << 40))


def time_launches(torch, fn, reps, warmup=3, hold=True):
    """Mean duration of `fn` (one or more launches on torch's current stream) from HIP events recorded
    on that stream around each call, in seconds.  hold: the stream is held by a spin kernel while the
    calls are enqueued, so each pair of events brackets the launch as the GPU runs it; without it, a
    short launch's pair also brackets the host's time to issue it (the GPU reaches the first event
    before the host has launched the kernel)."""
    for _ in range(warmup):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    if hold:
        _hold_stream(torch, 1e-3 + 40e-6 * reps)
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in ev) / reps / 1e3


def bench_c1(td, torch, inputs, dev, ops_per_block, reps=200):
    """C1: one 1 MiB message (2^17 blocks), one 3-key triple, encrypt then decrypt the ciphertext on one
    stream, in and out distinct.  Kernel-only: HIP events around each launch, enqueued while the stream
    is held (encrypt_us_with_issue: the same without holding it, which adds the host's time to issue
    a launch); also the back-to-back rate of whole steps (wall time over many steps), which includes
    the launch gaps."""
    n = 1 << 17
    keys = inputs.key_triple(inputs.KEY_SEED_BASE + 0)
    sched = torch.empty(td.TDES_SCHED_BYTES, dtype=torch.uint8, device=dev)
    td.tdes_sched_upload(td.tdes_expand_key(*keys), sched)
    src = torch.empty(n * 8, dtype=torch.uint8, device=dev)
    td.tdes_fill_splitmix64(src, n, inputs.DATA_SEED_BASE + 0, 0)
    ct, pt = torch.empty_like(src), torch.empty_like(src)
    out = {"workload": "1 MiB message (2^17 blocks), 3-key triple, encrypt then decrypt, kernel-only per launch"}
    for name, v in (("auto", td.TDES_VARIANT_AUTO), ("table", td.TDES_VARIANT_TABLE),
                    ("bitslice", td.TDES_VARIANT_BITSLICE)):
        enc = time_launches(torch, lambda: td.tdes_ecb_run(sched, src, ct, n, td.TDES_ENCRYPT, v), reps)
        dec = time_launches(torch, lambda: td.tdes_ecb_run(sched, ct, pt, n, td.TDES_DECRYPT, v), reps)
        enc_issue = time_launches(torch, lambda: td.tdes_ecb_run(sched, src, ct, n, td.TDES_ENCRYPT, v), reps,
                                  hold=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            td.tdes_ecb_run(sched, src, ct, n, td.TDES_ENCRYPT, v)
            td.tdes_ecb_run(sched, ct, pt, n, td.TDES_DECRYPT, v)
        torch.cuda.synchronize()
        step = (time.perf_counter() - t0) / reps
        kernel_s = (enc + dec) / 2
        out[name] = {"encrypt_us": round(enc * 1e6, 2), "decrypt_us": round(dec * 1e6, 2),
                     "encrypt_us_with_issue": round(enc_issue * 1e6, 2),
                     "gbs": round(n * 8 / kernel_s / 1e9, 3),
                     "step_us_back_to_back": round(step * 1e6, 2),
                     "alu_frac": round(ops_per_block * n / kernel_s / 1e12 / ALU_PEAK_TOPS, 4),
                     "roundtrip_ok": bool(torch.equal(pt, src))}
    return out


def bench_c3(td, torch, inputs, dev):
    """C3: {3, 2, 1}-key triples x {2^13, 2^19, 2^25, 2^29} blocks (64 KiB .. 4 GiB) x {encrypt, decrypt},
    the shipped automatic variant, one launch each, kernel-only (HIP events, mean of repeats)."""
    rows = []
    top = 1 << 29
    src = torch.empty(top * 8, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    for keying in (3, 2, 1):
        keys = inputs.key_triple(inputs.KEY_SEED_BASE + 3 + keying, keying)
        sched = torch.empty(td.TDES_SCHED_BYTES, dtype=torch.uint8, device=dev)
        td.tdes_sched_upload(td.tdes_expand_key(*keys), sched)
        td.tdes_fill_splitmix64(src, top, inputs.DATA_SEED_BASE + 3 + 16 * keying, 0)
        for log_n in (13, 19, 25, 29):
            n = 1 << log_n
            for d in (td.TDES_ENCRYPT, td.TDES_DECRYPT):
                t = time_launches(torch, lambda: td.tdes_ecb_run(sched, src, dst, n, d, td.TDES_VARIANT_AUTO),
                                  reps=5 if log_n >= 29 else 20)
                rows.append({"keying": keying, "blocks": n, "direction": "decrypt" if d else "encrypt",
                             "us": round(t * 1e6, 2), "gbs": round(n * 8 / t / 1e9, 3)})
    return {"workload": "keying x size x direction, the automatic variant (table below 2^20 blocks, bitsliced "
                        "from there), one launch each, kernel-only", "rows": rows}


def bench_paper_threads(td, torch, dev):
    """The analogue of Table I: threads per workgroup of the plain kernels under the paper's launch
    scheme (tdes_ecb_chunked, 131072 blocks per launch) over a 512 MiB message, in place."""
    total = 1 << 26
    msg = torch.empty(total * 8, dtype=torch.uint8, device=dev)
    td.tdes_fill_splitmix64(msg, total, DATA_SEED, 0)
    sched = torch.empty(td.TDES_SCHED_BYTES, dtype=torch.uint8, device=dev)
    from paper_1305_4376_amd import inputs
    td.tdes_sched_upload(td.tdes_expand_key(*inputs.key_triple(KEY_SEED)), sched)
    rows = []
    for name, v in (("table", td.TDES_VARIANT_TABLE), ("bitslice", td.TDES_VARIANT_BITSLICE)):
        for threads in (64, 128, 256, 512, 1024):
            td.tdes_ecb_chunked(sched, msg, msg, 131072, 64 * 131072, variant=v, threads=threads)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            td.tdes_ecb_chunked(sched, msg, msg, 131072, total, variant=v, threads=threads)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            rows.append({"kernel": name, "threads_per_workgroup": threads, "seconds": round(dt, 5),
                         "gbs": round(total * 8 / dt / 1e9, 3)})
    return {"workload": "512 MiB message, in place, 512 launches of 131072 blocks (the paper's chunk), threads "
                        "per workgroup swept for each kernel", "rows": rows}


def openssl_ecb_rate(keys, data):
    """Context beside the oracle: OpenSSL's EVP_des_ede3_ecb on one host thread over the same sample
    (GB/s), or None where libcrypto cannot be loaded."""
    import ctypes
    import ctypes.util
    lib = None
    for name in ("libcrypto.so.3", ctypes.util.find_library("crypto")):
        if name:
            try:
                lib = ctypes.CDLL(name)
                break
            except OSError:
                continue
    if lib is None:
        return None
    vp, ip = ctypes.c_void_p, ctypes.c_int
    lib.EVP_CIPHER_CTX_new.restype = vp
    lib.EVP_CIPHER_CTX_free.argtypes = [vp]
    lib.EVP_des_ede3_ecb.restype = vp
    lib.EVP_CipherInit_ex.argtypes = [vp, vp, vp, ctypes.c_char_p, ctypes.c_char_p, ip]
    lib.EVP_CIPHER_CTX_set_padding.argtypes = [vp, ip]
    lib.EVP_CipherUpdate.argtypes = [vp, vp, ctypes.POINTER(ip), vp, ip]
    lib.OpenSSL_version.restype = ctypes.c_char_p
    lib.OpenSSL_version.argtypes = [ip]
    out = bytearray(data.size + 16)
    buf = (ctypes.c_uint8 * len(out)).from_buffer(out)
    ctx = lib.EVP_CIPHER_CTX_new()
    try:
        if lib.EVP_CipherInit_ex(ctx, lib.EVP_des_ede3_ecb(), None, b"".join(keys), None, 1) != 1:
            return None
        lib.EVP_CIPHER_CTX_set_padding(ctx, 0)
        n = ctypes.c_int(0)
        t0 = time.perf_counter()
        ok = lib.EVP_CipherUpdate(ctx, ctypes.addressof(buf), ctypes.byref(n), data.ctypes.data, int(data.size))
        dt = time.perf_counter() - t0
    finally:
        lib.EVP_CIPHER_CTX_free(ctx)
    if ok != 1 or n.value != data.size:
        return None
    return {"value": round(data.size / dt / 1e9, 6), "unit": "GB/s", "threads": 1,
            "library": lib.OpenSSL_version(0).decode(), "sample": f"the same {data.size >> 20} MiB: {dt:.1f} s"}


def cpu_baseline(sample_blocks, one_thread_blocks):
    """The oracle on the host's cores (every core this process may use), and on one thread."""
    import oracle
    from paper_1305_4376_amd import inputs
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    keys = inputs.key_triple(KEY_SEED)
    data = inputs.message(DATA_SEED, sample_blocks)
    t0 = time.perf_counter()
    oracle.tdes_ecb(*keys, data, decrypt=False, threads=cores)
    dt = time.perf_counter() - t0
    one = data[: one_thread_blocks * 8]
    t0 = time.perf_counter()
    oracle.tdes_ecb(*keys, one, decrypt=False, threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": round(data.size / dt / 1e9, 6), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"encrypt the first {sample_blocks} blocks ({data.size >> 20} MiB) of the benchmark message "
                      f"with its key triple on {cores} threads: {dt:.1f} s",
            "one_thread": {"value": round(one.size / dt1 / 1e9, 6), "unit": "GB/s",
                           "sample": f"the first {one_thread_blocks} blocks on 1 thread: {dt1:.1f} s"},
            "openssl_context": openssl_ecb_rate(keys, data)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for {args.gpus}): every configuration here runs on a single "
              "MI355X; ECB shards need no communication, so a G-GPU job runs G independent shards.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1305_4376_amd as td
    from paper_1305_4376_amd import inputs

    td.load_library()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    keys = inputs.key_triple(KEY_SEED)
    sched = torch.empty(td.TDES_SCHED_BYTES, dtype=torch.uint8, device=dev)
    td.tdes_sched_upload(td.tdes_expand_key(*keys), sched)
    src = torch.empty(N_BLOCKS * 8, dtype=torch.uint8, device=dev)
    td.tdes_fill_splitmix64(src, N_BLOCKS, DATA_SEED, 0)
    ct, pt = torch.empty_like(src), torch.empty_like(src)
    torch.cuda.synchronize()

    if args.calib_copy:
        torch.bitwise_xor(src, 0x5A, out=ct)
        torch.cuda.synchronize()

    if args.c1_only:
        gates = circuit_gates()
        print(json.dumps({"c1": bench_c1(td, torch, inputs, dev, 12 * gates / 8 + 120)}), flush=True)
        return
    bytes_per_step = 2 * N_BLOCKS * 8
    # Kernel-only rate of each variant: plaintext bytes over the average launch (HIP events).
    variants = {}
    for name, v in (("table", td.TDES_VARIANT_TABLE), ("bitslice", td.TDES_VARIANT_BITSLICE)):
        if args.plain_only:
            break
        _, ms = time_plain(td, torch, sched, src, ct, pt, v, max(4, args.steps // 4), 2)
        variants[name] = round(N_BLOCKS * 8 / (sum(ms) / len(ms) / 1e3) / 1e9, 3)
    # CTR and CBC decryption on the same core: kernel-only rate over the same message.
    modes = {}
    iv = bytes.fromhex("0123456789abcdef")
    for name, fn in (("ctr", td.tdes_ctr_crypt), ("cbc_decrypt", td.tdes_cbc_decrypt)):
        if args.plain_only:
            break
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(6)]
        for i, (a, b) in enumerate([(None, None)] * 2 + ev):
            if a is not None:
                a.record()
            fn(sched, iv, src, ct, N_BLOCKS)
            if b is not None:
                b.record()
        torch.cuda.synchronize()
        ms = sum(a.elapsed_time(b) for a, b in ev) / len(ev)
        modes[name] = {"gbs": round(N_BLOCKS * 8 / (ms / 1e3) / 1e9, 3), "kernel_ms": round(ms, 4)}
    # The timed run: the shipped default (TDES_VARIANT_AUTO: the bitsliced kernel at this size).
    wall, launch_ms = time_plain(td, torch, sched, src, ct, pt, td.TDES_VARIANT_AUTO, args.steps, args.warmup)
    roundtrip_ok = bool(torch.equal(pt, src))
    value = bytes_per_step * args.steps / wall / 1e9
    avg_launch_s = sum(launch_ms) / len(launch_ms) / 1e3

    gates = circuit_gates()
    ops_per_block = 12 * gates / 8 + 120  # 48 rounds x (48 key XORs + gates + 32 XORs into L) / 32 blocks
    achieved = ops_per_block * N_BLOCKS / avg_launch_s / 1e12
    traffic = measured_traffic()
    issued = measured_issued_ops()
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "3DES-EDE ECB, one 1 GiB message (2^27 blocks of SplitMix64 bytes), one 3-key "
                               "triple, encrypt then decrypt per step, one launch each, HBM-resident",
                   "n_blocks": N_BLOCKS, "keying": 3, "kernel": "bitslice"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 3),
                     "unit": "Tops/s", "frac": round(achieved / ALU_PEAK_TOPS, 4),
                     "traffic": traffic,
                     "ops_per_block": ops_per_block, "kernel_ms": round(avg_launch_s * 1e3, 4),
                     "hbm_frac": round(16 * N_BLOCKS / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4),
                     "issued_ops_per_block": issued,
                     "valu_frac": None if issued is None else
                     round(issued * N_BLOCKS / avg_launch_s / 1e12 / ALU_PEAK_TOPS, 4),
                     "kernel_hash": kernel_hash()},
        "variants": variants,
        "modes": modes,
        "roundtrip_ok": roundtrip_ok,
    }
    del ct, pt
    torch.cuda.empty_cache()
    if args.plain_only:
        print(json.dumps(line), flush=True)
        return
    if not args.no_c1:
        line["c1"] = bench_c1(td, torch, inputs, dev, ops_per_block)
    if not args.no_c3:
        del src
        torch.cuda.empty_cache()
        line["c3"] = bench_c3(td, torch, inputs, dev)
        torch.cuda.empty_cache()
    if not args.no_host_path:
        line["host_path"] = bench_host_path(td, torch, sched, dev)
    if not args.no_paper_ablation:
        line["sizes"] = bench_sizes(td, torch, sched, dev)
        line["paper_scheme"] = bench_paper_scheme(td, torch, sched, dev)
        line["paper_threads"] = bench_paper_threads(td, torch, dev)
        torch.cuda.empty_cache()
    capacity, tuning = value * 1e9, None
    if not args.no_batched:
        line["batched"], capacity, tuning = bench_batched(td, torch, inputs, dev, cache=args.tuning_cache)
        torch.cuda.empty_cache()
    if not args.no_serving:
        line["serving"] = bench_serving(td, torch, inputs, dev, capacity, args.serve_seconds, tuning,
                                        cache=args.tuning_cache)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample_blocks, args.cpu_one_thread_blocks)
    # The paper's own figures (Table IV, seconds for a workload it sizes at 512 MB only in
    # Section III; rates derived for 512 MiB): context, not a target.
    line["paper_context"] = {"unit": "MB/s", "tesla_c2050": 26.3, "gts_250": 14.2,
                             "cpu_4x_xeon_e7_4860_80_threads": 7.72, "cpu_i7_950_8_threads": 1.52}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
