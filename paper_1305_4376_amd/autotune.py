"""Autotuner for the batched kernel's launch shape and tiling.

The paper tunes its launch by hand: threads per CUDA block (Table I) and
64-bit blocks per kernel launch (Table II).  Here the batch kernel is
persistent, and four parameters shape a launch: threads per workgroup (waves
per workgroup), workgroups per compute unit, the wave/lane cut-over (a
message's last partial tile of at least this many blocks runs as a wave tile
with one key per wave, a shorter one as 32-block lane slots with one key per
lane) and tiles per draw from the work counter.  `tune_batch` times graph
replays of a real batch through the C ABI: every launch shape first, then the
tiling axes at the best shape; it applies the fastest to the context and
records it in a JSON cache keyed by (GPU architecture, compute units, kernel,
log2 of the batch's blocks).  `cached_tuning` looks a recorded tuning up and
`apply_cached` applies it without timing anything.
"""
from __future__ import annotations

import json
import math
import os
import time

import paper_1305_4376_amd as td

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
THREADS = (64, 128, 256)
GROUPS_PER_CU = (1, 2, 3, 4, 6, 8, 12)
WAVE_REMAINDER = (1, 512, 1024, 1536, 1800, 2048)
TILES_PER_DRAW = (1, 2, 4)
FIELDS = ("threads", "groups_per_cu", "wave_remainder", "tiles_per_draw")


def _device_key(kernel: str, blocks: int) -> str:
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "unknown").split(":")[0]
    bucket = int(math.log2(max(1, blocks)))
    return f"{arch}/{props.multi_processor_count}/{kernel}/2^{bucket}"


def load_cache(path: str = CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str = CACHE) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def cached_tuning(blocks: int, kernel: str = "batch", path: str = CACHE) -> tuple[int, int, int, int] | None:
    """The recorded (threads, groups_per_cu, wave_remainder, tiles_per_draw) for batches of about
    `blocks` blocks on this GPU, or None."""
    entry = load_cache(path).get(_device_key(kernel, blocks))
    if not entry:
        return None
    return tuple(int(entry.get(k, 0)) for k in FIELDS)


def apply_cached(ctx: int, blocks: int, kernel: str = "batch", path: str = CACHE) -> tuple[int, int, int, int] | None:
    tuning = cached_tuning(blocks, kernel, path)
    if tuning:
        td.tdes_ctx_set_tuning(ctx, *tuning)
    return tuning


def _time_replays(ctx: int, tuning, reps: int) -> float:
    import torch
    td.tdes_ctx_set_tuning(ctx, *tuning)
    td.tdes_ecb_batch_replay(ctx, 0)  # captures the graph for this shape
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        td.tdes_ecb_batch_replay(ctx, 0)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def tune_batch(ctx: int, jobs, dev_sched_table, n_scheds: int, dev_base, reps: int = 5,
               path: str | None = CACHE) -> dict:
    """Time the candidate tunings on this batch (graph replays), apply and record the fastest.

    Launch shapes first (threads x workgroups per CU, default tiling), then the tiling axes at
    the best shape.  A change of the wave/lane cut-over re-plans the batch, so those candidates
    run tdes_ecb_batch once before their replays."""
    import torch
    default_tiling = (0, 0)
    td.tdes_ecb_batch(ctx, jobs, dev_sched_table, n_scheds, dev_base, 0)
    torch.cuda.synchronize()
    timings = []
    for threads in THREADS:
        for gpc in GROUPS_PER_CU:
            tuning = (threads, gpc) + default_tiling
            timings.append((_time_replays(ctx, tuning, reps), tuning))
    best = min(timings)[1]
    for rem in WAVE_REMAINDER:
        for per_draw in TILES_PER_DRAW:
            tuning = best[:2] + (rem, per_draw)
            td.tdes_ctx_set_tuning(ctx, *tuning)
            td.tdes_ecb_batch(ctx, jobs, dev_sched_table, n_scheds, dev_base, 0)  # plan with this cut-over
            timings.append((_time_replays(ctx, tuning, reps), tuning))
    timings.sort()
    best_t, tuning = timings[0]
    td.tdes_ctx_set_tuning(ctx, *tuning)
    td.tdes_ecb_batch(ctx, jobs, dev_sched_table, n_scheds, dev_base, 0)  # the last plan uses the chosen tuning
    torch.cuda.synchronize()
    info = td.tdes_ctx_get_info(ctx)
    result = {k: info[k] for k in FIELDS}
    result["seconds"] = best_t
    result["candidates"] = [[round(t * 1e3, 4), *tun] for t, tun in timings]
    if path:
        cache = load_cache(path)
        cache[_device_key("batch", int(info["blocks"]))] = {k: v for k, v in result.items() if k != "candidates"}
        save_cache(cache, path)
    return result


def tune_serving(saturated_gbs, shapes, max_step_blocks: int, path: str | None = CACHE) -> dict:
    """Choose a server's batch shape by saturated throughput.

    saturated_gbs(shape) runs a saturating trace on a server whose steps use that shape and returns
    its delivered GB/s (shape None: the library's default).  The fastest is recorded in the cache
    under kernel "serve" for steps of max_step_blocks blocks."""
    results = {sh: saturated_gbs(sh) for sh in shapes}
    shape = max(results, key=results.get)
    entry = {k: v for k, v in zip(FIELDS, shape or (0, 0, 0, 0))}
    entry["gbs"] = results[shape]
    if path:
        cache = load_cache(path)
        cache[_device_key("serve", max_step_blocks)] = entry
        save_cache(cache, path)
    return {"shape": shape, "results": results}


def cached_serving(max_step_blocks: int, path: str = CACHE) -> tuple[int, int, int, int] | None:
    """The batch shape recorded for a server with steps of max_step_blocks blocks on this GPU, or None
    (also when the recorded best was the library's default)."""
    entry = load_cache(path).get(_device_key("serve", max_step_blocks))
    if not entry:
        return None
    shape = tuple(int(entry.get(k, 0)) for k in FIELDS)
    return shape if shape[0] else None


def main():
    """Tune the batched workload (4096 messages, log-uniform 1..131072 blocks) and write the cache."""
    import argparse

    import numpy as np
    import torch

    from paper_1305_4376_amd import inputs

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--out", default=CACHE)
    ap.add_argument("--messages", type=int, default=4096)
    args = ap.parse_args()
    dev = torch.device("cuda", 0)
    keys = inputs.key_triples(inputs.KEY_SEED_BASE + 4, args.messages)
    host = np.concatenate([td.tdes_expand_key(k[:8].tobytes(), k[8:16].tobytes(), k[16:].tobytes()) for k in keys])
    table = torch.empty(host.size, dtype=torch.uint8, device=dev)
    td.tdes_sched_upload(host, table)
    lengths = inputs.log_uniform_lengths(inputs.DATA_SEED_BASE + 4, args.messages, 131072)
    starts = np.concatenate([[0], np.cumsum(lengths)[:-1]]) * 8
    total = int(lengths.sum()) * 8
    buf = torch.empty(2 * total, dtype=torch.uint8, device=dev)
    td.tdes_fill_splitmix64(buf, total // 8, inputs.DATA_SEED_BASE + 4, 0)
    jobs = np.zeros(args.messages, dtype=td.JOB_DTYPE)
    jobs["in_off"], jobs["out_off"], jobs["n_blocks"] = starts, starts + total, lengths
    jobs["sched_idx"] = np.arange(args.messages)
    ctx = td.tdes_ctx_create()
    try:
        res = tune_batch(ctx, jobs, table, args.messages, buf, path=args.out)
    finally:
        td.tdes_ctx_destroy(ctx)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
