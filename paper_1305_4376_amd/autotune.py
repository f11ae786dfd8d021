"""Autotuner for the batched kernel's launch shape.

The paper tunes its launch by hand: threads per CUDA block (Table I) and
64-bit blocks per kernel launch (Table II).  Here the batch kernel is
persistent, so the shape to choose is threads per workgroup (waves per
workgroup) and workgroups per compute unit.  `tune_batch` times graph replays
of a real batch for each candidate through the C ABI, applies the fastest to
the context, and records it in a JSON cache keyed by
(GPU architecture, compute units, kernel, log2 of the batch's blocks); `apply_cached`
applies a recorded shape without timing anything.
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


def apply_cached(ctx: int, blocks: int, kernel: str = "batch", path: str = CACHE) -> tuple[int, int] | None:
    entry = load_cache(path).get(_device_key(kernel, blocks))
    if not entry:
        return None
    td.tdes_ctx_set_tuning(ctx, entry["threads"], entry["groups_per_cu"])
    return entry["threads"], entry["groups_per_cu"]


def tune_batch(ctx: int, jobs, dev_sched_table, n_scheds: int, dev_base, reps: int = 5,
               path: str | None = CACHE) -> dict:
    """Time every candidate shape on this batch (graph replays), apply and record the fastest."""
    import torch
    td.tdes_ecb_batch(ctx, jobs, dev_sched_table, n_scheds, dev_base, 0)
    torch.cuda.synchronize()
    timings = []
    for threads in THREADS:
        for gpc in GROUPS_PER_CU:
            td.tdes_ctx_set_tuning(ctx, threads, gpc)
            td.tdes_ecb_batch_replay(ctx, 0)  # captures the graph for this shape
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                td.tdes_ecb_batch_replay(ctx, 0)
            torch.cuda.synchronize()
            timings.append(((time.perf_counter() - t0) / reps, threads, gpc))
    timings.sort()
    best_t, threads, gpc = timings[0]
    td.tdes_ctx_set_tuning(ctx, threads, gpc)
    blocks = int(td.tdes_ctx_get_info(ctx)["blocks"])
    result = {"threads": threads, "groups_per_cu": gpc, "seconds": best_t,
              "candidates": [[round(t * 1e3, 4), th, g] for t, th, g in timings]}
    if path:
        cache = load_cache(path)
        cache[_device_key("batch", blocks)] = {k: v for k, v in result.items() if k != "candidates"}
        save_cache(cache, path)
    return result


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
