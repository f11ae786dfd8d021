"""Benchmark: Triple-DES (EDE) ECB throughput on one MI355X.

One step = encrypt one 1 GiB message (2^27 blocks of seeded random bytes,
HBM-resident) under a random three-key triple, then decrypt the ciphertext:
one launch each, as in the paper's kernel-only timing (inputs already on the
device; transfers excluded).  value = plaintext bytes processed per second
(GB = 1e9 bytes) over the timed steps.

Also reported on the same JSON line:
  roofline      the dominant kernel against the integer-ALU roofline
  cpu_baseline  the CPU oracle timed on this host's cores on a bounded sample
  variants      GB/s of each kernel variant on the same message
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "3DES-ECB GB/s on 1 MI355X (plain vs batched); serving p50/p99 latency"
N_BLOCKS = 1 << 27
DATA_SEED = 0x3DE50000 + 1
KEY_SEED = 0x4B455900 + 1

# MI355X: 256 CUs x 64 lanes x 2.4 GHz = 39.32e12 32-bit integer lane-operations per second.
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-blocks", type=int, default=1 << 21)
    return ap.parse_args()


def time_variant(td, torch, sched, src, ct, pt, variant, steps, warmup):
    """Wall time of `steps` encrypt+decrypt steps and per-launch HIP-event durations."""
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
    launch_ms = [a.elapsed_time(b) for a, b in ev]
    return wall, launch_ms


def cpu_baseline(sample_blocks):
    import oracle
    from paper_1305_4376_amd import inputs
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    keys = inputs.key_triple(KEY_SEED)
    data = inputs.message(DATA_SEED, sample_blocks)
    t0 = time.perf_counter()
    oracle.tdes_ecb(*keys, data, decrypt=False, threads=cores)
    dt = time.perf_counter() - t0
    return {"value": round(data.size / dt / 1e9, 6), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"encrypt the first {sample_blocks} blocks ({data.size >> 20} MiB) of the same message "
                      f"with the same key triple, {cores} threads, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); ECB shards need no "
              "communication, so the whole-job rate is the one-GPU rate times the GPU count.", file=sys.stderr)
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

    variants = {"table": td.TDES_VARIANT_TABLE, "bitslice": td.TDES_VARIANT_BITSLICE}
    results = {}
    for name, v in variants.items():
        wall, launch_ms = time_variant(td, torch, sched, src, ct, pt, v, args.steps, args.warmup)
        results[name] = (wall, launch_ms)
    shipped = "table"
    wall, launch_ms = results[shipped]
    # The last decrypt must give the message back.
    ok = bool(torch.equal(pt, src))

    bytes_per_step = 2 * N_BLOCKS * 8
    value = bytes_per_step * args.steps / wall / 1e9
    avg_launch_s = sum(launch_ms) / len(launch_ms) / 1e3
    # VALU instructions per block of the table kernel's round loop: 15 per round x 48 rounds
    # (the prologue and epilogue add about 60 more per block and are not counted).
    ops_per_block = 15 * 48
    achieved_tops = ops_per_block * N_BLOCKS / avg_launch_s / 1e12
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "3DES-EDE ECB, one 1 GiB message (2^27 blocks, SplitMix64 bytes), one 3-key "
                               "triple, encrypt then decrypt per step, one launch each, HBM-resident",
                   "n_blocks": N_BLOCKS, "keying": 3, "variant": shipped},
        "roofline": {"bound": "alu", "achieved": round(achieved_tops, 3), "peak": round(ALU_PEAK_TOPS, 3),
                     "unit": "Tops/s", "frac": round(achieved_tops / ALU_PEAK_TOPS, 4), "traffic": None,
                     "hbm_frac": round(16 * N_BLOCKS / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4)},
        "variants": {n: round(bytes_per_step * args.steps / r[0] / 1e9, 3) for n, r in results.items()},
        "kernel_ms": round(avg_launch_s * 1e3, 4),
        "roundtrip_ok": ok,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample_blocks)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
