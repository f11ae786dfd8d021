"""VALU issue rates on the GPU: the measurement behind the integer-ALU peak.

    python tests/units/issue_rate.py [--iters N]

For each instruction kind of the bitsliced kernel (two-source XOR and add,
shifts, v_bitop3_b32 with its three sources in three register banks or two of
them in one bank, v_perm_b32, v_bitop3_b32 chains in which each instruction
reads the result of the one 1, 2, 3, 4 or 8 before it, and the round's scalar
operand forms: a scalar key mask as a v_bitop3_b32 or v_xor_b32 source, and a
scalar bit-field extract per five v_bitop3_b32), the probe in k_units.hip runs streams of
independent instructions (blocks of 128 between the loop's scalar branch)
at 1, 2, 4 and 8 waves per SIMD (256-thread
workgroups, compute-unit count x waves workgroups).  Each wave records the
shader clock counter (s_memtime) and the 100 MHz real-time counter
(s_memrealtime) around its stream, and the SIMD it ran on (HW_ID and XCC_ID
registers).  Per SIMD, the rate is the instructions of all its waves over the
shader cycles from the first wave's start to the last wave's end; the table
gives the median over SIMDs, the spread of waves per SIMD (the placement the
hardware chose), the rate from the launch's wall time at the nominal 2.4 GHz,
and the shader clock (s_memtime cycles over real time).  One
wave-instruction per SIMD per cycle is 64 lane-operations; 0.5 per cycle on
each of a CU's 4 SIMDs is 128 lane-operations per CU per cycle, the rate
behind 256 CUs x 128 x 2.4 GHz = 78.6 T lane-operations per second.
"""
from __future__ import annotations

import argparse
import ctypes
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libtdes_units.so")
OPS = ["v_xor_b32", "v_add_u32", "v_lshrrev_b32", "v_lshlrev_b32", "v_bitop3_b32 (3 banks)",
       "v_bitop3_b32 (2 in one bank)", "v_perm_b32", "v_bitop3_b32 chain, each on the one before",
       "v_bitop3_b32 chain, each on the one 2 before", "v_bitop3_b32 chain, each on the one 4 before",
       "v_bitop3_b32 chain, each on the one 3 before", "v_bitop3_b32 chain, each on the one 8 before",
       "v_bitop3_b32 chain, each on the one 4 before, results in rotating banks",
       "v_bitop3_b32, sources in banks 0, 1, 2, result in bank 3", "v_bitop3_b32, sources in banks 0, 1, 2, result in bank 0",
       "v_bitop3_b32 with a scalar third source", "v_xor_b32 with a scalar first source",
       "s_bfe_i32 then five v_bitop3_b32, the first reading its result (counted: VALU only)"]
NOMINAL_HZ = 2.4e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=1000, help="128-instruction blocks per wave")
    ap.add_argument("--lib", default=LIB, help="unit-kernel library to load")
    ap.add_argument("--ops", default=",".join(str(i) for i in range(len(OPS))),
                    help="instruction kinds to time (indices into the list); empty for the round pair only")
    args = ap.parse_args()
    import torch
    if not os.path.exists(args.lib):
        sys.exit(f"{args.lib} is missing: build with __graft_entry__.build()")
    lib = ctypes.CDLL(args.lib)
    lib.units_issue_probe.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
    dev = torch.device("cuda", 0)
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    print(f"device: {torch.cuda.get_device_name(dev)}, {n_cu} compute units; {args.iters} x 128 instructions per wave")
    print("| instruction | waves/SIMD | per SIMD per cycle (median over SIMDs) | waves per SIMD (min-max) | "
          "per SIMD per cycle (wall, 2.4 GHz) | lane-ops/CU/cycle | shader clock GHz |")
    print("|---|---|---|---|---|---|---|")
    for op in [int(v) for v in args.ops.split(",") if v.strip()]:
        name = OPS[op]
        for waves in (1, 2, 4, 8):
            groups = n_cu * waves
            clk = torch.zeros(6 * 4 * groups, dtype=torch.int64, device=dev)
            assert lib.units_issue_probe(op, groups, 20, clk.data_ptr()) == 0  # warm-up
            start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            start.record()
            rc = lib.units_issue_probe(op, groups, args.iters, clk.data_ptr())
            stop.record()
            torch.cuda.synchronize()
            assert rc == 0
            wall = start.elapsed_time(stop) / 1e3
            c = clk.cpu().numpy().reshape(-1, 6)
            instr = (640.0 if op == 17 else 128.0) * args.iters   # VALU instructions per wave
            simd = (c[:, 5] << 16) | (c[:, 4] & 0xFF30)  # XCC, SE, SH, CU, SIMD
            rates, counts = [], []
            for key in np.unique(simd):
                w = c[simd == key]
                span = float(w[:, 1].max() - w[:, 0].min())
                rates.append(len(w) * instr / span)
                counts.append(len(w))
            per_cycle = float(np.median(rates))
            per_wall = (4 * groups * instr) / (4 * n_cu) / (wall * NOMINAL_HZ)
            cycles = (c[:, 1] - c[:, 0]).astype(np.float64)
            seconds = (c[:, 3] - c[:, 2]).astype(np.float64) / 100e6
            ghz = float(np.median(cycles / seconds)) / 1e9
            print(f"| {name} | {waves} | {per_cycle:.3f} | {min(counts)}-{max(counts)} | {per_wall:.3f} | "
                  f"{per_cycle * 64 * 4:.1f} | {ghz:.3f} |", flush=True)
    rounds_rate(lib, torch, dev, n_cu, 200, 514)


def rounds_rate(lib, torch, dev, n_cu, iters, valu_per_pair):
    """The bitsliced kernels' folded round pair alone (generated assembly, no memory): its VALU rate
    per SIMD at 4 waves per SIMD (the kernels' occupancy), measured as above."""
    lib.units_rounds_probe.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    groups = n_cu * 4
    clk = torch.zeros(6 * 4 * groups, dtype=torch.int64, device=dev)
    sink = torch.zeros(256 * groups, dtype=torch.int32, device=dev)
    assert lib.units_rounds_probe(groups, 4, clk.data_ptr(), sink.data_ptr()) == 0
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    assert lib.units_rounds_probe(groups, iters, clk.data_ptr(), sink.data_ptr()) == 0
    stop.record()
    torch.cuda.synchronize()
    c = clk.cpu().numpy().reshape(-1, 6)
    simd = (c[:, 5] << 16) | (c[:, 4] & 0xFF30)
    rates = []
    for key in np.unique(simd):
        w = c[simd == key]
        rates.append(len(w) * iters * valu_per_pair / float(w[:, 1].max() - w[:, 0].min()))
    cycles = (c[:, 1] - c[:, 0]).astype(np.float64)
    ghz = float(np.median(cycles / ((c[:, 3] - c[:, 2]).astype(np.float64) / 100e6))) / 1e9
    print(f"| folded round pair ({valu_per_pair} VALU) | 4 | {float(np.median(rates)):.3f} | | "
          f"{n_cu * 16 * iters * valu_per_pair / (4 * n_cu) / (start.elapsed_time(stop) / 1e3 * NOMINAL_HZ):.3f} | "
          f"{float(np.median(rates)) * 256:.1f} | {ghz:.3f} |", flush=True)


if __name__ == "__main__":
    main()
