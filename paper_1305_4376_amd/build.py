"""Build libtdes.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1305_4376_amd.build

Objects go to paper_1305_4376_amd/_build/ (not committed); the library lands
next to this file, where the Python binding loads it.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtdes.so")
ROOT = os.path.dirname(HERE)

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for all device code (none is used on purpose).
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include")]

SOURCES = ["api.cpp", "keysched.cpp", "batch.cpp", "serve.cpp", "host_path.cpp", "k_table.hip", "k_bitslice.hip", "k_batch.hip", "k_batch_capped.hip", "k_static.hip", "k_util.hip"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # hipcc's host pass does not know the packed-FP32 target feature; that notice is expected.
    noise = "'-packed-fp32-ops' is not a recognized feature"
    text = "\n".join(l for l in res.stdout.splitlines() if noise not in l)
    if text.strip():
        print(text, flush=True)
    if res.returncode != 0:
        raise subprocess.CalledProcessError(res.returncode, cmd)


UNITS_SRC = os.path.join(ROOT, "tests", "units", "k_units.hip")
UNITS_LIB = os.path.join(ROOT, "tests", "units", "libtdes_units.so")


def build_units(verbose: bool = False) -> str:
    """The GPU unit tests' kernels (test infrastructure): tests/units/libtdes_units.so.  Loop headers
    are aligned to 64 bytes: the issue-rate probes' timed loops otherwise start at arbitrary offsets,
    and some placements measured up to 16% slower for reasons of placement alone."""
    tmp = UNITS_LIB + ".tmp"
    _run([HIPCC, *COMMON, "-falign-loops=64", "-x", "hip", "-shared", "-o", tmp, UNITS_SRC], verbose)
    os.replace(tmp, UNITS_LIB)
    return UNITS_LIB


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        _run([HIPCC, *COMMON, *lang, "-c", path, "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
    print(build_units(verbose="-v" in sys.argv))
