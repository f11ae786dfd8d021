"""Helpers shared by the GPU tests: device buffers, schedules and sampled oracle checks."""
from __future__ import annotations

import os

import numpy as np
import torch

import oracle
import paper_1305_4376_amd as td
from paper_1305_4376_amd import inputs

DEV = torch.device("cuda", 0)
# Host threads for the oracle: the cores this process may use, at most 16.
ORACLE_THREADS = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 8))


def device_sched(k1, k2, k3):
    host = td.tdes_expand_key(k1, k2, k3)
    dev = torch.empty(td.TDES_SCHED_BYTES, dtype=torch.uint8, device=DEV)
    td.tdes_sched_upload(host, dev)
    return dev


def to_device(a: np.ndarray, offset: int = 0) -> torch.Tensor:
    """Copy a host uint8 array to a fresh device buffer, `offset` bytes into a 256-aligned allocation."""
    buf = torch.empty(a.size + offset + 16, dtype=torch.uint8, device=DEV)
    view = buf[offset: offset + a.size]
    view.copy_(torch.from_numpy(np.ascontiguousarray(a)))
    return view


def empty_like_dev(n_bytes: int, offset: int = 0) -> torch.Tensor:
    buf = torch.empty(n_bytes + offset + 16, dtype=torch.uint8, device=DEV)
    return buf[offset: offset + n_bytes]


def run(sched, src, dst, n, direction, variant):
    td.tdes_ecb_run(sched, src, dst, n, direction, variant)
    torch.cuda.synchronize()


def device_message(seed: int, n_blocks: int) -> torch.Tensor:
    buf = torch.empty(n_blocks * 8, dtype=torch.uint8, device=DEV)
    td.tdes_fill_splitmix64(buf, n_blocks, seed, 0)
    return buf


def sample_indices(n_blocks: int, count: int, seed: int, boundaries=()) -> np.ndarray:
    rng = np.random.default_rng(seed)
    idx = set(rng.integers(0, n_blocks, size=count).tolist())
    idx.update(range(min(n_blocks, 2048)))
    idx.update(range(max(0, n_blocks - 2048), n_blocks))
    for b in boundaries:
        for d in (-1, 0, 1):
            if 0 <= b + d < n_blocks:
                idx.add(b + d)
    return np.array(sorted(idx), dtype=np.int64)


def gather_blocks(buf: torch.Tensor, idx: np.ndarray) -> np.ndarray:
    t = torch.from_numpy(idx).to(DEV)
    return buf.view(-1, 8)[t].cpu().numpy().reshape(-1)


def oracle_on_blocks(keys, blocks: np.ndarray, decrypt: bool) -> np.ndarray:
    return oracle.tdes_ecb(*keys, blocks, decrypt=decrypt, threads=ORACLE_THREADS)
