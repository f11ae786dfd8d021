"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no part of the cipher: only the SplitMix64 generator
(Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014) used counter-style, so that any slice of a message can be
regenerated on its own, and the key recipe.

Recipe:
  * word i of a stream with seed s is the (i+1)-th SplitMix64 output,
    mix(s + (i + 1) * 0x9E3779B97F4A7C15);
  * message block i is the 8 little-endian bytes of word i;
  * a key triple is 24 bytes taken the same way from a key seed, each byte's
    least significant bit then set so that the byte has odd parity (the
    standard's parity convention; the cipher ignores these bits);
  * a served request's payload (made on the device when it is admitted) takes
    the stream's words as chain heads: word i = 256 * (64 * c + k) + t
    (t < 256, k < 64) is X^k(SplitMix64 word 16384 * c + t), X the xorshift64
    step (Marsaglia, "Xorshift RNGs", J. Stat. Softw. 8(14), 2003, shifts
    13, 7, 17), which costs the device three shifts and XORs per word instead
    of two 64-bit multiplications.

The device-side generator in the library implements the same published
definition on its own; tests compare the two.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Seeds of the workloads: data 0x3DE50000 + config + 16 * repetition, keys 0x4B455900 + config.
DATA_SEED_BASE = 0x3DE50000
KEY_SEED_BASE = 0x4B455900


def splitmix64(seed: int, first: int, count: int) -> np.ndarray:
    """Words first .. first+count-1 of the SplitMix64 stream seeded with `seed`."""
    with np.errstate(over="ignore"):
        idx = np.arange(first + 1, first + 1 + count, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_at(seed: int, indices: np.ndarray) -> np.ndarray:
    """Words at arbitrary indices of the stream (for sampled checks of huge messages)."""
    with np.errstate(over="ignore"):
        idx = np.asarray(indices, dtype=np.uint64) + np.uint64(1)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


PAYLOAD_COLUMNS = 256
PAYLOAD_CHAIN = 64


def xorshift64(x: np.ndarray) -> np.ndarray:
    """One xorshift64 step (shifts 13, 7, 17) on each 64-bit word."""
    x = x ^ (x << np.uint64(13))
    x = x ^ (x >> np.uint64(7))
    return x ^ (x << np.uint64(17))


def payload_words_at(seed: int, indices) -> np.ndarray:
    """Words at the given indices of a served request's payload (chain heads from the SplitMix64
    stream, each following word one xorshift64 step on from the one 256 before it in its chain)."""
    i = np.asarray(indices, dtype=np.uint64)
    col = i % np.uint64(PAYLOAD_COLUMNS)
    row = i // np.uint64(PAYLOAD_COLUMNS)
    step = (row % np.uint64(PAYLOAD_CHAIN)).astype(np.int64)
    head = (row // np.uint64(PAYLOAD_CHAIN)) * np.uint64(PAYLOAD_COLUMNS * PAYLOAD_CHAIN) + col
    x = splitmix64_at(seed, head)
    for k in range(1, PAYLOAD_CHAIN):
        x = np.where(step >= k, xorshift64(x), x)
    return x


def payload(seed: int, n_blocks: int) -> np.ndarray:
    """A served request's n_blocks-block payload (uint8 array of 8*n_blocks)."""
    span = PAYLOAD_COLUMNS * PAYLOAD_CHAIN
    chains = -(-n_blocks // span)
    w = np.empty((chains, PAYLOAD_CHAIN, PAYLOAD_COLUMNS), dtype=np.uint64)
    heads = (np.arange(chains, dtype=np.uint64)[:, None] * np.uint64(span)
             + np.arange(PAYLOAD_COLUMNS, dtype=np.uint64)[None, :])
    w[:, 0, :] = splitmix64_at(seed, heads)
    for k in range(1, PAYLOAD_CHAIN):
        w[:, k, :] = xorshift64(w[:, k - 1, :])
    return w.reshape(-1)[:n_blocks].astype("<u8").view(np.uint8)


def message(seed: int, n_blocks: int, first_block: int = 0) -> np.ndarray:
    """n_blocks 8-byte blocks (uint8 array of 8*n_blocks) of a seeded message."""
    w = splitmix64(seed, first_block, n_blocks).astype("<u8")
    return w.view(np.uint8)


def blocks_at(seed: int, indices) -> np.ndarray:
    """The 8-byte blocks at the given indices, as a uint8 array of 8*len(indices)."""
    return splitmix64_at(seed, indices).astype("<u8").view(np.uint8)


def odd_parity(key: bytes) -> bytes:
    """Set each byte's least significant bit so that the byte has an odd number of ones."""
    out = bytearray()
    for b in key:
        hi = b & 0xFE
        out.append(hi | (0 if bin(hi).count("1") % 2 else 1))
    return bytes(out)


def key_triple(seed: int, keying: int = 3) -> tuple[bytes, bytes, bytes]:
    """A random triple with odd parity.  keying 3: three keys; 2: K3 = K1; 1: K1 = K2 = K3."""
    raw = splitmix64(seed, 0, 3).astype("<u8").view(np.uint8).tobytes()
    k1, k2, k3 = (odd_parity(raw[8 * i: 8 * i + 8]) for i in range(3))
    if keying == 2:
        k3 = k1
    elif keying == 1:
        k2 = k3 = k1
    elif keying != 3:
        raise ValueError("keying option is 1, 2 or 3")
    return k1, k2, k3


def key_triples(seed: int, count: int) -> np.ndarray:
    """count random three-key triples, shape (count, 24) uint8, odd parity in every byte."""
    raw = splitmix64(seed, 0, 3 * count).astype("<u8").view(np.uint8).reshape(count, 24)
    hi = raw & np.uint8(0xFE)
    ones = np.unpackbits(hi[..., None], axis=-1).sum(axis=-1)
    return (hi | ((ones % 2) == 0).astype(np.uint8)).astype(np.uint8)


def log_uniform_lengths(seed: int, count: int, max_blocks: int) -> np.ndarray:
    """Message lengths min(max, floor(exp(u * ln(max + 1)))) with u uniform in [0, 1); at least 1."""
    u = (splitmix64(seed, 0, count) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    n = np.floor(np.exp(u * np.log(max_blocks + 1.0))).astype(np.int64)
    return np.clip(n, 1, max_blocks)
