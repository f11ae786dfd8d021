"""Plain CPU reference for DES / Triple-DES (EDE) in ECB mode, and in the CBC and CTR modes.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product library never does.

The arithmetic lives in ``des_oracle.c`` (a literal transcription of the
Data Encryption Standard, bit by bit); this module only builds it with gcc and
marshals arguments through ctypes.  See that file's header for the passages
of the paper it follows (ECB independence of blocks: Abstract; the EDE order
and its reversal for decryption: Section II.A; three keys giving 48 subkeys:
Listing 1.1).  CBC and CTR go beyond the paper, which is ECB only; they follow
the modes' definitions in NIST SP 800-38A (stated in the C file).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "des_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile des_oracle.c into liboracle.so next to it (gcc -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-pthread",
                               "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u8p = ctypes.c_void_p
        lib.oracle_tdes_ecb.argtypes = [u8p, u8p, u8p, u8p, u8p, ctypes.c_uint64, ctypes.c_int, ctypes.c_int]
        lib.oracle_tdes_ecb.restype = ctypes.c_int
        lib.oracle_des_block.argtypes = [u8p, u8p, u8p, ctypes.c_int]
        lib.oracle_des_block.restype = None
        lib.oracle_des_subkeys_u64.argtypes = [u8p, u8p]
        lib.oracle_des_subkeys_u64.restype = None
        lib.oracle_des_cd_u64.argtypes = [u8p, u8p]
        lib.oracle_des_cd_u64.restype = None
        lib.oracle_des_trace.argtypes = [u8p, u8p, ctypes.c_int, u8p]
        lib.oracle_des_trace.restype = None
        lib.oracle_tdes_cbc.argtypes = [u8p, u8p, u8p, u8p, u8p, u8p, ctypes.c_uint64, ctypes.c_int]
        lib.oracle_tdes_cbc.restype = ctypes.c_int
        lib.oracle_tdes_ctr.argtypes = [u8p, u8p, u8p, u8p, u8p, u8p, ctypes.c_uint64]
        lib.oracle_tdes_ctr.restype = ctypes.c_int
        lib.oracle_table.argtypes = [ctypes.c_char_p, u8p]
        lib.oracle_table.restype = ctypes.c_int
        _lib = lib
    return _lib


def _key(k) -> np.ndarray:
    a = np.frombuffer(bytes(k), dtype=np.uint8) if not isinstance(k, np.ndarray) else k.astype(np.uint8)
    if a.size != 8:
        raise ValueError("a DES key is 8 bytes")
    return np.ascontiguousarray(a)


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def tdes_ecb(k1, k2, k3, data, decrypt: bool = False, threads: int = 1) -> np.ndarray:
    """EDE (or its inverse) over whole 8-byte blocks; returns a new uint8 array."""
    src = np.ascontiguousarray(np.frombuffer(bytes(data), dtype=np.uint8)
                               if isinstance(data, (bytes, bytearray)) else np.asarray(data, dtype=np.uint8).reshape(-1))
    if src.size % 8:
        raise ValueError("ECB works on whole 8-byte blocks")
    out = np.empty_like(src)
    a, b, c = _key(k1), _key(k2), _key(k3)
    rc = _load().oracle_tdes_ecb(_ptr(a), _ptr(b), _ptr(c), _ptr(src), _ptr(out),
                                 src.size // 8, int(bool(decrypt)), int(threads))
    if rc != 0:
        raise RuntimeError("oracle_tdes_ecb failed")
    return out


def _blocks(data) -> np.ndarray:
    src = np.ascontiguousarray(np.frombuffer(bytes(data), dtype=np.uint8)
                               if isinstance(data, (bytes, bytearray)) else np.asarray(data, dtype=np.uint8).reshape(-1))
    if src.size % 8:
        raise ValueError("the modes work on whole 8-byte blocks")
    return src


def tdes_cbc(k1, k2, k3, iv, data, decrypt: bool = False) -> np.ndarray:
    """CBC with TDEA as the block cipher (SP 800-38A), sequential; returns a new uint8 array."""
    src = _blocks(data)
    out = np.empty_like(src)
    a, b, c, v = _key(k1), _key(k2), _key(k3), _key(iv)
    if _load().oracle_tdes_cbc(_ptr(a), _ptr(b), _ptr(c), _ptr(v), _ptr(src), _ptr(out), src.size // 8,
                               int(bool(decrypt))) != 0:
        raise RuntimeError("oracle_tdes_cbc failed")
    return out


def tdes_ctr(k1, k2, k3, iv, data) -> np.ndarray:
    """CTR with TDEA as the block cipher (SP 800-38A): counter block j = IV + j mod 2^64, big-endian."""
    src = _blocks(data)
    out = np.empty_like(src)
    a, b, c, v = _key(k1), _key(k2), _key(k3), _key(iv)
    if _load().oracle_tdes_ctr(_ptr(a), _ptr(b), _ptr(c), _ptr(v), _ptr(src), _ptr(out), src.size // 8) != 0:
        raise RuntimeError("oracle_tdes_ctr failed")
    return out


def tdes_ecb_encrypt(k1, k2, k3, data, threads: int = 1) -> np.ndarray:
    return tdes_ecb(k1, k2, k3, data, False, threads)


def tdes_ecb_decrypt(k1, k2, k3, data, threads: int = 1) -> np.ndarray:
    return tdes_ecb(k1, k2, k3, data, True, threads)


def des_block(key, block, decrypt: bool = False) -> bytes:
    """Single DES on one 8-byte block."""
    k = _key(key)
    b = np.ascontiguousarray(np.frombuffer(bytes(block), dtype=np.uint8))
    if b.size != 8:
        raise ValueError("a DES block is 8 bytes")
    out = np.empty(8, dtype=np.uint8)
    _load().oracle_des_block(_ptr(k), _ptr(b), _ptr(out), int(bool(decrypt)))
    return out.tobytes()


def des_subkeys(key) -> list[int]:
    """K1..K16 as 48-bit integers, subkey bit 1 in bit 47."""
    k = _key(key)
    out = np.empty(16, dtype=np.uint64)
    _load().oracle_des_subkeys_u64(_ptr(k), _ptr(out))
    return [int(v) for v in out]


def des_cd(key) -> list[int]:
    """C_i||D_i for i = 0..16 as 56-bit integers (C bit 1 in bit 55)."""
    k = _key(key)
    out = np.empty(17, dtype=np.uint64)
    _load().oracle_des_cd_u64(_ptr(k), _ptr(out))
    return [int(v) for v in out]


def des_trace(key, block, decrypt: bool = False) -> list[int]:
    """L_i||R_i for i = 0..16 of one DES block (L bit 1 in bit 63)."""
    k = _key(key)
    b = np.ascontiguousarray(np.frombuffer(bytes(block), dtype=np.uint8))
    out = np.empty(17, dtype=np.uint64)
    _load().oracle_des_trace(_ptr(k), _ptr(b), int(bool(decrypt)), _ptr(out))
    return [int(v) for v in out]


def table(name: str) -> list[int]:
    """One of the standard's tables as held by the oracle (IP, FP, E, P, PC1, PC2, SHIFTS, SBOX)."""
    lib = _load()
    n = lib.oracle_table(name.encode(), None)
    if n < 0:
        raise KeyError(name)
    out = np.empty(n, dtype=np.uint8)
    lib.oracle_table(name.encode(), _ptr(out))
    return [int(v) for v in out]
