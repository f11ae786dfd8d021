"""Triple-DES (EDE) in ECB mode for the AMD MI355X (gfx950).

A thin ctypes binding over libtdes.so, whose C ABI is include/tdes.h.  The
functions below carry the same names as the C entry points and only marshal
arguments: device buffers may be given as torch tensors (their data_ptr) or
as raw integer addresses, and `stream` defaults to torch's current stream.
Every step of the cipher runs in the library's HIP kernels; if the library
is missing, the first call raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "TdesError", "TDES_OK", "TDES_ENCRYPT", "TDES_DECRYPT", "TDES_CHECK_PARITY", "TDES_REJECT_WEAK",
    "TDES_VARIANT_AUTO", "TDES_VARIANT_TABLE", "TDES_VARIANT_BITSLICE", "TDES_SCHED_BYTES",
    "tdes_expand_key", "tdes_sched_upload", "tdes_ecb_encrypt", "tdes_ecb_decrypt", "tdes_ecb_run",
    "tdes_status_str", "tdes_fill_splitmix64", "library_path", "load_library",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtdes.so")

TDES_OK = 0
TDES_ENCRYPT, TDES_DECRYPT = 0, 1
TDES_CHECK_PARITY, TDES_REJECT_WEAK = 1, 2
TDES_VARIANT_AUTO, TDES_VARIANT_TABLE, TDES_VARIANT_BITSLICE = 0, 1, 2
TDES_SCHED_BYTES = 768

_lib = None


class TdesError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {tdes_status_str(code)} (status {code})")


def library_path() -> str:
    return LIB_PATH


def load_library():
    """Load libtdes.so (built in-tree by paper_1305_4376_amd.build); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1305_4376_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    sig = {
        "tdes_expand_key": ([vp, vp, vp, u32, vp], i32),
        "tdes_sched_upload": ([vp, u64, vp, vp], i32),
        "tdes_ecb_encrypt": ([vp, vp, vp, u64, vp], i32),
        "tdes_ecb_decrypt": ([vp, vp, vp, u64, vp], i32),
        "tdes_ecb_run": ([vp, vp, vp, u64, i32, i32, vp], i32),
        "tdes_status_str": ([i32], ctypes.c_char_p),
        "tdes_fill_splitmix64": ([vp, u64, u64, u64, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(x) -> int | None:
    """Device or host address of a torch tensor, numpy array or integer (None stays NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x).__name__}")


def _stream(stream, like=None):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    dev = like.device if hasattr(like, "device") and like.device.type == "cuda" else None
    return torch.cuda.current_stream(dev).cuda_stream


def _nblocks(buf, n_blocks):
    if n_blocks is not None:
        return int(n_blocks)
    if hasattr(buf, "numel"):
        nbytes = buf.numel() * buf.element_size()
        if nbytes % 8:
            raise ValueError("buffer is not a whole number of 8-byte blocks")
        return nbytes // 8
    raise ValueError("n_blocks is required for raw addresses")


def _check(rc: int, where: str):
    if rc != TDES_OK:
        raise TdesError(rc, where)


def tdes_status_str(code: int) -> str:
    return load_library().tdes_status_str(int(code)).decode()


def tdes_expand_key(k1: bytes, k2: bytes, k3: bytes, flags: int = 0) -> np.ndarray:
    """Host key expansion; returns the 768-byte schedule as a uint8 array."""
    keys = []
    for k in (k1, k2, k3):
        b = bytes(k)
        if len(b) != 8:
            raise ValueError("a DES key is 8 bytes")
        keys.append(ctypes.create_string_buffer(b, 8))
    out = np.zeros(TDES_SCHED_BYTES, dtype=np.uint8)
    _check(load_library().tdes_expand_key(*keys, int(flags), out.ctypes.data), "tdes_expand_key")
    return out


def tdes_sched_upload(host, dev_table, count: int | None = None, stream=None) -> None:
    """Copy `count` host schedules (a uint8 array of count*768 bytes) to a device table."""
    h = np.ascontiguousarray(np.asarray(host, dtype=np.uint8).reshape(-1))
    if count is None:
        if h.size % TDES_SCHED_BYTES:
            raise ValueError("host schedules must be a multiple of 768 bytes")
        count = h.size // TDES_SCHED_BYTES
    _check(load_library().tdes_sched_upload(h.ctypes.data, int(count), _ptr(dev_table), _stream(stream, dev_table)),
           "tdes_sched_upload")


def tdes_ecb_run(dev_sched, src, dst, n_blocks=None, direction: int = TDES_ENCRYPT,
                 variant: int = TDES_VARIANT_AUTO, stream=None) -> None:
    n = _nblocks(src, n_blocks)
    _check(load_library().tdes_ecb_run(_ptr(dev_sched), _ptr(src), _ptr(dst), n, int(direction), int(variant),
                                       _stream(stream, src)), "tdes_ecb_run")


def tdes_ecb_encrypt(dev_sched, src, dst, n_blocks=None, stream=None) -> None:
    n = _nblocks(src, n_blocks)
    _check(load_library().tdes_ecb_encrypt(_ptr(dev_sched), _ptr(src), _ptr(dst), n, _stream(stream, src)),
           "tdes_ecb_encrypt")


def tdes_ecb_decrypt(dev_sched, src, dst, n_blocks=None, stream=None) -> None:
    n = _nblocks(src, n_blocks)
    _check(load_library().tdes_ecb_decrypt(_ptr(dev_sched), _ptr(src), _ptr(dst), n, _stream(stream, src)),
           "tdes_ecb_decrypt")


def tdes_fill_splitmix64(dev, n_words: int, seed: int, first: int = 0, stream=None) -> None:
    _check(load_library().tdes_fill_splitmix64(_ptr(dev), int(n_words), int(seed) & (2**64 - 1), int(first),
                                               _stream(stream, dev)), "tdes_fill_splitmix64")
