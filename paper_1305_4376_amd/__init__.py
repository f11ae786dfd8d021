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
    "JOB_DTYPE", "TDES_BATCH_NO_GRAPH", "TDES_BATCH_PER_MESSAGE", "tdes_ctx_create", "tdes_ctx_destroy",
    "tdes_ecb_batch", "tdes_ecb_batch_replay", "tdes_ctx_set_tuning", "tdes_ctx_get_info",
    "REQUEST_DTYPE", "COMPLETION_DTYPE", "tdes_server_create", "tdes_server_destroy", "tdes_server_now",
    "tdes_server_submit", "tdes_server_cancel", "tdes_server_poll", "tdes_server_wait_idle",
    "tdes_server_release", "tdes_server_stats", "tdes_server_run_trace", "tdes_ecb_host",
    "tdes_ctr_crypt", "tdes_cbc_decrypt", "tdes_ecb_chunked", "TDES_STATIC_MAX_JOBS", "tdes_ecb_batch_static",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtdes.so")

TDES_OK = 0
TDES_ENCRYPT, TDES_DECRYPT = 0, 1
TDES_CHECK_PARITY, TDES_REJECT_WEAK = 1, 2
TDES_VARIANT_AUTO, TDES_VARIANT_TABLE, TDES_VARIANT_BITSLICE = 0, 1, 2
TDES_SCHED_BYTES = 1600
TDES_BATCH_NO_GRAPH, TDES_BATCH_PER_MESSAGE = 1, 2
TDES_STATIC_MAX_JOBS = 65536

# struct tdes_job (include/tdes.h): 32 bytes.
JOB_DTYPE = np.dtype([("in_off", "<u8"), ("out_off", "<u8"), ("n_blocks", "<u8"), ("sched_idx", "<u4"),
                      ("direction", "<u4")])


# struct tdes_request: 48 bytes; struct tdes_completion: 64 bytes.
REQUEST_DTYPE = np.dtype([("n_blocks", "<u8"), ("key_id", "<u4"), ("direction", "<u4"), ("seed", "<u8"),
                          ("host_in", "<u8"), ("host_out", "<u8"), ("user_tag", "<u8")])
COMPLETION_DTYPE = np.dtype([("id", "<u8"), ("user_tag", "<u8"), ("status", "<i4"), ("pad", "<u4"),
                             ("t_arrival", "<f8"), ("t_admit", "<f8"), ("t_launch", "<f8"),
                             ("t_complete", "<f8"), ("dev_out", "<u8")])


class _ServeConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_uint32),
                ("max_step_jobs", ctypes.c_uint32), ("max_step_blocks", ctypes.c_uint64),
                ("keep_outputs", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("threads", ctypes.c_uint32), ("groups_per_cu", ctypes.c_uint32),
                ("wave_remainder", ctypes.c_uint32), ("tiles_per_draw", ctypes.c_uint32),
                ("backlog_step_blocks", ctypes.c_uint64)]


class _ServeStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "canceled", "bytes", "steps",
                                               "max_step_jobs", "peak_pool_bytes", "pool_bytes_in_use",
                                               "pending")]


class _BatchInfo(ctypes.Structure):
    _fields_ = [("tiles", ctypes.c_uint64), ("wave_tiles", ctypes.c_uint64), ("lane_tiles", ctypes.c_uint64),
                ("slots", ctypes.c_uint64), ("blocks", ctypes.c_uint64), ("padded_blocks", ctypes.c_uint64),
                ("threads", ctypes.c_uint32), ("groups_per_cu", ctypes.c_uint32),
                ("graph_captures", ctypes.c_uint32), ("wave_remainder", ctypes.c_uint32),
                ("tiles_per_draw", ctypes.c_uint32), ("pad", ctypes.c_uint32)]

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
        "tdes_ctr_crypt": ([vp, vp, vp, vp, u64, vp], i32),
        "tdes_ecb_chunked": ([vp, vp, vp, u64, u64, i32, i32, u32, vp], i32),
        "tdes_cbc_decrypt": ([vp, vp, vp, vp, u64, vp], i32),
        "tdes_status_str": ([i32], ctypes.c_char_p),
        "tdes_fill_splitmix64": ([vp, u64, u64, u64, vp], i32),
        "tdes_ctx_create": ([ctypes.POINTER(vp), i32], i32),
        "tdes_ctx_destroy": ([vp], i32),
        "tdes_ecb_batch": ([vp, vp, u32, vp, u64, vp, u32, vp], i32),
        "tdes_ecb_batch_replay": ([vp, u32, vp], i32),
        "tdes_ecb_batch_static": ([vp, u32, vp, u64, vp, u64, vp, vp], i32),
        "tdes_ctx_set_tuning": ([vp, u32, u32, u32, u32], i32),
        "tdes_ctx_get_info": ([vp, ctypes.POINTER(_BatchInfo)], i32),
        "tdes_server_create": ([ctypes.POINTER(vp), ctypes.POINTER(_ServeConfig), vp, u64], i32),
        "tdes_server_destroy": ([vp], i32),
        "tdes_server_now": ([vp], ctypes.c_double),
        "tdes_server_submit": ([vp, vp, ctypes.POINTER(u64)], i32),
        "tdes_server_cancel": ([vp, u64], i32),
        "tdes_server_poll": ([vp, vp, u32, ctypes.POINTER(u32)], i32),
        "tdes_server_wait_idle": ([vp, ctypes.c_double], i32),
        "tdes_server_release": ([vp, u64], i32),
        "tdes_server_stats": ([vp, ctypes.POINTER(_ServeStats)], i32),
        "tdes_server_run_trace": ([vp, vp, vp, u64, vp], i32),
        "tdes_ecb_host": ([vp, vp, vp, u64, i32, u64, vp], i32),
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


def _nbytes(x) -> int | None:
    """Size in bytes of a torch tensor or numpy array (its data must be contiguous); None for raw addresses."""
    if x is None or isinstance(x, int):
        return None
    if hasattr(x, "numel"):
        if not x.is_contiguous():
            raise ValueError("buffers must be contiguous")
        return x.numel() * x.element_size()
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("buffers must be contiguous")
        return x.nbytes
    return None


def _need(x, nbytes: int, what: str) -> None:
    """Raise before any C call if a sized buffer is smaller than the call would touch."""
    have = _nbytes(x)
    if have is not None and nbytes > have:
        raise ValueError(f"{what}: the call touches {nbytes} bytes but the buffer holds {have}")


def _nblocks(buf, n_blocks):
    if n_blocks is not None:
        n = int(n_blocks)
        if n < 0:
            raise ValueError("n_blocks must not be negative")
        return n
    nbytes = _nbytes(buf)
    if nbytes is not None:
        if nbytes % 8:
            raise ValueError("buffer is not a whole number of 8-byte blocks")
        return nbytes // 8
    raise ValueError("n_blocks is required for raw addresses")


def _message_args(dev_sched, src, dst, n_blocks):
    """Block count of a one-message call, with every sized buffer checked against it."""
    n = _nblocks(src, n_blocks)
    _need(dev_sched, TDES_SCHED_BYTES, "schedule")
    _need(src, 8 * n, "input")
    _need(dst, 8 * n, "output")
    return n


def _check(rc: int, where: str):
    if rc != TDES_OK:
        raise TdesError(rc, where)


def tdes_status_str(code: int) -> str:
    return load_library().tdes_status_str(int(code)).decode()


def tdes_expand_key(k1: bytes, k2: bytes, k3: bytes, flags: int = 0) -> np.ndarray:
    """Host key expansion; returns the TDES_SCHED_BYTES-byte schedule as a uint8 array."""
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
    """Copy `count` host schedules (a uint8 array of count*TDES_SCHED_BYTES bytes) to a device table."""
    h = np.ascontiguousarray(np.asarray(host, dtype=np.uint8).reshape(-1))
    if count is None:
        if h.size % TDES_SCHED_BYTES:
            raise ValueError(f"host schedules must be a multiple of {TDES_SCHED_BYTES} bytes")
        count = h.size // TDES_SCHED_BYTES
    if int(count) * TDES_SCHED_BYTES > h.size:
        raise ValueError(f"{count} schedules need {int(count) * TDES_SCHED_BYTES} host bytes, {h.size} given")
    _need(dev_table, int(count) * TDES_SCHED_BYTES, "schedule table")
    _check(load_library().tdes_sched_upload(h.ctypes.data, int(count), _ptr(dev_table), _stream(stream, dev_table)),
           "tdes_sched_upload")


def tdes_ecb_run(dev_sched, src, dst, n_blocks=None, direction: int = TDES_ENCRYPT,
                 variant: int = TDES_VARIANT_AUTO, stream=None) -> None:
    n = _message_args(dev_sched, src, dst, n_blocks)
    _check(load_library().tdes_ecb_run(_ptr(dev_sched), _ptr(src), _ptr(dst), n, int(direction), int(variant),
                                       _stream(stream, src)), "tdes_ecb_run")


def _iv_buffer(iv):
    b = bytes(iv) if iv is not None else None
    if b is not None and len(b) != 8:
        raise ValueError("an IV is 8 bytes")
    return ctypes.create_string_buffer(b, 8) if b is not None else None


def tdes_ecb_chunked(dev_sched, src, dst, chunk_blocks: int, n_blocks=None, direction: int = TDES_ENCRYPT,
                     variant: int = TDES_VARIANT_AUTO, threads: int = 0, stream=None) -> None:
    """The paper's host loop: one launch per chunk of chunk_blocks blocks, workgroups of `threads` (0: default)."""
    n = _message_args(dev_sched, src, dst, n_blocks)
    _check(load_library().tdes_ecb_chunked(_ptr(dev_sched), _ptr(src), _ptr(dst), n, int(chunk_blocks),
                                           int(direction), int(variant), int(threads), _stream(stream, src)),
           "tdes_ecb_chunked")


def tdes_ctr_crypt(dev_sched, iv, src, dst, n_blocks=None, stream=None) -> None:
    """CTR mode (encrypt or decrypt): dst = src XOR EDE(iv + j)."""
    n = _message_args(dev_sched, src, dst, n_blocks)
    _check(load_library().tdes_ctr_crypt(_ptr(dev_sched), _iv_buffer(iv), _ptr(src), _ptr(dst), n,
                                         _stream(stream, src)), "tdes_ctr_crypt")


def tdes_cbc_decrypt(dev_sched, iv, src, dst, n_blocks=None, stream=None) -> None:
    """CBC decryption: dst[j] = EDE^-1(src[j]) XOR src[j-1], src[-1] = iv; src and dst must not overlap."""
    n = _message_args(dev_sched, src, dst, n_blocks)
    _check(load_library().tdes_cbc_decrypt(_ptr(dev_sched), _iv_buffer(iv), _ptr(src), _ptr(dst), n,
                                           _stream(stream, src)), "tdes_cbc_decrypt")


def tdes_ecb_encrypt(dev_sched, src, dst, n_blocks=None, stream=None) -> None:
    n = _message_args(dev_sched, src, dst, n_blocks)
    _check(load_library().tdes_ecb_encrypt(_ptr(dev_sched), _ptr(src), _ptr(dst), n, _stream(stream, src)),
           "tdes_ecb_encrypt")


def tdes_ecb_decrypt(dev_sched, src, dst, n_blocks=None, stream=None) -> None:
    n = _message_args(dev_sched, src, dst, n_blocks)
    _check(load_library().tdes_ecb_decrypt(_ptr(dev_sched), _ptr(src), _ptr(dst), n, _stream(stream, src)),
           "tdes_ecb_decrypt")


def tdes_fill_splitmix64(dev, n_words: int, seed: int, first: int = 0, stream=None) -> None:
    _need(dev, 8 * int(n_words), "output")
    _check(load_library().tdes_fill_splitmix64(_ptr(dev), int(n_words), int(seed) & (2**64 - 1), int(first),
                                               _stream(stream, dev)), "tdes_fill_splitmix64")


def tdes_ctx_create(device: int = -1) -> int:
    """A batch context on HIP device `device` (-1: the current device); an opaque handle."""
    h = ctypes.c_void_p()
    _check(load_library().tdes_ctx_create(ctypes.byref(h), int(device)), "tdes_ctx_create")
    return h.value


def tdes_ctx_destroy(ctx: int) -> None:
    _check(load_library().tdes_ctx_destroy(ctx), "tdes_ctx_destroy")


def tdes_ecb_batch(ctx: int, jobs: np.ndarray, dev_sched_table, n_scheds: int, dev_base, flags: int = 0,
                   stream=None) -> None:
    """jobs: a JOB_DTYPE array (host).  Offsets are relative to dev_base."""
    j = np.ascontiguousarray(jobs, dtype=JOB_DTYPE)
    _need(dev_sched_table, int(n_scheds) * TDES_SCHED_BYTES, "schedule table")
    if j.size and _nbytes(dev_base) is not None:
        ends = 8 * j["n_blocks"].astype(np.uint64)
        reach = max(int((j["in_off"] + ends).max()), int((j["out_off"] + ends).max()))
        _need(dev_base, reach, "batch base")
    _check(load_library().tdes_ecb_batch(ctx, j.ctypes.data, int(j.size), _ptr(dev_sched_table), int(n_scheds),
                                         _ptr(dev_base), int(flags), _stream(stream, dev_base)), "tdes_ecb_batch")


def tdes_ecb_batch_static(dev_jobs, n_jobs: int, dev_sched_table, n_scheds: int, dev_base, base_bytes=None,
                          dev_rejected=None, stream=None) -> None:
    """The allocation-free batch: dev_jobs is a device buffer of n_jobs JOB_DTYPE records; base_bytes
    defaults to dev_base's size; dev_rejected (device, one uint32, optional) receives the refused-job count."""
    _need(dev_jobs, int(n_jobs) * JOB_DTYPE.itemsize, "job table")
    _need(dev_sched_table, int(n_scheds) * TDES_SCHED_BYTES, "schedule table")
    _need(dev_rejected, 4, "rejected count")
    have = _nbytes(dev_base)
    if base_bytes is None:
        if have is None:
            raise ValueError("base_bytes is required for a raw base address")
        base_bytes = have
    _need(dev_base, int(base_bytes), "batch base")
    _check(load_library().tdes_ecb_batch_static(_ptr(dev_jobs), int(n_jobs), _ptr(dev_sched_table), int(n_scheds),
                                                _ptr(dev_base), int(base_bytes), _ptr(dev_rejected),
                                                _stream(stream, dev_base)), "tdes_ecb_batch_static")


def tdes_ecb_batch_replay(ctx: int, flags: int = 0, stream=None) -> None:
    _check(load_library().tdes_ecb_batch_replay(ctx, int(flags), _stream(stream)), "tdes_ecb_batch_replay")


def tdes_ctx_set_tuning(ctx: int, threads: int, groups_per_cu: int, wave_remainder: int = 0,
                        tiles_per_draw: int = 0) -> None:
    _check(load_library().tdes_ctx_set_tuning(ctx, int(threads), int(groups_per_cu), int(wave_remainder),
                                              int(tiles_per_draw)), "tdes_ctx_set_tuning")


def tdes_ctx_get_info(ctx: int) -> dict:
    info = _BatchInfo()
    _check(load_library().tdes_ctx_get_info(ctx, ctypes.byref(info)), "tdes_ctx_get_info")
    return {name: getattr(info, name) for name, _ in info._fields_ if name != "pad"}


def tdes_server_create(dev_sched_table, n_scheds: int, budget_bytes: int, max_inflight: int = 2,
                       max_step_jobs: int = 4096, max_step_blocks: int = 1 << 26, keep_outputs: bool = False,
                       tuning=None, backlog_step_blocks: int = 0) -> int:
    """Start a serving engine over a resident schedule table; returns an opaque handle.  tuning: the
    batch shape (threads, groups_per_cu, wave_remainder, tiles_per_draw) of every step, None for the
    library's defaults, or "cached" for the shape the autotuner recorded for servers with this step
    size on this GPU (the defaults if none).  backlog_step_blocks: the largest step while the queue
    is long (see tdes_serve_config); 0 keeps every step at max_step_blocks."""
    _need(dev_sched_table, int(n_scheds) * TDES_SCHED_BYTES, "schedule table")
    if isinstance(tuning, str):
        if tuning != "cached":
            raise ValueError('tuning is a 4-tuple, None or "cached"')
        from paper_1305_4376_amd import autotune
        tuning = autotune.cached_serving(int(max_step_blocks))
    t = tuple(int(v) for v in tuning) if tuning is not None else (0, 0, 0, 0)
    if len(t) != 4:
        raise ValueError("tuning is (threads, groups_per_cu, wave_remainder, tiles_per_draw)")
    cfg = _ServeConfig(int(budget_bytes), int(max_inflight), int(max_step_jobs), int(max_step_blocks),
                       int(bool(keep_outputs)), 0, *t, int(backlog_step_blocks))
    h = ctypes.c_void_p()
    _check(load_library().tdes_server_create(ctypes.byref(h), ctypes.byref(cfg), _ptr(dev_sched_table),
                                             int(n_scheds)), "tdes_server_create")
    return h.value


def tdes_server_destroy(server: int) -> None:
    _check(load_library().tdes_server_destroy(server), "tdes_server_destroy")


def tdes_server_now(server: int) -> float:
    return load_library().tdes_server_now(server)


def tdes_server_submit(server: int, req: np.ndarray) -> int:
    """req: one REQUEST_DTYPE record; returns the request id."""
    r = np.ascontiguousarray(np.asarray(req, dtype=REQUEST_DTYPE).reshape(1))
    rid = ctypes.c_uint64()
    _check(load_library().tdes_server_submit(server, r.ctypes.data, ctypes.byref(rid)), "tdes_server_submit")
    return rid.value


def tdes_server_cancel(server: int, rid: int) -> None:
    _check(load_library().tdes_server_cancel(server, int(rid)), "tdes_server_cancel")


def tdes_server_poll(server: int, max_records: int = 4096) -> np.ndarray:
    out = np.zeros(max_records, dtype=COMPLETION_DTYPE)
    n = ctypes.c_uint32()
    _check(load_library().tdes_server_poll(server, out.ctypes.data, int(max_records), ctypes.byref(n)),
           "tdes_server_poll")
    return out[: n.value]


def tdes_server_wait_idle(server: int, timeout_s: float = 60.0) -> None:
    _check(load_library().tdes_server_wait_idle(server, float(timeout_s)), "tdes_server_wait_idle")


def tdes_server_release(server: int, rid: int) -> None:
    _check(load_library().tdes_server_release(server, int(rid)), "tdes_server_release")


def tdes_server_stats(server: int) -> dict:
    st = _ServeStats()
    _check(load_library().tdes_server_stats(server, ctypes.byref(st)), "tdes_server_stats")
    return {name: getattr(st, name) for name, _ in st._fields_}


def tdes_server_run_trace(server: int, reqs: np.ndarray, arrival_s: np.ndarray) -> np.ndarray:
    """Open-loop run: request i is submitted arrival_s[i] seconds after the start; returns completions."""
    r = np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
    a = np.ascontiguousarray(arrival_s, dtype=np.float64)
    if r.size != a.size:
        raise ValueError("one arrival time per request")
    out = np.zeros(r.size, dtype=COMPLETION_DTYPE)
    _check(load_library().tdes_server_run_trace(server, r.ctypes.data, a.ctypes.data, int(r.size),
                                                out.ctypes.data), "tdes_server_run_trace")
    return out


def tdes_ecb_host(dev_sched, host_in, host_out, n_blocks=None, direction: int = TDES_ENCRYPT,
                  chunk_blocks: int = 1 << 22, stream=None) -> None:
    """ECB over a host-resident message (numpy arrays or pinned tensors), copies overlapped in chunks."""
    n = _message_args(dev_sched, host_in, host_out, n_blocks)
    _check(load_library().tdes_ecb_host(_ptr(dev_sched), _ptr(host_in), _ptr(host_out), int(n), int(direction),
                                        int(chunk_blocks), _stream(stream)), "tdes_ecb_host")
