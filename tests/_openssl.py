"""OpenSSL's DES, DES-EDE3-ECB and DES-EDE3-CBC through ctypes: an outside library used only to pin the oracle.

It is used only if libcrypto can be loaded; the tests that use it skip otherwise.
"""
from __future__ import annotations

import ctypes
import ctypes.util

import numpy as np

_lib = None


def available() -> bool:
    return _load() is not None


def _load():
    global _lib
    if _lib is None:
        for name in ("libcrypto.so.3", ctypes.util.find_library("crypto")):
            if not name:
                continue
            try:
                lib = ctypes.CDLL(name)
            except OSError:
                continue
            vp = ctypes.c_void_p
            lib.EVP_CIPHER_CTX_new.restype = vp
            lib.EVP_CIPHER_CTX_free.argtypes = [vp]
            lib.EVP_des_ede3_ecb.restype = vp
            lib.EVP_des_ede3_cbc.restype = vp
            lib.EVP_CipherInit_ex.argtypes = [vp, vp, vp, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int]
            lib.EVP_CIPHER_CTX_set_padding.argtypes = [vp, ctypes.c_int]
            lib.EVP_CipherUpdate.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int), vp, ctypes.c_int]
            lib.DES_set_key_unchecked.argtypes = [ctypes.c_char_p, vp]
            lib.DES_ecb_encrypt.argtypes = [ctypes.c_char_p, vp, vp, ctypes.c_int]
            _lib = lib
            break
    return _lib


def _evp(cipher, key: bytes, iv, data, decrypt: bool) -> np.ndarray:
    lib = _load()
    src = np.ascontiguousarray(np.asarray(data, dtype=np.uint8).reshape(-1))
    out = np.empty(src.size + 16, dtype=np.uint8)
    ctx = lib.EVP_CIPHER_CTX_new()
    try:
        if lib.EVP_CipherInit_ex(ctx, cipher, None, key, iv, 0 if decrypt else 1) != 1:
            raise RuntimeError("EVP_CipherInit_ex failed")
        lib.EVP_CIPHER_CTX_set_padding(ctx, 0)
        outl = ctypes.c_int(0)
        done = 0
        step = 1 << 28
        while done < src.size:
            n = min(step, src.size - done)
            if lib.EVP_CipherUpdate(ctx, out.ctypes.data + done, ctypes.byref(outl), src.ctypes.data + done, n) != 1:
                raise RuntimeError("EVP_CipherUpdate failed")
            done += outl.value
    finally:
        lib.EVP_CIPHER_CTX_free(ctx)
    return out[: src.size]


def tdes_ecb(k1: bytes, k2: bytes, k3: bytes, data, decrypt: bool = False) -> np.ndarray:
    """OpenSSL EVP_des_ede3_ecb, no padding."""
    return _evp(_load().EVP_des_ede3_ecb(), k1 + k2 + k3, None, data, decrypt)


def tdes_cbc(k1: bytes, k2: bytes, k3: bytes, iv: bytes, data, decrypt: bool = False) -> np.ndarray:
    """OpenSSL EVP_des_ede3_cbc, no padding."""
    return _evp(_load().EVP_des_ede3_cbc(), k1 + k2 + k3, bytes(iv), data, decrypt)


def des_block(key: bytes, block: bytes, decrypt: bool = False) -> bytes:
    """Single DES through OpenSSL's DES_ecb_encrypt."""
    lib = _load()
    ks = ctypes.create_string_buffer(128)
    lib.DES_set_key_unchecked(key, ks)
    out = ctypes.create_string_buffer(8)
    lib.DES_ecb_encrypt(block, out, ks, 0 if decrypt else 1)
    return out.raw
