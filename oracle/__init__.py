"""Python access to the test-infrastructure oracle (plain scalar C).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are its only users.  The decoder library never imports it.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "polar_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

DTYPE_CODE = {"f32": 0, "i16": 1, "i8": 2}
_NP = {"f32": np.float32, "i16": np.int16, "i8": np.int8}

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "oracle.h"))
    ):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-D_POSIX_C_SOURCE=200809L",
             "-Wall", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm", "-lpthread"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        vp = ctypes.c_void_p
        i64 = ctypes.c_int64
        ci = ctypes.c_int
        u64 = ctypes.c_uint64
        L.orc_crc.argtypes = [u8p, ci, u64, ci, ctypes.POINTER(u64)]
        L.orc_polar_transform.argtypes = [u8p, ci]
        L.orc_select.argtypes = [dp, ci, ci, ip]
        L.orc_decode_tree.argtypes = [ci, ci, u8p, u64, ci, ci, ci, ci, ci, vp, i64, u8p, u8p, dp, u8p, ci]
        L.orc_decode_tree_list.argtypes = [ci, ci, u8p, ci, ci, ci, ci, vp, ip, u8p, dp]
        L.orc_decode_scl.argtypes = [ci, ci, u8p, u64, ci, ci, ci, vp, i64, u8p, u8p, dp, u8p, ci]
        L.orc_decode_ml.argtypes = [ci, ci, u8p, u64, ci, ci, vp, i64, u8p, dp]
        for f in (L.orc_crc, L.orc_polar_transform, L.orc_select, L.orc_decode_tree,
                  L.orc_decode_tree_list, L.orc_decode_scl, L.orc_decode_ml):
            f.restype = ci
        _lib = L
    return _lib


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, what):
    if rc < 0:
        raise ValueError(f"oracle {what}: invalid arguments")
    return rc


def crc(bits, poly: int, r: int) -> int:
    b = np.ascontiguousarray(bits, dtype=np.uint8)
    rem = ctypes.c_uint64(0)
    _check(lib().orc_crc(_u8(b), int(b.size), poly, r, ctypes.byref(rem)), "crc")
    return int(rem.value)


def polar_transform(v) -> np.ndarray:
    x = np.array(v, dtype=np.uint8, copy=True).ravel()
    _check(lib().orc_polar_transform(_u8(x), int(x.size)), "transform")
    return x


def select(pm, L: int) -> np.ndarray:
    p = np.ascontiguousarray(pm, dtype=np.float64)
    keep = np.zeros(max(1, p.size), dtype=np.int32)
    m = _check(lib().orc_select(_dp(p), int(p.size), int(L),
                                keep.ctypes.data_as(ctypes.POINTER(ctypes.c_int))), "select")
    return keep[:m].copy()


def _prep(llr, dtype, N):
    a = np.ascontiguousarray(llr, dtype=_NP[dtype])
    if a.ndim == 1:
        a = a[None, :]
    if a.shape[1] != N:
        raise ValueError("llr rows must have N entries")
    return a


def _threads(threads):
    if threads is None:
        return max(1, min(os.cpu_count() or 1, 16))
    return int(threads)


def decode_tree(N, K, frozen, poly, r, L, llr, dtype="f32", spc_max=4, mode=0, threads=None):
    """Decoder A.  Returns (u_hat[F,K], crc_ok[F], pm[F], near_tie[F])."""
    fz = np.ascontiguousarray(frozen, dtype=np.uint8)
    a = _prep(llr, dtype, N)
    F = a.shape[0]
    u = np.zeros((F, K), np.uint8)
    ok = np.zeros(F, np.uint8)
    pm = np.zeros(F, np.float64)
    nt = np.zeros(F, np.uint8)
    _check(lib().orc_decode_tree(N, K, _u8(fz), poly, r, L, DTYPE_CODE[dtype], spc_max, mode,
                                 a.ctypes.data, F, _u8(u), _u8(ok), _dp(pm), _u8(nt),
                                 _threads(threads)), "decode_tree")
    return u, ok, pm, nt


def decode_tree_list(N, K, frozen, L, llr, dtype="f32", spc_max=4, mode=0):
    """Decoder A on one frame without CRC; returns (codewords[P,N], pm[P])."""
    fz = np.ascontiguousarray(frozen, dtype=np.uint8)
    a = _prep(llr, dtype, N)[0].copy()
    cw = np.zeros((L, N), np.uint8)
    pm = np.zeros(L, np.float64)
    n = ctypes.c_int(0)
    _check(lib().orc_decode_tree_list(N, K, _u8(fz), L, DTYPE_CODE[dtype], spc_max, mode,
                                      a.ctypes.data, ctypes.byref(n), _u8(cw), _dp(pm)),
           "decode_tree_list")
    return cw[: n.value].copy(), pm[: n.value].copy()


def decode_scl(N, K, frozen, poly, r, L, llr, dtype="f32", threads=None):
    """Decoder B.  Returns (u_hat[F,K], crc_ok[F], pm[F], near_tie[F])."""
    fz = np.ascontiguousarray(frozen, dtype=np.uint8)
    a = _prep(llr, dtype, N)
    F = a.shape[0]
    u = np.zeros((F, K), np.uint8)
    ok = np.zeros(F, np.uint8)
    pm = np.zeros(F, np.float64)
    nt = np.zeros(F, np.uint8)
    _check(lib().orc_decode_scl(N, K, _u8(fz), poly, r, L, DTYPE_CODE[dtype], a.ctypes.data, F,
                                _u8(u), _u8(ok), _dp(pm), _u8(nt), _threads(threads)), "decode_scl")
    return u, ok, pm, nt


def decode_ml(N, K, frozen, poly, r, llr, dtype="f32"):
    """Decoder C.  Returns (u_hat[F,K], dist[F])."""
    fz = np.ascontiguousarray(frozen, dtype=np.uint8)
    a = _prep(llr, dtype, N)
    F = a.shape[0]
    u = np.zeros((F, K), np.uint8)
    d = np.zeros(F, np.float64)
    _check(lib().orc_decode_ml(N, K, _u8(fz), poly, r, DTYPE_CODE[dtype], a.ctypes.data, F,
                               _u8(u), _dp(d)), "decode_ml")
    return u, d
