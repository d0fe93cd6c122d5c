"""ctypes wrapper of the plain CPU oracle (vr_oracle.c).

TEST INFRASTRUCTURE ONLY: the product path (the HIP library and its binding)
never imports this package. Only tests, the smoke check and the CPU-baseline
leg of the benchmark may use it. See vr_oracle.h for what it computes and the
paper passages each function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvroracle.so")
SRC = os.path.join(HERE, "vr_oracle.c")

M1_BOUNDARY, M1_COBOUNDARY, M2_STREAMED, M3_REDUCTION_MATRIX = 0, 1, 2, 3
FLAG_NO_ENCLOSING, FLAG_NO_CLEARING = 1, 2

PAIR_DTYPE = np.dtype(
    [
        ("dim", "<i4"),
        ("essential", "<i4"),
        ("birth", "<u8"),
        ("death", "<u8"),
        ("birth_diam", "<f4"),
        ("death_diam", "<f4"),
    ]
)
assert PAIR_DTYPE.itemsize == 32


def build(force: bool = True) -> str:
    """Compile libvroracle.so with gcc (no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = [
            "gcc", "-std=c11", "-O2", "-Wall", "-ffp-contract=off", "-fPIC", "-shared",
            "-o", LIB_PATH, SRC, "-lm",
        ]
        subprocess.check_call(cmd)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        f32p, u64p, i64p = P(ctypes.c_float), P(ctypes.c_uint64), P(ctypes.c_int64)
        L.orc_pdist.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, f32p]
        L.orc_enclosing_radius.argtypes = [f32p, ctypes.c_int64]
        L.orc_enclosing_radius.restype = ctypes.c_float
        L.orc_binomial.argtypes = [ctypes.c_int64, ctypes.c_int32]
        L.orc_binomial.restype = ctypes.c_uint64
        L.orc_barcode.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float,
                                  ctypes.c_int32, ctypes.c_uint32, P(ctypes.c_void_p)]
        L.orc_result_count.argtypes = [ctypes.c_void_p]
        L.orc_result_count.restype = ctypes.c_int64
        L.orc_result_pairs.argtypes = [ctypes.c_void_p]
        L.orc_result_pairs.restype = ctypes.c_void_p
        L.orc_result_columns.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.orc_result_columns.restype = ctypes.c_int64
        L.orc_result_free.argtypes = [ctypes.c_void_p]
        L.orc_reduce_explicit.argtypes = [ctypes.c_int32, i64p, i64p, i64p]
        L.orc_apparent_pairs.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float,
                                         ctypes.c_uint32, u64p, u64p, ctypes.c_int64, i64p]
        L.orc_is_apparent.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                      ctypes.c_float, ctypes.c_uint32, u64p]
        L.orc_h0_kruskal.argtypes = [f32p, ctypes.c_int64, ctypes.c_float, ctypes.c_uint32,
                                     ctypes.c_void_p, ctypes.c_int64, i64p]
        L.orc_diameter_edge.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                        P(ctypes.c_int32), P(ctypes.c_int32)]
        L.orc_gradient.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, f32p, ctypes.c_void_p,
                                   ctypes.c_int64, f32p, f32p, P(ctypes.c_double)]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _check(rc):
    if rc != 0:
        raise OracleError(f"oracle status {rc}")


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def pdist(X) -> np.ndarray:
    X = _f32(X)
    n, m = X.shape
    D = np.empty((n, n), np.float32)
    _check(lib().orc_pdist(_ptr(X, ctypes.c_float), n, m, _ptr(D, ctypes.c_float)))
    return D


def enclosing_radius(D) -> float:
    D = _f32(D)
    return float(lib().orc_enclosing_radius(_ptr(D, ctypes.c_float), D.shape[0]))


def binomial(v: int, k: int) -> int:
    return int(lib().orc_binomial(v, k))


def barcode(D, max_dim: int, threshold: float = float("inf"), mode: int = M2_STREAMED,
            flags: int = 0, with_columns: bool = False):
    """All persistence pairs of dimensions 0..max_dim, canonical order."""
    D = _f32(D)
    res = ctypes.c_void_p()
    L = lib()
    _check(L.orc_barcode(_ptr(D, ctypes.c_float), D.shape[0], max_dim, threshold, mode, flags,
                         ctypes.byref(res)))
    try:
        cnt = L.orc_result_count(res)
        out = np.empty(cnt, PAIR_DTYPE)
        if cnt:
            ctypes.memmove(out.ctypes.data, L.orc_result_pairs(res), cnt * PAIR_DTYPE.itemsize)
        cols = [int(L.orc_result_columns(res, q)) for q in range(max_dim + 1)]
    finally:
        L.orc_result_free(res)
    return (out, cols) if with_columns else out


def reduce_explicit(columns):
    """Alg. 2 over Z/2; columns: list of row-index lists. Returns lows (-1 = zero)."""
    ptr = np.zeros(len(columns) + 1, np.int64)
    rows = []
    for j, c in enumerate(columns):
        rows.extend(c)
        ptr[j + 1] = len(rows)
    rows = np.asarray(rows if rows else [0], np.int64)
    low = np.empty(max(len(columns), 1), np.int64)
    _check(lib().orc_reduce_explicit(len(columns), _ptr(ptr, ctypes.c_int64),
                                     _ptr(rows, ctypes.c_int64), _ptr(low, ctypes.c_int64)))
    return low[: len(columns)]


def apparent_pairs(D, dim: int, threshold: float = float("inf"), flags: int = 0):
    """Def. 5.3.4 on the explicit coboundary matrix. Returns (s, t) arrays."""
    D = _f32(D)
    cnt = ctypes.c_int64()
    L = lib()
    _check(L.orc_apparent_pairs(_ptr(D, ctypes.c_float), D.shape[0], dim, threshold, flags,
                                None, None, 0, ctypes.byref(cnt)))
    s = np.empty(max(cnt.value, 1), np.uint64)
    t = np.empty(max(cnt.value, 1), np.uint64)
    _check(L.orc_apparent_pairs(_ptr(D, ctypes.c_float), D.shape[0], dim, threshold, flags,
                                _ptr(s, ctypes.c_uint64), _ptr(t, ctypes.c_uint64), cnt.value,
                                ctypes.byref(cnt)))
    return s[: cnt.value], t[: cnt.value]


def is_apparent(D, dim: int, s: int, threshold: float = float("inf"), flags: int = 0):
    """Def. 5.3.4 for one column; returns the cofacet t or None."""
    D = _f32(D)
    t = ctypes.c_uint64()
    rc = lib().orc_is_apparent(_ptr(D, ctypes.c_float), D.shape[0], dim, s, threshold, flags,
                               ctypes.byref(t))
    if rc < 0:
        raise OracleError(f"oracle status {rc}")
    return int(t.value) if rc == 1 else None


def h0_kruskal(D, threshold: float = float("inf"), flags: int = 0):
    D = _f32(D)
    n = D.shape[0]
    out = np.empty(max(n, 1), PAIR_DTYPE)
    cnt = ctypes.c_int64()
    _check(lib().orc_h0_kruskal(_ptr(D, ctypes.c_float), n, threshold, flags,
                                out.ctypes.data, n, ctypes.byref(cnt)))
    return out[: cnt.value]


def diameter_edge(D, dim: int, cidx: int):
    D = _f32(D)
    u, v = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().orc_diameter_edge(_ptr(D, ctypes.c_float), D.shape[0], dim, cidx,
                                   ctypes.byref(u), ctypes.byref(v)))
    return u.value, v.value


def gradient(X, D, pairs, g_birth, g_death) -> np.ndarray:
    X, D = _f32(X), _f32(D)
    pairs = np.ascontiguousarray(pairs, PAIR_DTYPE)
    gb, gd = _f32(g_birth), _f32(g_death)
    n, m = X.shape
    gX = np.empty((n, m), np.float64)
    _check(lib().orc_gradient(_ptr(X, ctypes.c_float), n, m, _ptr(D, ctypes.c_float),
                              pairs.ctypes.data, len(pairs), _ptr(gb, ctypes.c_float),
                              _ptr(gd, ctypes.c_float), _ptr(gX, ctypes.c_double)))
    return gX


def nonzero(pairs):
    """Pairs with birth diameter != death diameter (essential ones included)."""
    return pairs[pairs["birth_diam"] != pairs["death_diam"]]
