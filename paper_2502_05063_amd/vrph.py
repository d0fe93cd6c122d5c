"""Python binding of libvrph.so (include/vrph.h): argument marshalling only.

Every step of the computation runs in the HIP library. PyTorch supplies
device memory and the current stream. If the library is missing the import
fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvrph.so")

OK, EINVAL, ENOMEM, EOVERFLOW, EDEVICE, ESTATE = 0, -1, -2, -3, -4, -5
KEEP_ZERO_PERSISTENCE = 1
NO_ENCLOSING_RADIUS = 2
AUTOTUNE = 4
NO_LDS = 8
HASHED_CLEARING = 16
BOUNDARY_NO_CLEARING = 32
BOUNDARY_NO_COMPRESSION = 64
HOST_REDUCTION = 128
DEVICE_REDUCTION = 512
FULL_SORT = 256
EXT_ORD0, EXT_REL1, EXT_EXT0, EXT_EXT1 = 0, 1, 2, 3
EXT_BAR_DTYPE = np.dtype([("kind", "<i4"), ("birth", "<i4"), ("death", "<i4"),
                          ("birth_value", "<f4"), ("death_value", "<f4"),
                          ("birth_vertex", "<i4"), ("death_vertex", "<i4")])
MAX_DIM = 6

PAIR_DTYPE = np.dtype(
    [
        ("dim", "<i4"),
        ("essential", "<i4"),
        ("birth", "<u8"),
        ("death", "<u8"),
        ("birth_diam", "<f4"),
        ("death_diam", "<f4"),
        ("birth_edge", "<i4", (2,)),
        ("death_edge", "<i4", (2,)),
    ]
)
assert PAIR_DTYPE.itemsize == 48


class Stats(ctypes.Structure):
    _fields_ = [
        ("candidates", ctypes.c_int64 * (MAX_DIM + 1)),
        ("columns", ctypes.c_int64 * (MAX_DIM + 1)),
        ("apparent", ctypes.c_int64 * (MAX_DIM + 1)),
        ("reduced", ctypes.c_int64 * (MAX_DIM + 1)),
        ("additions", ctypes.c_int64 * (MAX_DIM + 1)),
        ("pairs", ctypes.c_int64 * (MAX_DIM + 1)),
        ("cofacets", ctypes.c_int64 * (MAX_DIM + 1)),
        ("facets", ctypes.c_int64 * (MAX_DIM + 1)),
        ("emergent", ctypes.c_int64 * (MAX_DIM + 1)),
        ("gpu_ms", ctypes.c_double * (MAX_DIM + 1)),
        ("apparent_ms", ctypes.c_double * (MAX_DIM + 1)),
        ("host_ms", ctypes.c_double * (MAX_DIM + 1)),
        ("grid", ctypes.c_int32 * (MAX_DIM + 1)),
        ("device_reduced", ctypes.c_int32),
        ("tau_eff", ctypes.c_float),
        ("max_dim", ctypes.c_int32),
        ("total_ms", ctypes.c_double),
    ]

    def to_dict(self):
        k = self.max_dim + 1
        out = {f: list(getattr(self, f))[:k] for f, t in self._fields_
               if issubclass(t, ctypes.Array)}
        out.update(tau_eff=self.tau_eff, max_dim=self.max_dim, total_ms=self.total_ms,
                   device_reduced=self.device_reduced)
        return out


class BoundaryStats(ctypes.Structure):
    _fields_ = [("columns", ctypes.c_int64), ("zero", ctypes.c_int64), ("stable", ctypes.c_int64),
                ("scan_pivots", ctypes.c_int64), ("unstable", ctypes.c_int64),
                ("additions", ctypes.c_int64), ("compress_additions", ctypes.c_int64),
                ("compressed", ctypes.c_int64), ("scan_ms", ctypes.c_double),
                ("host_ms", ctypes.c_double)]

    def to_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class VrphError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"vrph status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2502_05063_amd.build_lib`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_float
    P = ctypes.POINTER
    sig = {
        "vrph_create": (i32, [ctypes.c_int, P(vp)]),
        "vrph_destroy": (None, [vp]),
        "vrph_last_error": (ctypes.c_char_p, []),
        "vrph_pdist": (i32, [vp, vp, i64, i32, vp, vp]),
        "vrph_barcode_from_dist": (i32, [vp, vp, i64, i32, f32, u32, vp, P(vp)]),
        "vrph_barcode_from_points": (i32, [vp, vp, i64, i32, i32, f32, u32, vp, P(vp)]),
        "vrph_barcode_from_sparse": (i32, [vp, i64, i64, vp, vp, vp, i32, f32, u32, vp, P(vp)]),
        "vrph_barcode_count": (i64, [vp, i32]),
        "vrph_barcode_pairs": (vp, [vp, i32]),
        "vrph_barcode_stats": (P(Stats), [vp]),
        "vrph_barcode_free": (None, [vp]),
        "vrph_batch_plan": (i32, [vp, vp, i32, i32, i32, f32, u32, P(vp)]),
        "vrph_batch_forward": (i32, [vp, vp, vp]),
        "vrph_batch_result": (i32, [vp, i32, P(vp)]),
        "vrph_batch_destroy": (None, [vp]),
        "vrph_backward": (i32, [vp, vp, i64, i32, vp, i64, vp, vp, vp, vp]),
        "vrph_backward_noalloc": (i32, [vp, vp, i64, i32, vp, i64, vp, vp, vp, vp]),
        "vrph_boundary_pivots": (i32, [vp, i64, vp, vp, u32, vp, vp, P(BoundaryStats)]),
        "vrph_graph_extended": (i32, [vp, i32, vp, vp, vp, vp, vp, vp]),
        "vrph_graph_extended_backward": (i32, [vp, i32, vp, vp, vp, vp, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status):
    if status != OK:
        raise VrphError(status, lib().vrph_last_error().decode(errors="replace"))


def _stream_ptr():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Barcode:
    """Host copy of a result: `pairs` (PAIR_DTYPE records, canonical order) and `stats`."""

    def __init__(self, handle, owned=True):
        L = lib()
        cnt = L.vrph_barcode_count(handle, -1)
        self.pairs = np.empty(cnt, PAIR_DTYPE)
        if cnt:
            ctypes.memmove(self.pairs.ctypes.data, L.vrph_barcode_pairs(handle, -1),
                           cnt * PAIR_DTYPE.itemsize)
        self.stats = L.vrph_barcode_stats(handle).contents.to_dict()
        if owned:
            L.vrph_barcode_free(handle)

    def dim(self, d):
        return self.pairs[self.pairs["dim"] == d]


class Context:
    """A library context on the current torch CUDA device."""

    def __init__(self, device=None):
        import torch

        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = ctypes.c_void_p()
        _check(lib().vrph_create(self.device, ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().vrph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _f32(t):
        import torch

        if not t.is_cuda or t.dtype != torch.float32:
            raise ValueError("expected a float32 CUDA tensor")
        return t.contiguous()

    def pdist(self, X):
        import torch

        X = self._f32(X)
        n, m = X.shape
        D = torch.empty((n, n), dtype=torch.float32, device=X.device)
        _check(lib().vrph_pdist(self.h, _dev_ptr(X), n, m, _dev_ptr(D), _stream_ptr()))
        return D

    def barcode(self, *, X=None, D=None, max_dim=1, threshold=float("inf"), keep_zero=False,
                no_enclosing=False, autotune=False, lds=True, hashed_clearing=False,
                full_sort=False):
        flags = ((KEEP_ZERO_PERSISTENCE if keep_zero else 0) | (NO_ENCLOSING_RADIUS if no_enclosing else 0)
                 | (AUTOTUNE if autotune else 0) | (0 if lds else NO_LDS)
                 | (HASHED_CLEARING if hashed_clearing else 0) | (FULL_SORT if full_sort else 0))
        out = ctypes.c_void_p()
        if X is not None:
            X = self._f32(X)
            n, m = X.shape
            _check(lib().vrph_barcode_from_points(self.h, _dev_ptr(X), n, m, max_dim, threshold,
                                                  flags, _stream_ptr(), ctypes.byref(out)))
        else:
            D = self._f32(D)
            _check(lib().vrph_barcode_from_dist(self.h, _dev_ptr(D), D.shape[0], max_dim,
                                                threshold, flags, _stream_ptr(), ctypes.byref(out)))
        return Barcode(out)

    def barcode_sparse(self, n, row, col, val, *, max_dim=1, threshold=float("inf"),
                       keep_zero=False, no_enclosing=False, autotune=False, lds=True,
                       hashed_clearing=False):
        """Barcode of a sparse distance matrix: entries (row[k], col[k], val[k]) on the
        device (int32, int32, float32); pairs not given are not edges."""
        import torch

        flags = ((KEEP_ZERO_PERSISTENCE if keep_zero else 0) | (NO_ENCLOSING_RADIUS if no_enclosing else 0)
                 | (AUTOTUNE if autotune else 0) | (0 if lds else NO_LDS)
                 | (HASHED_CLEARING if hashed_clearing else 0))
        for t, dt in ((row, torch.int32), (col, torch.int32), (val, torch.float32)):
            if not t.is_cuda or t.dtype != dt or t.dim() != 1:
                raise ValueError("row, col: 1-D int32 CUDA tensors; val: 1-D float32 CUDA tensor")
        if not (row.numel() == col.numel() == val.numel()):
            raise ValueError("row, col and val must have the same length")
        row, col, val = row.contiguous(), col.contiguous(), val.contiguous()
        out = ctypes.c_void_p()
        _check(lib().vrph_barcode_from_sparse(self.h, n, row.numel(), _dev_ptr(row), _dev_ptr(col),
                                              _dev_ptr(val), max_dim, threshold, flags,
                                              _stream_ptr(), ctypes.byref(out)))
        return Barcode(out)

    def boundary_pivots(self, col_ptr, rows, *, clearing=True, compression=True):
        """Pivots low(R_j) of Alg. 2 for an explicit boundary matrix in CSC form
        (col_ptr, rows: 1-D int64 CUDA tensors; rows strictly increasing within a
        column and below it). Returns (low: int64 numpy array, -1 for a zero
        column, stats dict)."""
        import torch

        for t in (col_ptr, rows):
            if not t.is_cuda or t.dtype != torch.int64 or t.dim() != 1:
                raise ValueError("col_ptr and rows must be 1-D int64 CUDA tensors")
        if col_ptr.numel() < 1:
            raise ValueError("col_ptr needs ncols + 1 entries")
        col_ptr, rows = col_ptr.contiguous(), rows.contiguous()
        ncols = col_ptr.numel() - 1
        if int(col_ptr[-1]) > rows.numel():
            raise ValueError("col_ptr[-1] is past the end of rows")
        low = np.empty(max(ncols, 1), np.int64)
        st = BoundaryStats()
        _check(lib().vrph_boundary_pivots(self.h, ncols, _dev_ptr(col_ptr),
                                          _dev_ptr(rows) if rows.numel() else None,
                                          (0 if clearing else BOUNDARY_NO_CLEARING)
                                          | (0 if compression else BOUNDARY_NO_COMPRESSION),
                                          _stream_ptr(),
                                          low.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st)))
        return low[:ncols], st.to_dict()

    def backward(self, X, edges, g_birth, g_death, gX):
        """gX += scatter of g_birth/g_death onto the diameter edges (edges: int32 [npairs, 4])."""
        import torch

        X = self._f32(X)
        edges = edges.to(torch.int32).contiguous()
        g_birth, g_death = self._f32(g_birth), self._f32(g_death)
        if not gX.is_contiguous():
            raise ValueError("gX must be contiguous")
        _check(lib().vrph_backward(self.h, _dev_ptr(X), X.shape[0], X.shape[1], _dev_ptr(edges),
                                   edges.shape[0], _dev_ptr(g_birth), _dev_ptr(g_death),
                                   _dev_ptr(gX), _stream_ptr()))
        return gX

    def backward_noalloc(self, X, edges, g_birth, g_death, gX):
        """The same as backward through vrph_backward_noalloc: no device memory is
        allocated, so the arguments are taken as they are (float32 X, g_birth,
        g_death, gX; int32 edges [npairs, 4]; all contiguous on the device)."""
        import torch

        for name, t, dt in (("X", X, torch.float32), ("edges", edges, torch.int32),
                            ("g_birth", g_birth, torch.float32),
                            ("g_death", g_death, torch.float32), ("gX", gX, torch.float32)):
            if t.dtype != dt or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{name} must be a contiguous {dt} device tensor")
        _check(lib().vrph_backward_noalloc(self.h, _dev_ptr(X), X.shape[0], X.shape[1],
                                           _dev_ptr(edges), edges.shape[0], _dev_ptr(g_birth),
                                           _dev_ptr(g_death), _dev_ptr(gX), _stream_ptr()))
        return gX

    def graph_extended(self, f, edges, v_off, e_off, host=True):
        """Extended persistence of a batch of graphs (vrph_graph_extended):
        f float32 [V] and edges int32 [E, 2] (endpoints numbered within their
        graph) on the device, v_off / e_off the count + 1 offsets. Returns the
        device int32 tensor of bars ([V + E, 7], vrph_ext_bar records) and,
        with host=True, a list of EXT_BAR_DTYPE arrays, one per graph."""
        import torch

        f = self._f32(f)
        edges = edges.to(torch.int32).contiguous()
        v_off = np.ascontiguousarray(v_off, dtype=np.int64)
        e_off = np.ascontiguousarray(e_off, dtype=np.int64)
        count = len(v_off) - 1
        bars = torch.empty((int(v_off[-1] + e_off[-1]), 7), dtype=torch.int32, device=f.device)
        _check(lib().vrph_graph_extended(self.h, count, v_off.ctypes.data_as(ctypes.c_void_p),
                                         e_off.ctypes.data_as(ctypes.c_void_p), _dev_ptr(f),
                                         _dev_ptr(edges), _dev_ptr(bars), _stream_ptr()))
        if not host:
            return bars
        rec = bars.cpu().numpy().reshape(-1).view(EXT_BAR_DTYPE)
        start = v_off + e_off
        return bars, [rec[start[g]:start[g + 1]] for g in range(count)]

    def graph_extended_backward(self, bars, g_birth, g_death, v_off, e_off, g_f):
        """vrph_graph_extended_backward: adds g_birth / g_death (float32, one
        per bar, device; None for zero) to g_f (float32 [V], device) at the
        vertices the bars (the int32 [V + E, 7] tensor of graph_extended) name."""
        v_off = np.ascontiguousarray(v_off, dtype=np.int64)
        e_off = np.ascontiguousarray(e_off, dtype=np.int64)
        gb = None if g_birth is None else self._f32(g_birth)
        gd = None if g_death is None else self._f32(g_death)
        _check(lib().vrph_graph_extended_backward(
            self.h, len(v_off) - 1, v_off.ctypes.data_as(ctypes.c_void_p),
            e_off.ctypes.data_as(ctypes.c_void_p), _dev_ptr(bars.contiguous()),
            None if gb is None else _dev_ptr(gb), None if gd is None else _dev_ptr(gd),
            _dev_ptr(g_f), _stream_ptr()))

    def batch(self, sizes, m, max_dim=1, threshold=float("inf"), keep_zero=False,
              no_enclosing=False, host_reduction=False, autotune=False, device_reduction=False):
        return Batch(self, sizes, m, max_dim, threshold, keep_zero, no_enclosing, host_reduction,
                     autotune, device_reduction)


class Batch:
    """A batch plan: fixed cloud sizes, one captured graph replayed per forward."""

    def __init__(self, ctx, sizes, m, max_dim, threshold, keep_zero, no_enclosing,
                 host_reduction=False, autotune=False, device_reduction=False):
        self.ctx = ctx
        self.sizes = np.ascontiguousarray(sizes, dtype=np.int64)
        flags = ((KEEP_ZERO_PERSISTENCE if keep_zero else 0)
                 | (NO_ENCLOSING_RADIUS if no_enclosing else 0)
                 | (HOST_REDUCTION if host_reduction else 0)
                 | (DEVICE_REDUCTION if device_reduction else 0)
                 | (AUTOTUNE if autotune else 0))
        h = ctypes.c_void_p()
        _check(lib().vrph_batch_plan(ctx.h, self.sizes.ctypes.data_as(ctypes.c_void_p),
                                     len(self.sizes), m, max_dim, threshold, flags,
                                     ctypes.byref(h)))
        self.h = h
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)])

    def forward(self, X_packed):
        X_packed = Context._f32(X_packed)
        _check(lib().vrph_batch_forward(self.h, _dev_ptr(X_packed), _stream_ptr()))
        out = []
        for i in range(len(self.sizes)):
            v = ctypes.c_void_p()
            _check(lib().vrph_batch_result(self.h, i, ctypes.byref(v)))
            out.append(Barcode(v, owned=False))
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().vrph_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
