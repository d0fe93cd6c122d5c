"""Differentiable persistence: torch.autograd.Function over the HIP library.

The forward computes the barcodes (batched graph or one cloud) and returns
the birth and death values of the finite pairs of one dimension. Each value
is the length of its simplex's diameter edge (u, v), so the backward is the
library's scatter kernel: gX[u] += g (x_u - x_v)/|x_u - x_v|, gX[v] -= same.
The pairing itself is piecewise constant in the points and has no gradient.
"""
from __future__ import annotations

import numpy as np
import torch

from . import vrph


def _finite_pairs(bc, dim, offset):
    p = bc.dim(dim)
    p = p[p["essential"] == 0]
    e = np.concatenate([p["birth_edge"], p["death_edge"]], axis=1).astype(np.int64)
    e = np.where(e >= 0, e + offset, -1)
    return p["birth_diam"], p["death_diam"], e


class _BatchPersistence(torch.autograd.Function):
    @staticmethod
    def forward(fctx, X, batch, dim):
        results = batch.forward(X.detach())
        b, d, e, c = [], [], [], []
        for i, bc in enumerate(results):
            bi, di, ei = _finite_pairs(bc, dim, int(batch.offsets[i]))
            b.append(bi)
            d.append(di)
            e.append(ei)
            c.append(np.full(len(bi), i, np.int64))
        dev = X.device
        births = torch.from_numpy(np.concatenate(b).astype(np.float32)).to(dev)
        deaths = torch.from_numpy(np.concatenate(d).astype(np.float32)).to(dev)
        edges = torch.from_numpy(np.concatenate(e).astype(np.int32).reshape(-1, 4)).to(dev)
        cloud = torch.from_numpy(np.concatenate(c)).to(dev)
        fctx.save_for_backward(X, edges)
        fctx.lib = batch.ctx
        fctx.mark_non_differentiable(cloud)
        return births, deaths, cloud

    @staticmethod
    def backward(fctx, g_birth, g_death, g_cloud):
        X, edges = fctx.saved_tensors
        gX = torch.zeros_like(X)
        if g_birth is None:
            g_birth = torch.zeros(edges.shape[0], device=X.device, dtype=torch.float32)
        if g_death is None:
            g_death = torch.zeros(edges.shape[0], device=X.device, dtype=torch.float32)
        fctx.lib.backward(X.detach(), edges, g_birth.float().contiguous(),
                          g_death.float().contiguous(), gX)
        return gX, None, None


class _CloudPersistence(torch.autograd.Function):
    @staticmethod
    def forward(fctx, X, lib_ctx, dim, max_dim, threshold):
        bc = lib_ctx.barcode(X=X.detach(), max_dim=max_dim, threshold=threshold)
        b, d, e = _finite_pairs(bc, dim, 0)
        dev = X.device
        births = torch.from_numpy(b.astype(np.float32)).to(dev)
        deaths = torch.from_numpy(d.astype(np.float32)).to(dev)
        edges = torch.from_numpy(e.astype(np.int32).reshape(-1, 4)).to(dev)
        fctx.save_for_backward(X, edges)
        fctx.lib = lib_ctx
        return births, deaths

    @staticmethod
    def backward(fctx, g_birth, g_death):
        X, edges = fctx.saved_tensors
        gX = torch.zeros_like(X)
        if g_birth is None:
            g_birth = torch.zeros(edges.shape[0], device=X.device, dtype=torch.float32)
        if g_death is None:
            g_death = torch.zeros(edges.shape[0], device=X.device, dtype=torch.float32)
        fctx.lib.backward(X.detach(), edges, g_birth.float().contiguous(),
                          g_death.float().contiguous(), gX)
        return gX, None, None, None, None


def batch_persistence(X_packed: torch.Tensor, batch: "vrph.Batch", dim: int = 1):
    """(births, deaths, cloud) of the finite dimension-`dim` pairs of every cloud;
    births and deaths are differentiable w.r.t. X_packed."""
    return _BatchPersistence.apply(X_packed, batch, dim)


def cloud_persistence(X: torch.Tensor, lib_ctx: "vrph.Context", dim: int = 1, max_dim: int = 1,
                      threshold: float = float("inf")):
    """(births, deaths) of the finite dimension-`dim` pairs of one cloud."""
    return _CloudPersistence.apply(X, lib_ctx, dim, max_dim, threshold)


class _GraphExtended(torch.autograd.Function):
    @staticmethod
    def forward(fctx, f, lib_ctx, edges, v_off, e_off):
        bars = lib_ctx.graph_extended(f.detach(), edges, v_off, e_off, host=False)
        births = bars[:, 3].contiguous().view(torch.float32)
        deaths = bars[:, 4].contiguous().view(torch.float32)
        kinds = bars[:, 0].contiguous()
        fctx.save_for_backward(bars)
        fctx.lib = lib_ctx
        fctx.offsets = (v_off, e_off)
        fctx.mark_non_differentiable(kinds)
        return births, deaths, kinds

    @staticmethod
    def backward(fctx, g_birth, g_death, g_kind):
        (bars,) = fctx.saved_tensors
        v_off, e_off = fctx.offsets
        g_f = torch.zeros(int(np.asarray(v_off)[-1]), device=bars.device, dtype=torch.float32)
        fctx.lib.graph_extended_backward(
            bars, None if g_birth is None else g_birth.float().contiguous(),
            None if g_death is None else g_death.float().contiguous(), v_off, e_off, g_f)
        return g_f, None, None, None, None


def graph_extended_values(lib_ctx, f, edges, v_off, e_off):
    """Extended persistence of a batch of graphs as a differentiable layer
    (Sec. 7.2; the readouts of Ch. 7): returns the birth and death values of
    every bar (differentiable with respect to the vertex values f, float32
    [V] on the device) and their kinds (vrph.EXT_*), in the bar order of
    vrph_graph_extended. Each value is f at the vertex the bar names, so the
    gradient is the library's scatter onto those vertices."""
    return _GraphExtended.apply(f, lib_ctx, edges, v_off, e_off)

