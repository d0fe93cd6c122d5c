"""H0 of large single clouds (the Boruvka row scans spread over the chip,
from 512 points on): the pairs must be Kruskal's over the edges in
filtration order (the oracle's h0_kruskal), with components left apart by a
low threshold, with many tied distances, and on a sparse input whose graph
falls apart.
"""
import numpy as np
import pytest

import oracle
from paper_2502_05063_amd import synth

from test_gpu_parity import assert_same, ctx, dev  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def h0_of(bc):
    return np.sort(bc.dim(0), order=["birth", "death"])


def kruskal(D, thr=float("inf")):
    return np.sort(oracle.h0_kruskal(D, thr), order=["birth", "death"])


@pytest.mark.parametrize("n,thr", [(512, float("inf")), (600, 0.06), (1500, 0.03), (2047, 0.2)])
def test_thresholded_clouds(ctx, n, thr):
    X = synth.uniform_cube(n, 3, seed=n)
    D = oracle.pdist(X)
    got = ctx.barcode(X=dev(X), max_dim=0, threshold=thr, keep_zero=True)
    assert_same(h0_of(got), kruskal(D, thr), f"H0 n={n} thr={thr}")
    if thr < 0.1:
        assert int((got.dim(0)["essential"] == 1).sum()) > 1  # several components


def test_many_ties(ctx):
    D = synth.integer_distances(700, 6, seed=3)
    got = ctx.barcode(D=dev(D), max_dim=0, keep_zero=True)
    assert_same(h0_of(got), kruskal(D), "H0 with ties")


def test_sparse_disconnected(ctx):
    import torch

    rng = np.random.default_rng(9)
    n = 800
    X = synth.uniform_cube(n, 3, seed=9)
    D = oracle.pdist(X)
    keep = np.triu(D < 0.08, 1) & (rng.random((n, n)) < 0.7)
    iu, ju = np.nonzero(keep)
    r = torch.from_numpy(iu.astype(np.int32)).cuda()
    c = torch.from_numpy(ju.astype(np.int32)).cuda()
    got = ctx.barcode_sparse(n, r, c, dev(D[iu, ju]), max_dim=0, keep_zero=True)
    tau = float(D[iu, ju].max())
    Dp = D.copy()
    off = ~np.eye(n, dtype=bool)
    sym = keep | keep.T
    Dp[off & ~sym] = np.float32(2 * tau + 1)
    assert_same(h0_of(got), kruskal(Dp, tau), "sparse H0")
    assert int((got.dim(0)["essential"] == 1).sum()) > 1
