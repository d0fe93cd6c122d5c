"""Hashed clearing sets and clouds above 2048 points, against the oracle.

Dimension d's cleared columns (Alg. 17) live in a hash set instead of a
bitmap over all C(n, d+1) indices when the bitmap would be too large; the
flag VRPH_HASHED_CLEARING forces that for every dimension >= 2. Clearing
never changes a pair (Prop. 5.3.9, Lemma 4.2.2), so both must give the
oracle's pairs bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2502_05063_amd import synth

from test_gpu_parity import assert_same, ctx, dev  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,n,max_dim,thr", [("sphere", 70, 3, float("inf")),
                                                 ("cube", 120, 2, float("inf")),
                                                 ("cube", 260, 3, 0.35),
                                                 ("o3", 300, 3, 1.6)])
def test_hashed_clearing_matches_oracle(ctx, name, n, max_dim, thr):
    if name == "sphere":
        X = synth.sphere(n, 3, seed=n)
    elif name == "o3":
        X = synth.orthogonal_3x3(n, seed=n)
    else:
        X = synth.uniform_cube(n, 3, seed=n)
    D = oracle.pdist(X)
    want = oracle.barcode(D, max_dim, threshold=thr)
    got = ctx.barcode(X=dev(X), max_dim=max_dim, threshold=thr, keep_zero=True,
                      hashed_clearing=True)
    assert_same(got.pairs, want, f"hashed {name} n={n}")
    plain = ctx.barcode(X=dev(X), max_dim=max_dim, threshold=thr, keep_zero=True)
    assert np.array_equal(plain.pairs, got.pairs)
    assert plain.stats["columns"] == got.stats["columns"]
    if n <= 200:  # the global-memory kernel reads the hashed sets too
        g2 = ctx.barcode(X=dev(X), max_dim=max_dim, threshold=thr, keep_zero=True,
                         hashed_clearing=True, lds=False)
        assert np.array_equal(g2.pairs, got.pairs)


def test_hashed_sparse_input(ctx):
    rng = np.random.default_rng(5)
    n = 90
    X = synth.uniform_cube(n, 3, seed=5)
    D = oracle.pdist(X)
    keep = np.triu(rng.random((n, n)) < 0.7, 1)
    keep = keep | keep.T
    iu, ju = np.nonzero(np.triu(keep, 1))
    import torch

    r = torch.from_numpy(iu.astype(np.int32)).cuda()
    c = torch.from_numpy(ju.astype(np.int32)).cuda()
    v = dev(D[iu, ju])
    tau = float(D[iu, ju].max())
    Dp = D.copy()
    off = ~np.eye(n, dtype=bool)
    Dp[off & ~keep] = np.float32(2 * tau + 1)
    want = oracle.barcode(Dp, 3, threshold=tau)
    got = ctx.barcode_sparse(n, r, c, v, max_dim=3, keep_zero=True, hashed_clearing=True)
    assert_same(got.pairs, want, "hashed sparse")


@pytest.mark.parametrize("n,max_dim,thr", [(3000, 2, 0.06), (4096, 3, 0.04)])
def test_large_cloud_matches_oracle(ctx, n, max_dim, thr):
    """Above the former 2048-point limit; at 4096 points dimension 3's
    bitmap would take 1.5 TB, so its clearing set is hashed by itself."""
    X = synth.uniform_cube(n, 3, seed=n)
    D = oracle.pdist(X)
    want = oracle.barcode(D, max_dim, threshold=thr)
    got = ctx.barcode(X=dev(X), max_dim=max_dim, threshold=thr, keep_zero=True)
    assert_same(got.pairs, want, f"n={n}")
    assert got.stats["candidates"][max_dim] > 0


def test_large_h0_full_threshold(ctx):
    """H0 of 4096 points at the full threshold: the minimum spanning forest
    in filtration order equals Kruskal's on the oracle side."""
    X = synth.uniform_cube(4096, 3, seed=1)
    D = oracle.pdist(X)
    want = np.sort(oracle.h0_kruskal(D), order=["birth", "death"])
    got = ctx.barcode(X=dev(X), max_dim=0, keep_zero=True).dim(0)
    assert_same(np.sort(got, order=["birth", "death"]), want, "H0 of 4096 points")
