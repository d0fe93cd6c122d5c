"""The paper's unfused order (VRPH_FULL_SORT: every column written, sorted
into coboundary order, then tested, Alg. 17, 18 and 13) against the fused
path: the same pairs, columns, apparent pairs, reduced columns and
cofacets examined in every dimension, on small clouds with and without ties
and a threshold, and at full size on the 192-point S^3 workload; where the
flag does not apply (every pair reported, the global-memory kernel) the
fused path runs and the results are the same too."""
import numpy as np
import pytest

import oracle
from paper_2502_05063_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2502_05063_amd import vrph

    assert torch.cuda.is_available()
    c = vrph.Context()
    yield c
    c.close()


def same(a, b, dims):
    assert np.array_equal(a.pairs, b.pairs)
    for k in ("columns", "apparent", "reduced", "cofacets"):
        for d in dims:
            assert a.stats[k][d] == b.stats[k][d], (k, d, a.stats[k][d], b.stats[k][d])


@pytest.mark.parametrize("case", ["cube", "sphere", "lattice", "threshold"])
def test_full_sort_matches_fused(ctx, case):
    import torch

    thr = float("inf")
    if case == "cube":
        X = synth.uniform_cube(90, 3, seed=21)
    elif case == "sphere":
        X = synth.sphere(120, 3, seed=22)
    elif case == "lattice":  # many equal distances
        g = np.stack(np.meshgrid(*[np.arange(4)] * 3, indexing="ij"), -1).reshape(-1, 3)
        X = (g * 0.5).astype(np.float32)
    else:
        X = synth.uniform_cube(150, 3, seed=23)
        thr = 0.35
    Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
    fused = ctx.barcode(X=Xd, max_dim=3, threshold=thr)
    unfused = ctx.barcode(X=Xd, max_dim=3, threshold=thr, full_sort=True)
    same(fused, unfused, (2, 3))
    if case == "cube":  # and against the oracle
        ref = oracle.nonzero(oracle.barcode(oracle.pdist(X), 3, thr))
        got = np.empty(len(unfused.pairs), oracle.PAIR_DTYPE)
        for f in oracle.PAIR_DTYPE.names:
            got[f] = unfused.pairs[f]
        assert np.array_equal(got, ref)


def test_full_sort_not_applicable(ctx):
    import torch

    X = torch.from_numpy(synth.sphere(70, 3, seed=24)).cuda()
    for kw in (dict(keep_zero=True), dict(lds=False)):
        a = ctx.barcode(X=X, max_dim=3, **kw)
        b = ctx.barcode(X=X, max_dim=3, full_sort=True, **kw)
        same(a, b, (2, 3))


def test_full_sort_full_size(ctx):
    """The 192-point S^3 workload: 54.9 M candidates in dimension 3, all of
    the surviving 45.5 M columns sorted."""
    import torch

    X = torch.from_numpy(synth.sphere(192, 3, seed=0)).cuda()
    fused = ctx.barcode(X=X, max_dim=3)
    unfused = ctx.barcode(X=X, max_dim=3, full_sort=True)
    same(fused, unfused, (1, 2, 3))
    assert unfused.stats["columns"][3] == 45538709
