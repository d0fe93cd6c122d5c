"""Sparse distance-matrix input through the C ABI (vrph_barcode_from_sparse).

A pair that is not given is not an edge. The oracle takes dense matrices
only, so each sparse case is handed to it as the dense matrix with every
missing pair set above the largest given distance and the threshold set to
that largest distance: the same complex, the same filtration order, so the
same pairs bit for bit. The enclosing radius agrees as well: a point with a
missing pair has an infinite row maximum on the GPU side and one above the
threshold on the oracle side, so only complete rows can lower either.
"""
import numpy as np
import pytest

import oracle
from paper_2502_05063_amd import synth

from test_gpu_parity import assert_same, ctx, dev  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def coo_of(D, keep, rng, flip=True):
    """Upper-triangle pairs where keep is True, in a shuffled order, each in a
    random orientation."""
    n = D.shape[0]
    iu, ju = np.triu_indices(n, 1)
    sel = keep[iu, ju]
    r, c = iu[sel], ju[sel]
    v = D[r, c].astype(np.float32)
    if flip:
        sw = rng.random(len(r)) < 0.5
        r, c = np.where(sw, c, r), np.where(sw, r, c)
    perm = rng.permutation(len(r))
    return r[perm].astype(np.int32), c[perm].astype(np.int32), v[perm]


def dense_stand_in(D, keep):
    """The dense matrix and threshold the oracle gets for a sparse matrix."""
    n = D.shape[0]
    off = ~np.eye(n, dtype=bool)
    given = keep & off
    tau = float(D[given].max()) if given.any() else 0.0
    Dp = D.copy()
    Dp[off & ~keep] = np.float32(2 * tau + 1)  # above every given distance
    return Dp, tau


def itensor(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()


def random_keep(n, p, rng):
    k = rng.random((n, n)) < p
    k = np.triu(k, 1)
    return k | k.T


def test_all_pairs_given_equals_dense(ctx):
    rng = np.random.default_rng(7)
    X = synth.uniform_cube(40, 3, seed=7)
    D = oracle.pdist(X)
    keep = ~np.eye(40, dtype=bool)
    r, c, v = coo_of(D, keep, rng)
    got = ctx.barcode_sparse(40, itensor(r), itensor(c), dev(v), max_dim=2, keep_zero=True)
    want = ctx.barcode(D=dev(D), max_dim=2, keep_zero=True)
    assert np.array_equal(got.pairs, want.pairs)


@pytest.mark.parametrize("n,p,max_dim,seed", [(30, 0.5, 2, 1), (60, 0.7, 2, 2), (48, 0.35, 3, 3),
                                                (120, 0.8, 1, 4), (150, 0.6, 2, 5)])
def test_random_sparse_matches_oracle(ctx, n, p, max_dim, seed):
    rng = np.random.default_rng(seed)
    X = synth.uniform_cube(n, 3, seed=seed)
    D = oracle.pdist(X)
    keep = random_keep(n, p, rng)
    r, c, v = coo_of(D, keep, rng)
    Dp, tau = dense_stand_in(D, keep)
    want = oracle.barcode(Dp, max_dim, threshold=tau)
    got = ctx.barcode_sparse(n, itensor(r), itensor(c), dev(v), max_dim=max_dim, keep_zero=True)
    assert_same(got.pairs, want, f"sparse n={n} p={p}")
    if max_dim >= 2:  # the global-memory enumeration gives the same pairs
        got2 = ctx.barcode_sparse(n, itensor(r), itensor(c), dev(v), max_dim=max_dim,
                                  keep_zero=True, lds=False)
        assert np.array_equal(got2.pairs, got.pairs)


def test_threshold_and_complete_rows(ctx):
    """A finite threshold and a point with all its pairs given (its row sets
    the enclosing radius on both sides)."""
    rng = np.random.default_rng(11)
    n = 50
    X = synth.uniform_cube(n, 3, seed=11)
    D = oracle.pdist(X)
    keep = random_keep(n, 0.6, rng)
    keep[0, 1:] = keep[1:, 0] = True
    r, c, v = coo_of(D, keep, rng)
    Dp, tau = dense_stand_in(D, keep)
    for thr in (0.5, float("inf")):
        want = oracle.barcode(Dp, 2, threshold=min(thr, tau))
        got = ctx.barcode_sparse(n, itensor(r), itensor(c), dev(v), max_dim=2, threshold=thr,
                                 keep_zero=True)
        assert_same(got.pairs, want, f"threshold {thr}")


def test_disconnected_graph(ctx):
    """Two triangles and an isolated point: three essential H0 classes, one
    zero-persistence H1 pair per triangle, nothing else."""
    D = np.array([[0, 1, 2, 0, 0, 0, 0],
                  [1, 0, 3, 0, 0, 0, 0],
                  [2, 3, 0, 0, 0, 0, 0],
                  [0, 0, 0, 0, 1.5, 2.5, 0],
                  [0, 0, 0, 1.5, 0, 2, 0],
                  [0, 0, 0, 2.5, 2, 0, 0],
                  [0, 0, 0, 0, 0, 0, 0]], np.float32)
    keep = D > 0
    rng = np.random.default_rng(0)
    r, c, v = coo_of(D, keep, rng)
    bc = ctx.barcode_sparse(7, itensor(r), itensor(c), dev(v), max_dim=1, keep_zero=True)
    h0 = bc.dim(0)
    assert int((h0["essential"] == 1).sum()) == 3
    h1 = bc.dim(1)
    assert len(h1) == 2 and not h1["essential"].any()
    assert np.array_equal(h1["birth_diam"], h1["death_diam"])
    Dp, tau = dense_stand_in(D, keep)
    assert_same(bc.pairs, oracle.barcode(Dp, 1, threshold=tau), "disconnected")


def test_no_entries(ctx):
    import torch

    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    bc = ctx.barcode_sparse(5, e, e, torch.zeros(0, dtype=torch.float32, device="cuda"),
                            max_dim=2, keep_zero=True)
    assert len(bc.pairs) == 5 and bc.pairs["essential"].all()


@pytest.mark.parametrize("case", ["repeat", "repeat_flipped", "out_of_range", "diagonal",
                                  "negative", "nan"])
def test_invalid_entries(ctx, case):
    from paper_2502_05063_amd import vrph

    r = np.array([0, 1, 2], np.int32)
    c = np.array([1, 2, 3], np.int32)
    v = np.array([1.0, 2.0, 3.0], np.float32)
    if case == "repeat":
        r, c, v = np.append(r, 1), np.append(c, 2), np.append(v, 2.0)
    elif case == "repeat_flipped":
        r, c, v = np.append(r, 2), np.append(c, 1), np.append(v, 2.0)
    elif case == "out_of_range":
        c[2] = 9
    elif case == "diagonal":
        c[2] = 2
    elif case == "negative":
        v[1] = -1.0
    elif case == "nan":
        v[1] = np.nan
    with pytest.raises(vrph.VrphError):
        ctx.barcode_sparse(4, itensor(r), itensor(c), dev(v), max_dim=1)
    # the context stays usable
    bc = ctx.barcode_sparse(4, itensor(r[:2]), itensor(np.array([1, 2], np.int32)),
                            dev(np.array([1.0, 2.0], np.float32)), max_dim=1)
    assert len(bc.dim(0)) >= 1
