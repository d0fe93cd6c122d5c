"""GPU path vs the CPU oracle, through the C ABI, element by element.

Barcodes must match bit-exactly (indices and float32 diameters) given the
same float32 distance matrix; distances from points must match the oracle's
distances bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2502_05063_amd import synth

pytestmark = pytest.mark.gpu
INF = float("inf")


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2502_05063_amd import vrph

    assert torch.cuda.is_available()
    c = vrph.Context()
    yield c
    c.close()


def dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def strip(pairs):
    """GPU records -> the oracle's 32-byte records."""
    out = np.empty(len(pairs), oracle.PAIR_DTYPE)
    for f in oracle.PAIR_DTYPE.names:
        out[f] = pairs[f]
    return out


def assert_same(gpu_pairs, orc_pairs, ctx_msg=""):
    g = strip(gpu_pairs)
    if len(g) != len(orc_pairs) or not np.array_equal(g, orc_pairs):
        gs = set(map(tuple, g.tolist()))
        os_ = set(map(tuple, orc_pairs.tolist()))
        raise AssertionError(f"{ctx_msg}: {len(g)} vs {len(orc_pairs)} pairs; "
                             f"gpu-only {sorted(gs - os_)[:5]} oracle-only {sorted(os_ - gs)[:5]}")


# ---------------------------------------------------------------------------
# distances


@pytest.mark.parametrize("n,m,scale", [(64, 3, 1.0), (192, 4, 1.0), (1024, 9, 1.0), (200, 3, 1e-3),
                                        (200, 5, 1e3), (1, 3, 1.0), (67, 1, 1.0)])
def test_pdist_bitexact(ctx, n, m, scale):
    rng = np.random.default_rng(n * 31 + m)
    X = (rng.standard_normal((n, m)) * scale).astype(np.float32)
    D = ctx.pdist(dev(X)).cpu().numpy()
    assert np.array_equal(D.view(np.uint32), oracle.pdist(X).view(np.uint32))


# ---------------------------------------------------------------------------
# full barcodes at oracle-friendly sizes


def test_c1_cube64_full_list(ctx):
    X = synth.uniform_cube(64, 3, seed=0)
    bc = ctx.barcode(X=dev(X), max_dim=1, keep_zero=True)
    ref = oracle.barcode(oracle.pdist(X), 1)
    assert_same(bc.pairs, ref, "c1 keep_zero")
    bc2 = ctx.barcode(X=dev(X), max_dim=1)
    assert_same(bc2.pairs, oracle.nonzero(ref), "c1 nonzero")
    s = bc.stats
    assert s["columns"][1] == sum(1 for p in ref if p["dim"] == 1)


@pytest.mark.parametrize("seed", range(12))
def test_random_sweep(ctx, seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(4, 48))
    max_dim = int(rng.integers(1, 4)) if n <= 24 else int(rng.integers(1, 3))
    kind = seed % 4
    if kind == 0:
        D = oracle.pdist(rng.random((n, 3)).astype(np.float32))
    elif kind == 1:
        D = synth.integer_distances(n, 4, seed)
    elif kind == 2:
        D = synth.permutation_distances(n, seed)
    else:
        D = oracle.pdist(synth.sphere(n, 2, seed))
    thr = [INF, float(np.quantile(D[D > 0], 0.7))][seed % 2]
    flags = [0, oracle.FLAG_NO_ENCLOSING][(seed // 2) % 2]
    ref = oracle.barcode(D, max_dim, thr, flags=flags)
    bc = ctx.barcode(D=dev(D), max_dim=max_dim, threshold=thr, keep_zero=True,
                     no_enclosing=bool(flags))
    assert_same(bc.pairs, ref, f"seed {seed} n {n} d {max_dim}")


@pytest.mark.parametrize("seed", range(6))
def test_lds_and_global_kernels_agree(ctx, seed):
    """The rank-matrix (LDS) and weight-matrix (global) enumeration kernels
    give the same pairs, and both the oracle's; sizes straddle the LDS limit."""
    rng = np.random.default_rng(500 + seed)
    n = [12, 47, 64, 130, 199, 200][seed]
    md = 3 if n <= 64 else 2
    X = [synth.uniform_cube, synth.sphere][seed % 2](n, 3, seed=seed)
    D = oracle.pdist(X)
    thr = [INF, float(np.quantile(D[D > 0], 0.6))][seed % 3 == 2]
    a = ctx.barcode(D=dev(D), max_dim=md, threshold=thr, keep_zero=True)
    b = ctx.barcode(D=dev(D), max_dim=md, threshold=thr, keep_zero=True, lds=False)
    assert np.array_equal(a.pairs, b.pairs)
    if n <= 64 or md <= 2:
        assert_same(a.pairs, oracle.barcode(D, md, thr), f"n {n}")


def test_ragged_tile_sizes(ctx):
    """Sizes that leave ragged tails in every kernel's launch."""
    for n in (2, 3, 65, 129):
        X = synth.uniform_cube(n, 3, seed=n)
        D = oracle.pdist(X)
        md = 2 if n < 100 else 1
        ref = oracle.barcode(D, md)
        bc = ctx.barcode(D=dev(D), max_dim=md, keep_zero=True)
        assert_same(bc.pairs, ref, f"n {n}")


def test_degenerate_inputs(ctx):
    """Edge cases the method has: one point, max_dim beyond the complex,
    threshold 0, a threshold equal to an edge length (inclusive, Eq. 5.3),
    duplicate points (zero off-diagonal distances) and no edge below the
    threshold; every one against the oracle, all pairs included."""
    cases = []
    cases.append((oracle.pdist(np.zeros((1, 3), np.float32)), 2, INF))
    X = synth.uniform_cube(5, 3, seed=7)
    cases.append((oracle.pdist(X), 4, INF))
    cases.append((oracle.pdist(X), 2, 0.0))
    D = oracle.pdist(synth.uniform_cube(20, 3, seed=8))
    edge = float(np.sort(D[np.triu_indices(20, 1)])[60])
    cases.append((D, 2, edge))
    Xd = synth.uniform_cube(12, 3, seed=9)
    Xd[6:] = Xd[:6]  # every point twice
    cases.append((oracle.pdist(Xd), 2, INF))
    cases.append((oracle.pdist(synth.uniform_cube(15, 3, seed=10)), 2,
                  float(np.min(oracle.pdist(synth.uniform_cube(15, 3, seed=10))[np.triu_indices(15, 1)])) / 2))
    for i, (D, md, thr) in enumerate(cases):
        ref = oracle.barcode(D, md, thr)
        bc = ctx.barcode(D=dev(D), max_dim=md, threshold=thr, keep_zero=True)
        assert_same(bc.pairs, ref, f"case {i}")
        if md >= 2:
            assert_same(ctx.barcode(D=dev(D), max_dim=md, threshold=thr, keep_zero=True,
                                    lds=False).pairs, ref, f"case {i} global")


def test_all_equal_distances_thm_5_4_2(ctx):
    for n0, d in ((9, 1), (9, 2), (8, 3)):
        D = np.ones((n0, n0), np.float32) - np.eye(n0, dtype=np.float32)
        bc = ctx.barcode(D=dev(D), max_dim=d, keep_zero=True)
        assert bc.stats["apparent"][d] == __import__("math").comb(n0 - 1, d + 1)
        assert_same(bc.pairs, oracle.barcode(D, d), f"equal {n0} {d}")


def test_diameter_edges(ctx):
    X = synth.uniform_cube(40, 3, seed=5)
    D = oracle.pdist(X)
    bc = ctx.barcode(D=dev(D), max_dim=2, keep_zero=True)
    for p in bc.pairs[::7]:
        if p["dim"] >= 1:
            assert tuple(p["birth_edge"]) == oracle.diameter_edge(D, int(p["dim"]), int(p["birth"]))
        if not p["essential"]:
            assert tuple(p["death_edge"]) == oracle.diameter_edge(D, int(p["dim"]) + 1, int(p["death"]))


def test_apparent_count_matches_definition(ctx):
    X = synth.sphere(30, 2, seed=3)
    D = oracle.pdist(X)
    bc = ctx.barcode(D=dev(D), max_dim=2, keep_zero=True)
    for d in (1, 2):
        s, _ = oracle.apparent_pairs(D, d)
        assert bc.stats["apparent"][d] == len(s)


def test_deterministic(ctx):
    X = synth.sphere(60, 3, seed=1)
    a = ctx.barcode(X=dev(X), max_dim=2, keep_zero=True).pairs
    for _ in range(3):
        assert np.array_equal(a, ctx.barcode(X=dev(X), max_dim=2, keep_zero=True).pairs)


# ---------------------------------------------------------------------------
# error paths (forced from the host)


def test_invalid_inputs_are_rejected(ctx):
    from paper_2502_05063_amd import vrph

    D = oracle.pdist(synth.uniform_cube(10, 3, 0))
    bad = []
    x = D.copy(); x[1, 2] = np.nan; bad.append(x)
    x = D.copy(); x[1, 2] += 1; bad.append(x)
    x = D.copy(); x[3, 3] = 1; bad.append(x)
    x = D.copy(); x[1, 2] = x[2, 1] = -1; bad.append(x)
    for B in bad:
        with pytest.raises(vrph.VrphError) as e:
            ctx.barcode(D=dev(B), max_dim=1)
        assert e.value.status == vrph.EINVAL
    with pytest.raises(vrph.VrphError):
        ctx.barcode(D=dev(D), max_dim=7)
    with pytest.raises(vrph.VrphError):
        ctx.barcode(D=dev(D), max_dim=1, threshold=-1.0)
    import ctypes

    Dd = dev(D)
    out = ctypes.c_void_p()
    st = vrph.lib().vrph_barcode_from_dist(ctx.h, Dd.data_ptr(), D.shape[0], 1, float("inf"),
                                           1 << 7, None, ctypes.byref(out))  # an unknown flag
    assert st == vrph.EINVAL and not out.value
    # the context still works afterwards
    ref = oracle.barcode(D, 1)
    assert_same(ctx.barcode(D=dev(D), max_dim=1, keep_zero=True).pairs, ref, "after errors")


def test_index_overflow_is_reported(ctx):
    from paper_2502_05063_amd import vrph

    X = synth.uniform_cube(2048, 3, 0)
    with pytest.raises(vrph.VrphError) as e:
        ctx.barcode(X=dev(X), max_dim=6)
    assert e.value.status == vrph.EOVERFLOW


def test_autotune_keeps_results(tmp_path, monkeypatch):
    from paper_2502_05063_amd import vrph

    tf = tmp_path / "tuning.txt"
    monkeypatch.setenv("VRPH_TUNING_FILE", str(tf))
    X = synth.sphere(70, 3, seed=2)
    ref = oracle.barcode(oracle.pdist(X), 2)
    c1 = vrph.Context()
    try:
        bc = c1.barcode(X=dev(X), max_dim=2, keep_zero=True, autotune=True)
        assert_same(bc.pairs, ref, "autotuned")
        assert all(g > 0 for g in bc.stats["grid"][1:])
        again = c1.barcode(X=dev(X), max_dim=2, keep_zero=True)  # the tuned launch, cached
        assert np.array_equal(again.pairs, bc.pairs) and again.stats["grid"] == bc.stats["grid"]
    finally:
        c1.close()
    # one line per tuned dimension: arch, dimension, size bucket, kernel variant, unit
    # size, groups per CU
    lines = [ln.split() for ln in tf.read_text().splitlines()]
    assert sorted(int(f[1]) for f in lines) == [1, 2] and all(len(f) == 6 for f in lines)
    c2 = vrph.Context()  # reads the file
    try:
        loaded = c2.barcode(X=dev(X), max_dim=2, keep_zero=True)
        assert np.array_equal(loaded.pairs, bc.pairs) and loaded.stats["grid"] == bc.stats["grid"]
    finally:
        c2.close()
