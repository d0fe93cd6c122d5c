"""The allocation-free backward (vrph_backward_noalloc) against vrph_backward.

Two calls in a row on one context, the second with a smaller input, each
compared with the allocating entry point on the same pairs and with the
binary64 gradient oracle (1e-5 relative); then the error path: an edge
outside X is rejected with gX unchanged, and the next call is right again
(the shared scratch flag is cleared by every call).
"""
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


def _h1_pairs(ctx, X):
    """Nonzero H1 pairs of X from the GPU barcode, with loss sum (d - b)^2."""
    import torch

    Xd = torch.from_numpy(X).cuda()
    bc = ctx.barcode(X=Xd, max_dim=1)
    h1 = bc.dim(1)
    h1 = h1[h1["essential"] == 0]
    pers = (h1["death_diam"] - h1["birth_diam"]).astype(np.float32)
    edges = np.concatenate([h1["birth_edge"], h1["death_edge"]], axis=1).astype(np.int32)
    ref = np.empty(len(h1), oracle.PAIR_DTYPE)
    for f in oracle.PAIR_DTYPE.names:
        ref[f] = h1[f]
    return Xd, edges, -2 * pers, 2 * pers, ref


@pytest.mark.parametrize("sizes", [(500, 120)])
def test_noalloc_backward_matches_backward_twice(ctx, sizes):
    import torch

    for k, n in enumerate(sizes):
        X = synth.torus_batch(1, n, 0.1, seed=11 + k)[0]
        Xd, edges, gb, gd, ref = _h1_pairs(ctx, X)
        assert len(edges) > 0
        e = torch.from_numpy(edges).cuda()
        gbd, gdd = torch.from_numpy(gb).cuda(), torch.from_numpy(gd).cuda()
        g_ref = torch.zeros_like(Xd)
        ctx.backward(Xd, e, gbd, gdd, g_ref)
        g_new = torch.zeros_like(Xd)
        ctx.backward_noalloc(Xd, e, gbd, gdd, g_new)
        torch.cuda.synchronize()
        a, b = g_new.cpu().numpy(), g_ref.cpu().numpy()
        scale = np.abs(b).max()
        assert scale > 0
        # float32 atomics: the summation order may differ, nothing else
        assert np.abs(a - b).max() / scale <= 1e-5, (n, np.abs(a - b).max() / scale)
        G = oracle.gradient(X, oracle.pdist(X), ref, gb, gd)
        assert np.abs(a - G).max() / np.abs(G).max() <= 1e-5


def test_noalloc_backward_errors_and_recovery(ctx):
    import torch

    from paper_2502_05063_amd import vrph

    X = torch.rand(10, 3, device="cuda")
    gX = torch.zeros_like(X)
    g = torch.ones(1, device="cuda")
    for bad in ([0, 10, -1, -1], [-2, 1, -1, -1], [1, 0, 3, 2**31 - 1]):
        edges = torch.tensor([bad], dtype=torch.int32, device="cuda")
        with pytest.raises(vrph.VrphError) as ei:
            ctx.backward_noalloc(X, edges, g, g, gX)
        assert ei.value.status == vrph.EINVAL
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(gX)) == 0, "a rejected call changed gX"
    # the flag left set by the rejected call does not leak into the next one
    edges = torch.tensor([[1, 0, -1, -1]], dtype=torch.int32, device="cuda")
    ctx.backward_noalloc(X, edges, g, g, gX)
    d = (X[1] - X[0]) / torch.linalg.norm(X[1] - X[0])
    assert torch.allclose(gX[1], d) and torch.allclose(gX[0], -d)
    # no pairs: nothing to do
    empty = torch.empty((0, 4), dtype=torch.int32, device="cuda")
    ge = torch.empty(0, device="cuda")
    ctx.backward_noalloc(X, empty, ge, ge, gX)
    assert torch.allclose(gX[1], d)


def test_noalloc_backward_rejects_converting_arguments(ctx):
    import torch

    X = torch.rand(10, 3, device="cuda", dtype=torch.float64)
    gX = torch.zeros(10, 3, device="cuda")
    edges = torch.tensor([[1, 0, -1, -1]], dtype=torch.int32, device="cuda")
    g = torch.ones(1, device="cuda")
    with pytest.raises(ValueError):
        ctx.backward_noalloc(X, edges, g, g, gX)
