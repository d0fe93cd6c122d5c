"""Extended persistence of graphs on the GPU (vrph_graph_extended) against
the oracle (oracle/graph_ext.py: Alg. 2 on the coned graph's boundary
matrix in the extended filtration), graph by graph and bar by bar, on
batches of random graphs with distinct and with heavily tied values,
isolated vertices, single vertices and edgeless graphs, large graphs up to
the 4096-vertex limit, and the error paths."""
import numpy as np
import pytest

from oracle import graph_ext as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2502_05063_amd import vrph

    assert torch.cuda.is_available()
    c = vrph.Context()
    yield c
    c.close()


def random_graph(rng, n, p, levels=None):
    E = [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < p]
    E = [(b, a) if rng.random() < 0.5 else (a, b) for a, b in E]
    E = [E[i] for i in rng.permutation(len(E))]
    f = (rng.integers(0, levels, n) if levels else rng.standard_normal(n)).astype(np.float32)
    return np.asarray(E, np.int32).reshape(-1, 2), f


def run_batch(ctx, graphs):
    import torch

    v_off = np.concatenate([[0], np.cumsum([len(f) for _, f in graphs])])
    e_off = np.concatenate([[0], np.cumsum([len(E) for E, _ in graphs])])
    f = torch.from_numpy(np.concatenate([f for _, f in graphs])).cuda()
    E = torch.from_numpy(np.concatenate([E for E, _ in graphs]).reshape(-1, 2)).cuda()
    _, per = ctx.graph_extended(f, E, v_off, e_off)
    return per


def compare(graphs, per):
    for g, ((E, f), got) in enumerate(zip(graphs, per)):
        n = len(f)
        ref = G.extended_persistence(n, [tuple(e) for e in E], f)
        assert len(got) == n + len(E), g
        srt = np.sort(got.copy().view(G.BAR_DTYPE), order=["kind", "birth", "death"])
        assert np.array_equal(srt, ref), f"graph {g} (n {n}, m {len(E)})"


@pytest.mark.parametrize("levels", [None, 3], ids=["distinct", "ties"])
def test_random_batch_matches_oracle(ctx, levels):
    rng = np.random.default_rng(1 if levels else 2)
    graphs = []
    for k in range(120):
        n = int(rng.integers(1, 70))
        p = float(rng.uniform(0.02, 0.6))
        graphs.append(random_graph(rng, n, p, levels))
    compare(graphs, run_batch(ctx, graphs))


def test_edge_cases(ctx):
    rng = np.random.default_rng(3)
    single = (np.zeros((0, 2), np.int32), np.array([0.5], np.float32))
    empty = (np.zeros((0, 2), np.int32), rng.random(5).astype(np.float32))
    path = (np.array([[0, 1], [1, 2], [2, 3]], np.int32), np.array([3, 1, 2, 0], np.float32))
    cycle = (np.array([[i, (i + 1) % 7] for i in range(7)], np.int32),
             rng.random(7).astype(np.float32))
    clique = (np.array([[a, b] for a in range(9) for b in range(a)], np.int32),
              rng.random(9).astype(np.float32))
    equal = (np.array([[a, b] for a in range(6) for b in range(a)], np.int32),
             np.zeros(6, np.float32))
    isolated = (np.array([[0, 3], [3, 5]], np.int32), rng.random(8).astype(np.float32))
    negz = (np.array([[0, 1], [1, 2], [2, 0]], np.int32), np.array([-0.0, 0.0, -1.0], np.float32))
    graphs = [single, empty, path, cycle, clique, equal, isolated, negz]
    compare(graphs, run_batch(ctx, graphs))


@pytest.mark.parametrize("n,p,levels", [(500, 0.05, None), (2000, 0.004, None), (4096, 0.001, 5)])
def test_large_graphs(ctx, n, p, levels):
    rng = np.random.default_rng(n)
    graphs = [random_graph(rng, n, p, levels), random_graph(rng, 40, 0.3)]
    compare(graphs, run_batch(ctx, graphs))


def test_invalid_input(ctx):
    import torch

    from paper_2502_05063_amd import vrph

    f = torch.rand(6, device="cuda")
    v_off, e_off = [0, 3, 6], [0, 1, 2]
    for bad in ([[0, 1], [0, 3]], [[0, 1], [2, 2]], [[0, -1], [0, 1]]):
        E = torch.tensor(bad, dtype=torch.int32, device="cuda")
        with pytest.raises(vrph.VrphError) as ei:
            ctx.graph_extended(f, E, v_off, e_off)
        assert ei.value.status == vrph.EINVAL
    E = torch.tensor([[0, 1], [0, 2]], dtype=torch.int32, device="cuda")
    fn = f.clone()
    fn[4] = float("nan")
    with pytest.raises(vrph.VrphError):
        ctx.graph_extended(fn, E, v_off, e_off)
    with pytest.raises(vrph.VrphError):  # a graph without vertices
        ctx.graph_extended(f, E, [0, 3, 3, 6], [0, 1, 1, 2])
    # a valid call after the rejected ones
    _, per = ctx.graph_extended(f, E, v_off, e_off)
    assert [len(b) for b in per] == [4, 4]
