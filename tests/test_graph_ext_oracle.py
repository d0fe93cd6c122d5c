"""Pins of the extended-persistence oracle (oracle/graph_ext.py) by facts
that do not come from its own construction: the bar counts of Theorem
7.6.2, the closed forms of a single cycle and of a clique (Obs. 7.6.5),
per-component minima and maxima for Ext0, spanning-forest weights (scipy)
for the death values of Ord0 and Rel1 and for the edge values of Ext1, and
the symmetry of extended persistence under f -> -f. Mistakes planted in
the cone, the order or the value rule are caught."""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components, minimum_spanning_tree

from oracle import graph_ext as G


def random_graph(rng, n, p, levels=None):
    E = [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < p]
    E = [(b, a) if rng.random() < 0.5 else (a, b) for a, b in E]
    order = rng.permutation(len(E))
    E = [E[i] for i in order]
    if levels:
        f = rng.integers(0, levels, n).astype(np.float32)
    else:
        f = rng.random(n).astype(np.float32)
    return E, f


def components(n, E):
    if not E:
        return n, np.arange(n)
    e = np.asarray(E)
    A = coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(n, n))
    return connected_components(A, directed=False)


def forest_values(n, E, w):
    """Multiset of edge weights of a minimum spanning forest (scipy), with
    weights shifted to be positive (scipy reads 0 as no edge)."""
    if not E:
        return []
    e = np.asarray(E)
    w = np.asarray(w, np.float64)
    shift = 1.0 - w.min()
    A = coo_matrix((w + shift, (e[:, 0], e[:, 1])), shape=(n, n)).tocsr()
    T = minimum_spanning_tree(A)
    return sorted((T.data - shift).tolist())


def kinds(bars, k):
    return bars[bars["kind"] == k]


CASES = [(n, p, lv, s) for s, (n, p, lv) in enumerate(
    [(1, 0.5, None), (2, 1.0, None), (6, 0.5, None), (9, 0.3, 3), (12, 0.6, None), (14, 0.25, 2),
     (10, 1.0, 4), (13, 0.15, None)])]


def check_pins(n, E, f, bars):
    m = len(E)
    C, label = components(n, E)
    # Theorem 7.6.2
    assert len(kinds(bars, G.EXT1)) == m - n + C
    assert len(kinds(bars, G.EXT0)) == C
    assert len(kinds(bars, G.ORD0)) == n - C
    assert len(kinds(bars, G.REL1)) == n - C
    # Ext0: each component's minimum and maximum (ties by vertex index)
    want = []
    for c in range(C):
        vs = [v for v in range(n) if label[v] == c]
        lo = min(vs, key=lambda v: (f[v], v))
        hi = max(vs, key=lambda v: (f[v], v))
        want.append((lo, hi, float(f[lo]), float(f[hi])))
    got = [(int(b["birth"]), int(b["death"]), float(b["birth_value"]), float(b["death_value"]))
           for b in kinds(bars, G.EXT0)]
    assert sorted(got) == sorted(want)
    if m:
        e = np.asarray(E)
        flow = np.maximum(f[e[:, 0]], f[e[:, 1]])
        fup = np.minimum(f[e[:, 0]], f[e[:, 1]])
        # Ord0 deaths: a minimum spanning forest under F_low; Rel1 deaths: a
        # maximum spanning forest under F_up (values as multisets)
        assert sorted(kinds(bars, G.ORD0)["death_value"].tolist()) == pytest.approx(
            forest_values(n, E, flow))
        assert sorted(kinds(bars, G.REL1)["death_value"].tolist()) == pytest.approx(
            sorted(-x for x in forest_values(n, E, -fup)))
        # Ext1 births: the lower values of the edges outside a minimum spanning
        # forest; Ext1 deaths: the upper values outside a maximum one
        rest_low = sorted(flow.tolist())
        for x in forest_values(n, E, flow):
            rest_low.remove(pytest.approx(x))
        rest_up = sorted(fup.tolist())
        for x in forest_values(n, E, -fup):
            rest_up.remove(pytest.approx(-x))
        ext1 = kinds(bars, G.EXT1)
        assert sorted(ext1["birth_value"].tolist()) == pytest.approx(sorted(rest_low))
        assert sorted(ext1["death_value"].tolist()) == pytest.approx(sorted(rest_up))
    # every bar endpoint is f at the vertex the record names
    assert np.array_equal(bars["birth_value"], f[bars["birth_vertex"]])
    assert np.array_equal(bars["death_value"], f[bars["death_vertex"]])


@pytest.mark.parametrize("n,p,levels,seed", CASES)
def test_counts_components_and_forests(n, p, levels, seed):
    rng = np.random.default_rng(seed)
    E, f = random_graph(rng, n, p, levels)
    check_pins(n, E, f, G.extended_persistence(n, E, f))


def test_single_cycle_and_tree():
    rng = np.random.default_rng(11)
    for n in (3, 5, 9):
        f = rng.random(n).astype(np.float32)
        cyc = [(i, (i + 1) % n) for i in range(n)]
        ext1 = kinds(G.extended_persistence(n, cyc, f), G.EXT1)
        # the cycle closes at its largest value and is filled at its smallest
        assert len(ext1) == 1
        assert float(ext1["birth_value"][0]) == float(f.max())
        assert float(ext1["death_value"][0]) == float(f.min())
        path = cyc[:-1]
        bars = G.extended_persistence(n, path, f)
        assert len(kinds(bars, G.EXT1)) == 0
        ext0 = kinds(bars, G.EXT0)
        assert len(ext0) == 1 and float(ext0["birth_value"][0]) == float(f.min())
        assert float(ext0["death_value"][0]) == float(f.max())


def test_clique_has_the_longest_cycle_bar():
    # Obs. 7.6.5: in a clique the bar [max f, min f] is always there
    rng = np.random.default_rng(12)
    for n in (3, 6, 10):
        f = rng.random(n).astype(np.float32)
        E = [(a, b) for a in range(n) for b in range(a + 1, n)]
        ext1 = kinds(G.extended_persistence(n, E, f), G.EXT1)
        pairs = set(zip(ext1["birth_value"].tolist(), ext1["death_value"].tolist()))
        assert (float(f.max()), float(f.min())) in pairs


@pytest.mark.parametrize("seed", range(6))
def test_negation_symmetry(seed):
    # f -> -f reflects the extended bars, (b, d) -> (-d, -b), and exchanges
    # Ord0 with Rel1 (distinct values, so no tie rule is involved)
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 13))
    E, f = random_graph(rng, n, rng.uniform(0.2, 0.9))
    A = G.extended_persistence(n, E, f)
    B = G.extended_persistence(n, E, -f)
    for k in (G.EXT0, G.EXT1):
        a = sorted(zip((-kinds(A, k)["death_value"]).tolist(), (-kinds(A, k)["birth_value"]).tolist()))
        b = sorted(zip(kinds(B, k)["birth_value"].tolist(), kinds(B, k)["death_value"].tolist()))
        assert a == b
    a = sorted(zip((-kinds(A, G.ORD0)["birth_value"]).tolist(), (-kinds(A, G.ORD0)["death_value"]).tolist()))
    b = sorted(zip(kinds(B, G.REL1)["birth_value"].tolist(), kinds(B, G.REL1)["death_value"].tolist()))
    assert a == b


@pytest.mark.parametrize("mistake", ["triangle_misses_edge", "upper_ascending",
                                     "lower_value_at_min"])
def test_planted_mistake_is_caught(monkeypatch, mistake):
    """A mistake planted in the oracle's cone or order fails a pin."""
    real_cols, real_order = G.boundary_columns, G.cone_filtration

    def broken_cols(n_, edges, ff):
        cols, order, e2, f2 = real_cols(n_, edges, ff)
        for j, (kind, _) in enumerate(order):
            if mistake == "triangle_misses_edge" and kind == "ct":
                cols[j] = cols[j][1:]
        return cols, order, e2, f2

    def broken_order(n_, edges, ff):
        order, e2, f2 = real_order(n_, edges, ff)
        k = 1 + n_ + len(e2)  # alpha, then the lower part, then the upper part
        return order[:k] + order[k:][::-1], e2, f2

    if mistake == "upper_ascending":
        monkeypatch.setattr(G, "cone_filtration", broken_order)
    elif mistake == "lower_value_at_min":
        monkeypatch.setattr(G, "_vmax", G._vmin)
    else:
        monkeypatch.setattr(G, "boundary_columns", broken_cols)
    caught = 0
    for seed in range(4):
        rng = np.random.default_rng(50 + seed)
        n = 9
        E, f = random_graph(rng, n, 0.5)
        try:
            check_pins(n, E, f, G.extended_persistence(n, E, f))
        except (AssertionError, ValueError, KeyError):
            caught += 1
    assert caught > 0


def test_rejects_bad_graphs():
    with pytest.raises(ValueError):
        G.extended_persistence(3, [(0, 0)], np.zeros(3, np.float32))
    with pytest.raises(ValueError):
        G.extended_persistence(3, [(0, 1), (1, 0)], np.zeros(3, np.float32))
    with pytest.raises(ValueError):
        G.extended_persistence(3, [(0, 3)], np.zeros(3, np.float32))
