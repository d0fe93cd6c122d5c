"""Extended persistence of a graph with a vertex function, from its definition.

TEST INFRASTRUCTURE ONLY: the product path never imports this module. Only
tests, the smoke check and the CPU-baseline leg of the benchmark may use it.

What it computes (Zhang, "Computing and Learning on Combinatorial Data",
Ch. 7, Sec. 7.2): the cone of G (Eq. 7.3: a new vertex alpha, an edge
(alpha, v) per vertex v and a triangle (alpha, u, v) per edge (u, v)) with
the extended filtration (Eq. 7.4): the lower filtration of G followed by the
upper filtration of the cone simplices. Its persistence pairs are the pivots
of Alg. 2 on the Z/2 boundary matrix of that index filtration (the standard
reduction of the oracle's C library, `oracle.reduce_explicit`), sorted into
the four barcodes of Sec. 7.2 by the kinds of their two simplices:

  Ord0 (B0^low)  G vertex v  - G edge e          (f(v), F_low(e))
  Rel1 (B0^up)   cone edge over v - cone triangle over e   (f(v), F_up(e))
  Ext0 (B0^ext)  G vertex v  - cone edge over u  (f(v), f(u))
  Ext1 (B1^ext)  G edge e'   - cone triangle over e        (F_low(e'), F_up(e))

with F_low(u, v) = max(f(u), f(v)) and F_up(u, v) = min(f(u), f(v)).

Readings where the paper leaves a choice (the same ones the library takes):
  - Ties. The paper breaks ties between edge values with a small multiple of
    the other endpoint's value; here the index filtration is a total order
    on exact keys instead. Lower part, ascending: vertex v by (f(v), v); an
    edge by (F_low, then F_up, then edge id); at equal value a vertex comes
    before an edge. Upper part, descending: the cone edge over v by
    (f(v), v); the cone triangle over an edge by (F_up, then F_low, then
    edge id); at equal value a cone edge comes before a triangle.
  - The cone vertex alpha is the first simplex of the filtration (its value
    plays no part): it is then the one essential class of the contractible
    cone, and every component of G gives an Ext0 bar (its minimum and
    maximum), as Alg. 27 computes them.
  - Every endpoint of a bar is f at one vertex: a vertex, the endpoint of an
    edge with the larger (f, index) for F_low, the one with the smaller
    (f, index) for F_up. The records give that vertex (the gradient of the
    value flows to it).
"""
from __future__ import annotations

import numpy as np

import oracle

ORD0, REL1, EXT0, EXT1 = 0, 1, 2, 3
BAR_DTYPE = np.dtype([
    ("kind", "<i4"),          # ORD0, REL1, EXT0, EXT1
    ("birth", "<i4"),         # vertex (ORD0, REL1, EXT0) or edge id (EXT1)
    ("death", "<i4"),         # edge id (ORD0, REL1, EXT1) or vertex (EXT0)
    ("birth_value", "<f4"),
    ("death_value", "<f4"),
    ("birth_vertex", "<i4"),  # the vertex whose f is birth_value
    ("death_vertex", "<i4"),  # the vertex whose f is death_value
])


def _check_graph(n, edges, f):
    edges = np.asarray(edges, np.int64).reshape(-1, 2)
    f = np.asarray(f, np.float32)
    if f.shape != (n,) or not np.all(np.isfinite(f)):
        raise ValueError("f must hold n finite values")
    if len(edges) and (edges.min() < 0 or edges.max() >= n or np.any(edges[:, 0] == edges[:, 1])):
        raise ValueError("edges must join two distinct vertices in [0, n)")
    key = np.sort(edges, axis=1)
    if len({(int(a), int(b)) for a, b in key}) != len(key):
        raise ValueError("a repeated edge")
    return edges, f


def _vmax(f, u, v):
    """Endpoint with the larger (f, index): the vertex of F_low(u, v)."""
    return u if (f[u], u) > (f[v], v) else v


def _vmin(f, u, v):
    """Endpoint with the smaller (f, index): the vertex of F_up(u, v)."""
    return u if (f[u], u) < (f[v], v) else v


def cone_filtration(n, edges, f):
    """The simplices of Cone(G) in the extended index filtration, as
    (kind, id) with kind in {'alpha', 'v', 'e', 'cv', 'ct'} (G vertex, G
    edge, cone edge over vertex id, cone triangle over edge id)."""
    edges, f = _check_graph(n, edges, f)
    ff = [float(x) for x in f]
    lo = lambda e: max(ff[edges[e, 0]], ff[edges[e, 1]])  # noqa: E731
    up = lambda e: min(ff[edges[e, 0]], ff[edges[e, 1]])  # noqa: E731
    lower = [((ff[v], 0, ff[v], v), ("v", v)) for v in range(n)]
    lower += [((lo(e), 1, up(e), e), ("e", e)) for e in range(len(edges))]
    lower.sort()
    # upper part, descending in value: sort by negated keys
    upper = [((-ff[v], 0, -ff[v], -v), ("cv", v)) for v in range(n)]
    upper += [((-up(e), 1, -lo(e), -e), ("ct", e)) for e in range(len(edges))]
    upper.sort()
    return [("alpha", 0)] + [s for _, s in lower] + [s for _, s in upper], edges, f


def boundary_columns(n, edges, f):
    """Boundary matrix of the cone in that order: column j lists the
    positions of simplex j's facets."""
    order, edges, f = cone_filtration(n, edges, f)
    pos = {s: i for i, s in enumerate(order)}
    cols = []
    for kind, i in order:
        if kind in ("alpha", "v"):
            fac = []
        elif kind == "e":
            fac = [pos[("v", int(edges[i, 0]))], pos[("v", int(edges[i, 1]))]]
        elif kind == "cv":
            fac = [pos[("alpha", 0)], pos[("v", i)]]
        else:  # cone triangle over edge i = (a, b): facets (a, b), (alpha, a), (alpha, b)
            a, b = int(edges[i, 0]), int(edges[i, 1])
            fac = [pos[("e", i)], pos[("cv", a)], pos[("cv", b)]]
        cols.append(sorted(fac))
    return cols, order, edges, f


def extended_persistence(n, edges, f):
    """The four barcodes as BAR_DTYPE records, sorted by (kind, birth, death)."""
    cols, order, edges, f = boundary_columns(n, edges, f)
    low = oracle.reduce_explicit(cols)
    out = []
    for j, i in enumerate(low):
        if i < 0:
            continue
        (bk, b), (dk, d) = order[int(i)], order[j]
        if bk == "v" and dk == "e":
            u, w = int(edges[d, 0]), int(edges[d, 1])
            out.append((ORD0, b, d, f[b], max(f[u], f[w]), b, _vmax(f, u, w)))
        elif bk == "cv" and dk == "ct":
            u, w = int(edges[d, 0]), int(edges[d, 1])
            out.append((REL1, b, d, f[b], min(f[u], f[w]), b, _vmin(f, u, w)))
        elif bk == "v" and dk == "cv":
            out.append((EXT0, b, d, f[b], f[d], b, d))
        elif bk == "e" and dk == "ct":
            u, w = int(edges[b, 0]), int(edges[b, 1])
            x, y = int(edges[d, 0]), int(edges[d, 1])
            out.append((EXT1, b, d, max(f[u], f[w]), min(f[x], f[y]), _vmax(f, u, w),
                        _vmin(f, x, y)))
        else:
            raise AssertionError(f"unexpected pair {bk} - {dk}")
    bars = np.array(out, BAR_DTYPE) if out else np.zeros(0, BAR_DTYPE)
    return np.sort(bars, order=["kind", "birth", "death"])
