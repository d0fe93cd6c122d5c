"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

Holds no arithmetic of the persistence method: only random point clouds and
distance matrices with the shapes and distributions of the workloads:

  uniform_cube(64)            64 points i.i.d. U[0,1)^3
  sphere(192, 3)              192 points on S^3 in R^4 (normalised Gaussians);
                              stands in for the paper's sphere_3_192 dataset
  orthogonal_3x3(1024)        random O(3) matrices (QR of a Gaussian, signs fixed
                              by diag(R)), flattened row-major into R^9; stands
                              in for the paper's o3 dataset
  circle_or_torus_batch(256)  clouds of U{50..400} points, each a noisy circle
                              (radius 1) or torus (R=2, r=0.5), sigma 0.05
  torus_batch(64, 500)        noisy tori, sigma 0.1
  permutation_distances(n)    a random permutation of 1..n(n-1)/2 filling a
                              symmetric matrix (random distance matrices of the
                              paper's apparent-fraction experiment)
  rips2_boundary_csc(D, tau)  the explicit boundary matrix (CSC) of a Rips
                              2-skeleton, the input of the explicit-matrix
                              workload
"""
from __future__ import annotations

import numpy as np


def _rng(seed):
    return np.random.default_rng(seed)


def uniform_cube(n: int = 64, dim: int = 3, seed: int = 0) -> np.ndarray:
    return _rng(seed).random((n, dim)).astype(np.float32)


def sphere(n: int = 192, k: int = 3, seed: int = 0) -> np.ndarray:
    g = _rng(seed).standard_normal((n, k + 1))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return g.astype(np.float32)


def orthogonal_3x3(n: int = 1024, seed: int = 0) -> np.ndarray:
    rng = _rng(seed)
    out = np.empty((n, 9), np.float64)
    for i in range(n):
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))[None, :]
        out[i] = q.reshape(-1)
    return out.astype(np.float32)


def circle(n: int, radius: float, sigma: float, rng) -> np.ndarray:
    a = rng.uniform(0.0, 2.0 * np.pi, n)
    x = np.stack([radius * np.cos(a), radius * np.sin(a), np.zeros(n)], axis=1)
    return (x + rng.normal(0.0, sigma, (n, 3))).astype(np.float32)


def torus(n: int, R: float, r: float, sigma: float, rng) -> np.ndarray:
    a = rng.uniform(0.0, 2.0 * np.pi, n)
    b = rng.uniform(0.0, 2.0 * np.pi, n)
    x = np.stack(
        [(R + r * np.cos(b)) * np.cos(a), (R + r * np.cos(b)) * np.sin(a), r * np.sin(b)], axis=1
    )
    return (x + rng.normal(0.0, sigma, (n, 3))).astype(np.float32)


def circle_or_torus_batch(count: int = 256, nmin: int = 50, nmax: int = 400, sigma: float = 0.05,
                          seed: int = 0):
    rng = _rng(seed)
    clouds = []
    for _ in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        if rng.random() < 0.5:
            clouds.append(circle(n, 1.0, sigma, rng))
        else:
            clouds.append(torus(n, 2.0, 0.5, sigma, rng))
    return clouds


def torus_batch(count: int = 64, n: int = 500, sigma: float = 0.1, seed: int = 0):
    rng = _rng(seed)
    return [torus(n, 2.0, 0.5, sigma, rng) for _ in range(count)]


def permutation_distances(n: int, seed: int = 0) -> np.ndarray:
    """Symmetric float32 matrix whose n(n-1)/2 off-diagonal entries are a random
    permutation of 1..n(n-1)/2 (exact in float32 while n(n-1)/2 < 2^24)."""
    m = n * (n - 1) // 2
    vals = _rng(seed).permutation(m).astype(np.float64) + 1.0
    D = np.zeros((n, n), np.float32)
    iu = np.tril_indices(n, -1)
    D[iu] = vals
    return D + D.T


def integer_distances(n: int, levels: int, seed: int = 0) -> np.ndarray:
    """Symmetric matrix with entries drawn from {1..levels}: many exact ties."""
    rng = _rng(seed)
    D = np.zeros((n, n), np.float32)
    iu = np.tril_indices(n, -1)
    D[iu] = rng.integers(1, levels + 1, len(iu[0])).astype(np.float32)
    return D + D.T


CONFIGS = {
    "c1_cube64": dict(max_dim=1, threshold=float("inf")),
    "c2_sphere192": dict(max_dim=3, threshold=float("inf")),
    "c3_o3_1024": dict(max_dim=3, threshold=1.8),
    "c4_batch256": dict(max_dim=1, threshold=float("inf")),
    "c5_torus64x500": dict(max_dim=1, threshold=float("inf")),
    # the o3 recipe at the paper's size (Table 5.2: 4096 points, threshold 1.4)
    "o3_4096": dict(max_dim=3, threshold=1.4),
    # clouds above 4096 points (sparse complexes: about 15-25 neighbours per
    # point within the threshold)
    "cube6000": dict(max_dim=2, threshold=0.09),
    "cube10000": dict(max_dim=1, threshold=0.06),
    "cube16384": dict(max_dim=1, threshold=0.05),
}


def rips2_boundary_csc(D: np.ndarray, tau: float):
    """Boundary matrix (CSC: col_ptr, rows; int64) of the Rips 2-skeleton of
    the distance matrix D up to tau: vertices, edges and triangles within
    tau, in filtration order (diameter, then dimension, then cell number),
    which puts faces before cofaces; column j lists the positions of cell
    j's facets, increasing. An input generator for the explicit-matrix
    workload."""
    D = np.asarray(D, np.float64)
    n = D.shape[0]
    a, b = np.triu_indices(n, 1)
    ew = D[a, b]
    keep = ew <= tau
    a, b, ew = a[keep], b[keep], ew[keep]
    eid = np.full((n, n), -1, np.int64)
    eid[a, b] = np.arange(len(a))
    eid[b, a] = eid[a, b]
    tri = []
    idx = np.arange(n)
    for x in range(n):
        nb = np.nonzero((D[x] <= tau) & (idx > x))[0]
        if len(nb) < 2:
            continue
        i, j = np.triu_indices(len(nb), 1)
        y, z = nb[i], nb[j]
        ok = D[y, z] <= tau
        tri.append(np.stack([np.full(int(ok.sum()), x), y[ok], z[ok]], 1))
    tri = np.concatenate(tri) if tri else np.zeros((0, 3), np.int64)
    tw = np.maximum(np.maximum(D[tri[:, 0], tri[:, 1]], D[tri[:, 0], tri[:, 2]]),
                    D[tri[:, 1], tri[:, 2]])
    nv, ne, nt = n, len(a), len(tri)
    diam = np.concatenate([np.zeros(nv), ew, tw])
    dim = np.concatenate([np.zeros(nv), np.ones(ne), np.full(nt, 2.0)])
    order = np.lexsort((np.arange(nv + ne + nt), dim, diam))  # cell at each position
    pos = np.empty_like(order)
    pos[order] = np.arange(len(order))
    ecols = np.sort(np.stack([pos[a], pos[b]], 1), 1)
    tcols = np.sort(np.stack([pos[nv + eid[tri[:, 0], tri[:, 1]]], pos[nv + eid[tri[:, 0], tri[:, 2]]],
                              pos[nv + eid[tri[:, 1], tri[:, 2]]]], 1), 1)
    lens = np.concatenate([np.zeros(nv, np.int64), np.full(ne, 2, np.int64),
                           np.full(nt, 3, np.int64)])[order]
    col_ptr = np.zeros(len(order) + 1, np.int64)
    col_ptr[1:] = np.cumsum(lens)
    rows = np.empty(int(col_ptr[-1]), np.int64)
    pe = np.nonzero((order >= nv) & (order < nv + ne))[0]
    pt = np.nonzero(order >= nv + ne)[0]
    for k in range(2):
        rows[col_ptr[pe] + k] = ecols[order[pe] - nv, k]
    for k in range(3):
        rows[col_ptr[pt] + k] = tcols[order[pt] - nv - ne, k]
    return col_ptr, rows


def erdos_renyi(n: int, p: float, seed: int):
    """An Erdos-Renyi graph G(n, p) with a standard normal value per vertex
    (the graphs of the paper's extended-persistence timing, Fig. 7.7, with
    random instead of learned vertex values): int32 edges [m, 2] (a < b)
    and float32 f [n]."""
    rng = np.random.default_rng(seed)
    a, b = np.triu_indices(n, 1)
    keep = rng.random(len(a)) < p
    E = np.stack([a[keep], b[keep]], 1).astype(np.int32)
    f = rng.standard_normal(n).astype(np.float32)
    return E, f


def graph_batch(count: int, n_lo: int, n_hi: int, degree: float, seed: int):
    """A batch of graph-classification-like graphs: sizes uniform in
    [n_lo, n_hi], each G(n, degree / (n - 1)) with standard normal vertex
    values. Returns (graphs, v_off, e_off) with graphs a list of (E, f)."""
    rng = np.random.default_rng(seed)
    graphs = []
    for _ in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        graphs.append(erdos_renyi(n, min(1.0, degree / max(n - 1, 1)), int(rng.integers(2**31))))
    v_off = np.concatenate([[0], np.cumsum([len(f) for _, f in graphs])]).astype(np.int64)
    e_off = np.concatenate([[0], np.cumsum([len(E) for E, _ in graphs])]).astype(np.int64)
    return graphs, v_off, e_off
