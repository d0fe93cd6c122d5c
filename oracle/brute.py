"""Brute-force persistence check from ranks, independent of any reduction.

TEST INFRASTRUCTURE ONLY. Used to pin the oracle on tiny inputs (n <= 8).

Thm 3.2.20 with Eq. 3.99: for a simplex-wise filtration K_1 <= ... <= K_N and
a <= b, the rank of H_p(K_a) -> H_p(K_b) equals the number of p-dimensional
intervals [i, j) of the decomposition with i <= a < j, j > b (essential
intervals have j = infinity). Eq. 3.99 prints the second condition as
"i <= a"; it can only mean the interval is still alive at b, which is the
reading used here.

The rank is computed by linear algebra over GF(2) and nothing else:
    rank(H_p(K_a) -> H_p(K_b)) = dim Z_p(K_a) - dim(Z_p(K_a) n B_p(K_b)),
    dim Z_p(K_a) = #p-simplices of K_a - rank(d_p on K_a),
    dim(Z_p(K_a) n B_p(K_b)) = rank(M) - rank(M restricted to rows outside K_a),
where M is d_{p+1} with columns the (p+1)-simplices of K_b and rows the
p-simplices of K_b (a boundary is supported in K_a iff its rows outside K_a
vanish; those boundaries are images of ker of the restricted map).
"""
from __future__ import annotations

import itertools
from math import comb

import numpy as np


def gf2_rank(M: np.ndarray) -> int:
    M = (np.asarray(M, dtype=np.uint8) & 1).copy()
    if M.size == 0:
        return 0
    rows, cols = M.shape
    r = 0
    for c in range(cols):
        piv = None
        for i in range(r, rows):
            if M[i, c]:
                piv = i
                break
        if piv is None:
            continue
        if piv != r:
            M[[r, piv]] = M[[piv, r]]
        for i in range(rows):
            if i != r and M[i, c]:
                M[i] ^= M[r]
        r += 1
        if r == rows:
            break
    return r


def cidx(verts) -> int:
    """Eq. 5.6 with math.comb: vertices v_0 < ... < v_q -> sum C(v_i, i+1)."""
    return sum(comb(v, i + 1) for i, v in enumerate(sorted(verts)))


def filtration(D: np.ndarray, max_simplex_dim: int, tau: float):
    """All simplices with diam <= tau up to max_simplex_dim, in the order of
    Sec. 5.1.4 (diameter up, dimension up, index down)."""
    n = D.shape[0]
    out = []
    for k in range(1, max_simplex_dim + 2):
        for vs in itertools.combinations(range(n), k):
            d = max((float(D[a, b]) for a, b in itertools.combinations(vs, 2)), default=0.0)
            if d <= tau:
                out.append((d, k - 1, cidx(vs), vs))
    out.sort(key=lambda s: (s[0], s[1], -s[2]))
    return out


def persistent_ranks(S, p: int) -> np.ndarray:
    """beta[a, b] = rank of H_p(K_a) -> H_p(K_b) for 0 <= a <= b <= N (K_0 empty)."""
    N = len(S)
    index = {s[3]: i + 1 for i, s in enumerate(S)}  # 1-based filtration index
    P = [i + 1 for i, s in enumerate(S) if s[1] == p]
    Q = [i + 1 for i, s in enumerate(S) if s[1] == p + 1]
    Pm1 = [i + 1 for i, s in enumerate(S) if s[1] == p - 1]

    def boundary(rows, cols):
        rpos = {r: k for k, r in enumerate(rows)}
        M = np.zeros((len(rows), len(cols)), np.uint8)
        for c, j in enumerate(cols):
            vs = S[j - 1][3]
            for drop in range(len(vs)):
                f = vs[:drop] + vs[drop + 1:]
                if f:
                    M[rpos[index[f]], c] ^= 1
        return M

    dp = boundary(Pm1, P) if p >= 1 else np.zeros((0, len(P)), np.uint8)
    dp1 = boundary(P, Q)
    Pa = np.asarray(P, dtype=np.int64)
    Qa = np.asarray(Q, dtype=np.int64)
    Pm1a = np.asarray(Pm1, dtype=np.int64)
    beta = np.zeros((N + 1, N + 1), np.int64)
    for a in range(1, N + 1):
        pa = Pa <= a
        z = int(pa.sum()) - gf2_rank(dp[np.ix_(Pm1a <= a, pa)]) if p >= 1 else int(pa.sum())
        for b in range(a, N + 1):
            rows_b = Pa <= b
            cols_b = Qa <= b
            M = dp1[np.ix_(rows_b, cols_b)]
            outside = (Pa > a)[rows_b]
            inter = gf2_rank(M) - gf2_rank(M[outside])
            beta[a, b] = z - inter
    return beta


def check_pairs_against_ranks(D, max_dim: int, tau: float, pairs) -> None:
    """Raise AssertionError unless the oracle's pairs reproduce every rank."""
    S = filtration(D, max_dim + 1, tau)
    N = len(S)
    pos = {(s[1], s[2]): i + 1 for i, s in enumerate(S)}
    for p in range(max_dim + 1):
        beta = persistent_ranks(S, p)
        ivs = []
        for q in pairs[pairs["dim"] == p]:
            i = pos[(p, int(q["birth"]))]
            j = N + 1 if q["essential"] else pos[(p + 1, int(q["death"]))]
            ivs.append((i, j))
        for a in range(1, N + 1):
            for b in range(a, N + 1):
                alive = sum(1 for i, j in ivs if i <= a and j > b)
                assert alive == beta[a, b], (p, a, b, alive, int(beta[a, b]))
