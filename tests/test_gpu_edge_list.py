"""Large sparse clouds (512 points and more, fewer than half of the vertex
pairs within the threshold) hand the host their finite edges sorted by
weight instead of the n x n weights. On one context, over a sequence of
clouds and thresholds (the same size twice in a row, so that the host's
rank table is reset from the previous edge list, then other sizes, a dense
cloud in between, dimensions up to 3 so that the listed prefixes come from
the edge list too), every barcode, every pair reported, equals the one the
weight-matrix path gives (VRPH_DENSE_HOST_WEIGHTS); and the 6000-point cube
still equals its oracle golden after the sequence.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_2502_05063_amd import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def strip(pairs):
    out = np.empty(len(pairs), oracle.PAIR_DTYPE)
    for f in oracle.PAIR_DTYPE.names:
        out[f] = pairs[f]
    return out


def _run(ctx, X, **kw):
    import torch

    return ctx.barcode(X=torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda(), **kw)


def test_edge_list_matches_matrix_path():
    from paper_2502_05063_amd import vrph

    ctx = vrph.Context()
    try:
        seq = [(2500, 0.08, 1, 2), (2500, 0.06, 2, 2), (2048, 2.0, 3, 1), (3000, 0.07, 4, 3),
               (3000, 0.075, 5, 1), (700, 0.15, 7, 3), (700, 0.12, 8, 2), (2500, 0.09, 6, 2)]
        for n, thr, seed, max_dim in seq:
            X = synth.uniform_cube(n, 3, seed=seed)
            kw = dict(max_dim=max_dim, threshold=thr, keep_zero=True)
            got = _run(ctx, X, **kw)
            os.environ["VRPH_DENSE_HOST_WEIGHTS"] = "1"
            try:
                ref = _run(ctx, X, **kw)
            finally:
                del os.environ["VRPH_DENSE_HOST_WEIGHTS"]
            assert np.array_equal(got.pairs, ref.pairs), (n, thr, seed)
            for k in ("columns", "apparent", "reduced", "additions", "emergent"):
                assert got.stats[k] == ref.stats[k], (n, thr, seed, k)
        # and the golden after the sequence: nonzero pairs and the hash of
        # the full list, as in the full-size tests
        with open(os.path.join(HERE, "golden", "cube6000.json")) as f:
            g = json.load(f)
        X = synth.uniform_cube(6000, 3, seed=6000)
        bc = _run(ctx, X, max_dim=g["max_dim"], threshold=float(g["threshold"]))
        rows = g["nonzero_pairs"]
        want = np.empty(len(rows), oracle.PAIR_DTYPE)
        for i, (d, e, b, dd, bd, ddm) in enumerate(rows):
            want[i] = (d, e, b, (2**64 - 1) if e else dd, bd, np.inf if e else ddm)
        assert np.array_equal(strip(bc.pairs), want)
        full = _run(ctx, X, max_dim=g["max_dim"], threshold=float(g["threshold"]), keep_zero=True)
        assert hashlib.sha256(strip(full.pairs).tobytes()).hexdigest() == g["full_list_sha256"]
    finally:
        ctx.close()
