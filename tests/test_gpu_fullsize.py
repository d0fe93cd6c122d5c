"""Full-size parity: the GPU barcodes of the sphere_3_192-like and o3-like
workloads against expected values written by the CPU oracle alone
(tests/golden/make_golden.py): every pair including zero-persistence ones
(SHA-256 of the canonical list), the pairs of nonzero persistence one by
one, the columns per dimension, and the apparent decisions of sampled
columns against Def. 5.3.4 evaluated by the oracle column by column.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_2502_05063_amd import synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2502_05063_amd import vrph

    assert torch.cuda.is_available()
    c = vrph.Context()
    yield c
    c.close()


def strip(pairs):
    out = np.empty(len(pairs), oracle.PAIR_DTYPE)
    for f in oracle.PAIR_DTYPE.names:
        out[f] = pairs[f]
    return out


def golden_nonzero(g):
    rows = g["nonzero_pairs"]
    out = np.empty(len(rows), oracle.PAIR_DTYPE)
    for i, (d, e, b, dd, bd, ddm) in enumerate(rows):
        out[i] = (d, e, b, (2**64 - 1) if e else dd, bd, np.inf if e else ddm)
    return out


@pytest.mark.parametrize("name,gen", [
    ("c2_sphere192", lambda: synth.sphere(192, 3, seed=0)),
    ("c3_o3_1024", lambda: synth.orthogonal_3x3(1024, seed=0)),
])
def test_full_size_against_oracle_golden(ctx, name, gen):
    import torch

    path = os.path.join(GOLD, f"{name}.json")
    g = json.load(open(path))
    X = gen()
    thr = float(g["threshold"]) if g["threshold"] != "inf" else float("inf")
    Xd = torch.from_numpy(X).cuda()
    # the distances the barcode is computed from equal the oracle's, bit for bit
    D = ctx.pdist(Xd).cpu().numpy()
    assert np.array_equal(D.view(np.uint32), oracle.pdist(X).view(np.uint32))
    bc = ctx.barcode(X=Xd, max_dim=g["max_dim"], threshold=thr)
    assert np.array_equal(strip(bc.pairs), golden_nonzero(g)), f"{name}: nonzero pairs differ"
    assert bc.stats["columns"][1:] == g["columns_per_dim"][1:], (bc.stats["columns"], g["columns_per_dim"])
    full = ctx.barcode(X=Xd, max_dim=g["max_dim"], threshold=thr, keep_zero=True)
    counts = [int((full.pairs["dim"] == d).sum()) for d in range(g["max_dim"] + 1)]
    assert counts == g["pairs_per_dim"]
    rec = strip(full.pairs)
    assert hashlib.sha256(rec.tobytes()).hexdigest() == g["full_list_sha256"]

    # sampled columns: the GPU's apparent count equals Def. 5.3.4, and every
    # sampled column the oracle finds apparent is paired that way on the GPU
    rng = np.random.default_rng(7)
    d = g["max_dim"]
    cols = full.pairs[full.pairs["dim"] == d]
    pick = rng.choice(len(cols), 64, replace=False)
    for p in cols[pick]:
        t = oracle.is_apparent(D, d, int(p["birth"]), thr)
        if t is not None:
            assert int(p["death"]) == t
