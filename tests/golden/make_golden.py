"""Write full-size expected values with the CPU oracle (and nothing else).

Batched configurations (c4_batch256, c5_torus64x500) are written cloud by
cloud, on a process pool: for every cloud its size, the counts of pairs per
dimension and the SHA-256 of its full canonical pair list; for the
differentiable torus set also the oracle's H1 pairs of nonzero persistence
(birth and death indices), the input of the gradient oracle.

For a configuration, runs the oracle's streamed reduction-matrix mode (every
column reduced, no apparent-pair shortcut; Alg. 12 alone cannot finish the
S^3 input) on the seeded synthetic input and stores:
the counts of pairs per dimension, every pair of nonzero persistence, and a
SHA-256 of the full canonical pair list (32-byte records: dim, essential,
birth, death, birth_diam, death_diam) so that a GPU result including every
zero-persistence pair can be compared bit for bit.

    python tests/golden/make_golden.py c2_sphere192 c3_o3_1024
    python tests/golden/make_golden.py c4_batch256 c5_torus64x500
    python tests/golden/make_golden.py o3_4096
    python tests/golden/make_golden.py cube6000 cube10000 cube16384
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2502_05063_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def inputs(name):
    if name == "c1_cube64":
        return synth.uniform_cube(64, 3, seed=0)
    if name == "c2_sphere192":
        return synth.sphere(192, 3, seed=0)
    if name == "c3_o3_1024":
        return synth.orthogonal_3x3(1024, seed=0)
    if name == "o3_4096":
        return synth.orthogonal_3x3(4096, seed=0)
    if name in ("cube6000", "cube10000", "cube16384"):
        n = int(name[4:])
        return synth.uniform_cube(n, 3, seed=n)
    raise KeyError(name)


def canonical_hash(pairs) -> str:
    rec = np.ascontiguousarray(pairs, dtype=oracle.PAIR_DTYPE)
    return hashlib.sha256(rec.tobytes()).hexdigest()


def make(name):
    cfg = synth.CONFIGS[name]
    X = inputs(name)
    D = oracle.pdist(X)
    t0 = time.time()
    P, cols = oracle.barcode(D, cfg["max_dim"], cfg["threshold"],
                             mode=oracle.M3_REDUCTION_MATRIX, with_columns=True)
    dt = time.time() - t0
    nz = oracle.nonzero(P)
    out = {
        "config": name,
        "generator": (f"paper_2502_05063_amd.synth.uniform_cube({name[4:]}, 3, seed={name[4:]})"
                      if name.startswith("cube") else f"paper_2502_05063_amd.synth ({name}, seed 0)"),
        "max_dim": cfg["max_dim"],
        "threshold": cfg["threshold"] if np.isfinite(cfg["threshold"]) else "inf",
        "enclosing_radius": float(oracle.enclosing_radius(D)),
        "oracle_mode": "M3 streamed reduction matrix (Sec. 5.2.9)",
        "oracle_seconds": round(dt, 1),
        "columns_per_dim": cols,
        "pairs_per_dim": [int((P["dim"] == d).sum()) for d in range(cfg["max_dim"] + 1)],
        "essential_per_dim": [int(((P["dim"] == d) & (P["essential"] == 1)).sum())
                              for d in range(cfg["max_dim"] + 1)],
        "full_list_sha256": canonical_hash(P),
        "nonzero_pairs": [
            [int(p["dim"]), int(p["essential"]), int(p["birth"]), int(p["death"]),
             float(p["birth_diam"]), float(p["death_diam"]) if not p["essential"] else "inf"]
            for p in nz
        ],
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, "done in", round(dt, 1), "s; pairs", out["pairs_per_dim"], flush=True)


def batch_clouds(name):
    if name == "c4_batch256":
        return synth.circle_or_torus_batch(256, 50, 400, 0.05, seed=0)
    if name == "c5_torus64x500":
        return synth.torus_batch(64, 500, 0.1, seed=0)
    raise KeyError(name)


def _one_cloud(args):
    X, max_dim, keep_h1 = args
    P = oracle.barcode(oracle.pdist(X), max_dim)
    rec = {
        "n": int(X.shape[0]),
        "pairs_per_dim": [int((P["dim"] == d).sum()) for d in range(max_dim + 1)],
        "full_list_sha256": canonical_hash(P),
    }
    if keep_h1:
        h1 = oracle.nonzero(P[(P["dim"] == 1) & (P["essential"] == 0)])
        rec["h1_nonzero"] = [[int(p["birth"]), int(p["death"])] for p in h1]
    return rec


def make_batch(name):
    from multiprocessing import Pool

    cfg = synth.CONFIGS[name]
    clouds = batch_clouds(name)
    keep_h1 = name == "c5_torus64x500"
    t0 = time.time()
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        recs = pool.map(_one_cloud, [(X, cfg["max_dim"], keep_h1) for X in clouds], chunksize=1)
    dt = time.time() - t0
    out = {
        "config": name,
        "generator": f"paper_2502_05063_amd.synth ({name}, seed 0)",
        "max_dim": cfg["max_dim"],
        "threshold": "inf",
        "oracle_mode": "M2 streamed (Alg. 12)",
        "oracle_seconds_wall": round(dt, 1),
        "clouds": recs,
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(name, "done in", round(dt, 1), "s;", len(recs), "clouds", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:]:
        if name in ("c4_batch256", "c5_torus64x500"):
            make_batch(name)
        else:
            make(name)
