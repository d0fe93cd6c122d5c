"""Write full-size expected values with the CPU oracle (and nothing else).

For a configuration, runs the oracle's streamed reduction-matrix mode (every
column reduced, no apparent-pair shortcut; Alg. 12 alone cannot finish the
S^3 input) on the seeded synthetic input and stores:
the counts of pairs per dimension, every pair of nonzero persistence, and a
SHA-256 of the full canonical pair list (32-byte records: dim, essential,
birth, death, birth_diam, death_diam) so that a GPU result including every
zero-persistence pair can be compared bit for bit.

    python tests/golden/make_golden.py c2_sphere192 c3_o3_1024
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
        "generator": f"paper_2502_05063_amd.synth ({name}, seed 0)",
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


if __name__ == "__main__":
    for name in sys.argv[1:]:
        make(name)
