"""Wall times of the library on its workloads, one JSON line each.

    python -m paper_2502_05063_amd.workloads [names...]

Workloads (synthetic, seeded; see synth.py):
  c1        64 points U[0,1)^3, dimensions 0-1
  c2        192 points on S^3, dimensions 0-3, full threshold
  c2-all    the same, every pair reported (zero persistence included)
  c3        1024 random O(3) matrices in R^9, threshold 1.8, dimensions 0-3
  c4        256 clouds of 50-400 points (noisy circles and tori), dimensions
            0-1, one batch forward (dimension 1 reduced on the device, the
            clouds the cost model deems heaviest on host threads beside it)
  c5        64 noisy tori of 500 points, dimensions 0-1, one batch forward
  c4-device, c5-device
            the same batches with every cloud reduced on the device
  c4-host, c5-host
            the same batches with dimension 1 reduced on host threads
  o3-4096   4096 random O(3) matrices, threshold 1.4, dimensions 0-3 (the
            size of the paper's o3 run)
  cube6000, cube10000, cube16384
            uniform clouds in the unit cube above 4096 points under low
            thresholds (0.09, dimensions 0-2; 0.06 and 0.05, dimensions 0-1)
  boundary  the boundary matrix of a Rips 2-skeleton (2000 points, 0.22)
            through the explicit-matrix path
  graphs    extended persistence of 1024 graphs of 20-300 vertices (mean
            degree 4), one batch
  er-N      extended persistence of one Erdos-Renyi graph G(N, 0.1), N in
            200, 500, 1000, 2000 (the sizes of the paper's Fig. 7.7)

Each line holds the median wall time of the timed calls (after one untimed
call that also fills the autotuner's choices) and the last call's stats.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np


def _timed(fn, reps):
    import torch

    fn()
    torch.cuda.synchronize()
    times, last = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        last = fn()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(times)), last


def run(names=None, reps=3):
    import torch

    from . import synth, vrph

    ctx = vrph.Context(0)
    dev = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    out = []

    def single(name, X, **kw):
        ms, bc = _timed(lambda: ctx.barcode(X=X, **kw), reps)
        rec = {"workload": name, "ms": ms, "stats": bc.stats}
        print(json.dumps(rec), flush=True)
        out.append(rec)

    want = set(names or ["c1", "c2", "c2-all", "c3", "c4", "c5", "o3-4096", "boundary"])
    if "c1" in want:
        single("c1", dev(synth.uniform_cube(64, 3, 0)), max_dim=1)
    if "c2" in want:
        single("c2", dev(synth.sphere(192, 3, 0)), max_dim=3, autotune=True)
    if "c2-all" in want:
        single("c2-all", dev(synth.sphere(192, 3, 0)), max_dim=3, keep_zero=True)
    if "c3" in want:
        single("c3", dev(synth.orthogonal_3x3(1024, 0)), max_dim=3, threshold=1.8, autotune=True)
    if "o3-4096" in want:
        single("o3-4096", dev(synth.orthogonal_3x3(4096, 0)), max_dim=3, threshold=1.4,
               autotune=True)
    for name, cfg in synth.CONFIGS.items():
        if name.startswith("cube") and name in want:
            nn = int(name[4:])
            single(name, dev(synth.uniform_cube(nn, 3, seed=nn)), max_dim=cfg["max_dim"],
                   threshold=cfg["threshold"], autotune=True)
    for name in ("c4", "c4-device", "c4-host", "c5", "c5-device", "c5-host"):
        if name not in want:
            continue
        if name.startswith("c4"):
            clouds = synth.circle_or_torus_batch(256, 50, 400, 0.05, seed=0)
        else:
            clouds = synth.torus_batch(64, 500, 0.1, seed=0)
        b = ctx.batch([len(c) for c in clouds], 3, max_dim=1,
                      host_reduction=name.endswith("-host"),
                      device_reduction=name.endswith("-device"))
        Xb = dev(np.concatenate(clouds))
        ms, res = _timed(lambda: b.forward(Xb), reps)
        rec = {"workload": name, "ms": ms, "stats": res[0].stats,
               "additions": int(sum(r.stats["additions"][1] for r in res)),
               "device_reduced": int(sum(r.stats["device_reduced"] for r in res))}
        print(json.dumps(rec), flush=True)
        out.append(rec)
        b.close()
    if "boundary" in want:
        X = dev(synth.uniform_cube(2000, 3, seed=1))
        ptr, rows = synth.rips2_boundary_csc(ctx.pdist(X).cpu().numpy(), 0.22)
        dptr, drows = dev(ptr), dev(rows)
        ms, (low, st) = _timed(lambda: ctx.boundary_pivots(dptr, drows), reps)
        rec = {"workload": "boundary", "ms": ms, "stats": st, "pivots": int((low >= 0).sum())}
        print(json.dumps(rec), flush=True)
        out.append(rec)
    gsets = []
    if "graphs" in want:
        gsets.append(("graphs",) + synth.graph_batch(1024, 20, 300, 4.0, seed=0))
    for nn in (200, 500, 1000, 2000):
        if f"er-{nn}" in want:
            E, f = synth.erdos_renyi(nn, 0.1, seed=nn)
            gsets.append((f"er-{nn}", [(E, f)], np.array([0, nn]), np.array([0, len(E)])))
    for name, graphs, v_off, e_off in gsets:
        f = dev(np.concatenate([f for _, f in graphs]))
        E = dev(np.concatenate([E for E, _ in graphs]))
        ms, _ = _timed(lambda: ctx.graph_extended(f, E, v_off, e_off, host=False), reps)
        rec = {"workload": name, "ms": ms, "graphs": len(graphs), "vertices": int(v_off[-1]),
               "edges": int(e_off[-1])}
        print(json.dumps(rec), flush=True)
        out.append(rec)
    ctx.close()
    return out


if __name__ == "__main__":
    run(sys.argv[1:] or None)
