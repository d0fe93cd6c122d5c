"""Benchmark of the Vietoris–Rips barcode hot path on one MI355X.

A step is one whole barcode computation (distances, enclosing radius, H0,
enumeration + apparent-pairs test per dimension, coboundary-order sort,
host submatrix reduction, result assembly) of 192 points on S^3 in R^4
(normalised Gaussians, seed 0), dimensions 0..3, full threshold; the points
are resident in HBM before the timed region starts.

Prints one JSON line: the measured step, the roofline view of the dominant
kernel, the oracle baseline and the batched forward+backward comparison.
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "barcode wall time (ms) + simplices/sec and HBM GB/s; batched fwd+bwd clouds/sec vs plain"
# MI355X published peaks used for the roofline
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: 32-bit integer / compare lane-ops
# per second (a wave64 VALU instruction takes a SIMD 4 cycles)
CLOCK_HZ = 2.4e9
SIMDS = 256 * 4
ALU_PEAK_TOPS = SIMDS * 16 * CLOCK_HZ / 1e12


KERNEL_SRC = os.path.join(ROOT, "paper_2502_05063_amd", "csrc", "kernels.hip")
LDS_MAX_N = 200  # clouds up to this size enumerate from the LDS rank matrix
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "enum_apparent_lds_kernel_sphere3_192.md")


def profile_figures(grid):
    """Per-launch counter figures of the dominant kernel from the committed
    rocprofv3 summary: HBM bytes (FETCH_SIZE and WRITE_SIZE, scaled by the
    copy calibration recorded there) and wave64 VALU / SALU instructions
    (SQ_INSTS_VALU, SQ_INSTS_SALU). Empty unless that summary was taken on
    the current kernel source with the same launch grid."""
    try:
        with open(TRAFFIC_SUMMARY) as f:
            text = f.read()
        with open(KERNEL_SRC, "rb") as f:
            src_hash = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return {}
    h = re.search(r"kernels_hip_sha256:\s*([0-9a-f]{64})", text)
    g = re.search(r"grid_workgroups:\s*([0-9]+)", text)
    if not (h and g) or h.group(1) != src_hash or int(g.group(1)) != grid:
        return {}
    out = {}
    for key in ("hbm_bytes_per_launch", "sq_insts_valu_per_launch", "sq_insts_salu_per_launch"):
        m = re.search(key + r":\s*([0-9]+)", text)
        if m:
            out[key] = int(m.group(1))
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# the oracle's sample: the first points of the same S^3 cloud, every dimension
# 0..3 the GPU computes (the oracle's time grows about as n^5 here; all 192
# points take minutes)
CPU_SAMPLE_POINTS = 136


def cpu_baseline(X, max_dim):
    """The oracle as it stands (one thread: its reduction is sequential), on a
    bounded sample of the same workload: the first CPU_SAMPLE_POINTS points of
    the same cloud, dimensions 0..max_dim, full Rips."""
    import oracle

    Xs = X[:CPU_SAMPLE_POINTS]
    n = Xs.shape[0]
    t0 = time.perf_counter()
    D = oracle.pdist(Xs)
    oracle.barcode(D, max_dim, mode=oracle.M3_REDUCTION_MATRIX)
    dt = time.perf_counter() - t0
    # candidates as the GPU counts them: every d-simplex index, d = 0..max_dim
    simplices = sum(math.comb(n, d + 1) for d in range(max_dim + 1))
    return {
        "value": simplices / dt,
        "unit": "simplices/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"first {n} of the same 192 points on S^3, dimensions 0..{max_dim}, full Rips "
                   f"(streamed reduction-matrix mode, one thread), {dt:.1f} s"),
        "host_cpus": os.cpu_count(),
        "cpu_model": cpu_model(),
    }


def _oracle_fwd_bwd(X):
    """One cloud through the oracle: the barcode of dimensions 0-1 and the
    gradient of sum over finite H1 pairs of (death - birth)^2 with respect to
    the points (the batched leg's loss)."""
    import numpy as np

    import oracle

    D = oracle.pdist(X)
    pairs = oracle.barcode(D, 1)
    h1 = pairs[(pairs["dim"] == 1) & (pairs["death"] != np.iinfo(np.uint64).max)]
    g = 2.0 * (h1["death_diam"].astype(np.float64) - h1["birth_diam"].astype(np.float64))
    oracle.gradient(X, D, h1, -g, g)
    return len(h1)


def _oracle_ready(_):
    import oracle

    oracle.lib()
    return 0


def batched_cpu_baseline(clouds):
    """The oracle on a sample of the batched leg's clouds, one cloud per
    process across the host's cores (up to 16), forward and backward."""
    import multiprocessing as mp

    workers = max(1, min(16, os.cpu_count() or 1, len(clouds)))
    sample = clouds[:workers]
    with mp.get_context("spawn").Pool(workers) as pool:
        pool.map(_oracle_ready, range(4 * workers), chunksize=1)  # workers up, oracle loaded
        t0 = time.perf_counter()
        pool.map(_oracle_fwd_bwd, sample, chunksize=1)
        dt = time.perf_counter() - t0
    return {"value": len(sample) / dt, "unit": "clouds/s", "cores": workers, "kind": "oracle",
            "sample": (f"the first {len(sample)} of the 64 tori, one per process, barcode of "
                       f"dimensions 0-1 and the loss gradient, {dt:.1f} s"),
            "cpu_model": cpu_model()}


def batched_vs_plain(ctx, steps, cpu_leg=True):
    """Forward + backward of loss = sum over H1 of (death - birth)^2 on 64 noisy
    tori of 500 points (sigma 0.1), through torch.autograd on the same GPU:
    the batched forward (captured graphs; dimension 1 reduced on the device
    for most clouds, while host threads reduce the ones the cost model deems
    heaviest), the same batch with every cloud reduced on the device, and
    with every cloud reduced on host threads, and a per-cloud loop of the
    single-cloud path (whose reduction runs on the host)."""
    import numpy as np
    import torch

    from paper_2502_05063_amd import synth
    from paper_2502_05063_amd.autograd import batch_persistence, cloud_persistence

    clouds = synth.torus_batch(64, 500, 0.1, seed=0)
    X = torch.from_numpy(np.concatenate(clouds)).cuda().requires_grad_(True)
    sizes = [len(c) for c in clouds]
    # the first plan tunes its launch settings on its first forward (the
    # untimed warm-up below); the device-only plan, made after it, reads them
    plans = {}
    make = {"batched": lambda: ctx.batch(sizes, 3, max_dim=1, autotune=True),
            "batched_device_reduction": lambda: ctx.batch(sizes, 3, max_dim=1,
                                                          device_reduction=True),
            "batched_host_reduction": lambda: ctx.batch(sizes, 3, max_dim=1, host_reduction=True)}

    def batched_leg(key):
        def run():
            if key not in plans:
                plans[key] = make[key]()
            batched(plans[key])()
        return run

    def batched(b):
        def run():
            bi, d, _ = batch_persistence(X, b, 1)
            ((d - bi) ** 2).sum().backward()
        return run

    parts = [torch.from_numpy(c).cuda().requires_grad_(True) for c in clouds]

    def plain():
        for Xi in parts:
            b, d = cloud_persistence(Xi, ctx, 1)
            ((d - b) ** 2).sum().backward()

    out = {}
    for name, fn in (("batched", batched_leg("batched")),
                     ("batched_device_reduction", batched_leg("batched_device_reduction")),
                     ("batched_host_reduction", batched_leg("batched_host_reduction")),
                     ("plain", plain)):
        fn()
        # the garbage of earlier legs is collected before, not inside, the
        # timed steps (the collector stays on while they run)
        gc.collect()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            fn()
            print(f"{name} fwd+bwd {i} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[f"{name}_ms"] = dt * 1e3
        out[f"{name}_clouds_per_s"] = len(clouds) / dt
    out["speedup"] = out["plain_ms"] / out["batched_ms"]
    out["speedup_device_reduction"] = out["plain_ms"] / out["batched_device_reduction_ms"]
    out["speedup_host_reduction"] = out["plain_ms"] / out["batched_host_reduction_ms"]
    for key, b in plans.items():
        res = b.forward(X.detach())
        out[f"{key}_graph_ms"] = res[0].stats["gpu_ms"][0]
        out[f"{key}_host_ms"] = res[0].stats["host_ms"][1]
        out[f"{key}_forward_total_ms"] = res[0].stats["total_ms"]
        out[f"{key}_device_reduced_clouds"] = int(sum(r.stats["device_reduced"] for r in res))
    out["host_threads_batched_host_reduction"] = min(16, os.cpu_count() or 1)
    out["workload"] = "64 noisy tori x 500 points in R^3 (sigma 0.1), dims 0-1, loss sum (death-birth)^2 over H1"
    if cpu_leg:
        out["cpu_baseline"] = batched_cpu_baseline(clouds)
    for b in plans.values():
        b.close()
    return out


def graph_extended(ctx, reps=5):
    """Extended persistence of graphs (Sec. 7.2, Alg. 27), batched as a graph
    readout would call it: 1024 Erdos-Renyi graphs of 20-300 vertices with
    mean degree 4 and standard normal vertex values (seed 0), one call for
    the batch; the oracle (Alg. 2 on the coned graph's boundary matrix, one
    thread) timed on the first 64 graphs."""
    import numpy as np
    import torch

    import oracle.graph_ext as gx
    from paper_2502_05063_amd import synth

    graphs, v_off, e_off = synth.graph_batch(1024, 20, 300, 4.0, seed=0)
    f = torch.from_numpy(np.concatenate([f for _, f in graphs])).cuda()
    E = torch.from_numpy(np.concatenate([E for E, _ in graphs])).cuda()
    ctx.graph_extended(f, E, v_off, e_off, host=False)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        ctx.graph_extended(f, E, v_off, e_off, host=False)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    ms = float(np.median(times))
    sample = 64
    t0 = time.perf_counter()
    for Eg, fg in graphs[:sample]:
        gx.extended_persistence(len(fg), [tuple(e) for e in Eg], fg)
    cpu_s = time.perf_counter() - t0
    return {"workload": "1024 G(n, 4/(n-1)) graphs, n uniform in 20..300, N(0,1) vertex values",
            "vertices": int(v_off[-1]), "edges": int(e_off[-1]), "ms": ms,
            "graphs_per_s": len(graphs) / (ms / 1e3),
            "cpu_baseline": {"graphs_per_s": sample / cpu_s, "cores": 1, "kind": "oracle",
                             "sample": f"first {sample} graphs, {cpu_s:.2f} s"}}


def boundary_scan(ctx, reps=3):
    """The explicit-matrix workload: the boundary matrix of the Rips
    2-skeleton of 2000 points uniform in the unit cube (seed 1), edges and
    triangles up to 0.22, through vrph_boundary_pivots. The scan kernels are
    HBM-streaming: their algorithmic bytes are 38 B per column (offsets read
    twice, left/lookup/stable initialised, the lowest row and its leftmost
    column read) + 16 B per entry (the row read, the 4-byte atomic minimum
    read and written) + 6 B per scan pivot + 8 B per unstable column."""
    import numpy as np
    import torch

    from paper_2502_05063_amd import synth

    X = torch.from_numpy(synth.uniform_cube(2000, 3, seed=1)).cuda()
    D = ctx.pdist(X).cpu().numpy()
    ptr, rows = synth.rips2_boundary_csc(D, 0.22)
    dptr, drows = torch.from_numpy(ptr).cuda(), torch.from_numpy(rows).cuda()
    ctx.boundary_pivots(dptr, drows)
    runs = []
    for _ in range(reps):
        t0 = time.perf_counter()
        low, st = ctx.boundary_pivots(dptr, drows)
        runs.append((st["scan_ms"], (time.perf_counter() - t0) * 1e3, st))
    runs.sort(key=lambda r: r[0])
    scan_ms, wall_ms, st = runs[len(runs) // 2]
    # the same call without the compression step (same pivots), for comparison
    _, plain = ctx.boundary_pivots(dptr, drows, compression=False)
    ncols, nnz = len(ptr) - 1, len(rows)
    alg = 38 * ncols + 16 * nnz + 6 * st["scan_pivots"] + 8 * st["unstable"]
    gbs = alg / (scan_ms / 1e3) / 1e9
    return {"workload": "Rips 2-skeleton boundary matrix, 2000 points U[0,1)^3 (seed 1), tau 0.22",
            "columns": ncols, "nnz": nnz, "scan_ms": scan_ms, "call_ms": wall_ms,
            "host_ms": st["host_ms"], "stable": st["stable"], "unstable": st["unstable"],
            "scan_pivots": st["scan_pivots"], "additions": st["additions"],
            "compress_additions": st["compress_additions"], "compressed": st["compressed"],
            "no_compression": {"host_ms": plain["host_ms"], "additions": plain["additions"]},
            "pivots": int((low >= 0).sum()),
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes": alg}}


def full_sort_ab(ctx, Xd, max_dim, fused_stats, reps=3):
    """The fusion of the apparent-pairs test into the enumeration against the
    paper's unfused order (every column written, sorted into coboundary
    order, then tested; VRPH_FULL_SORT) on the same input: per dimension the
    device time of the fused kernel and of the three unfused stages (HIP
    events around them, stats apparent_ms), and the barcode wall times."""
    import numpy as np

    ctx.barcode(X=Xd, max_dim=max_dim, full_sort=True)  # buffers, code objects
    runs = [ctx.barcode(X=Xd, max_dim=max_dim, full_sort=True).stats for _ in range(reps)]
    dims = range(2, max_dim + 1)
    fused = {d: float(np.mean([s["apparent_ms"][d] for s in fused_stats])) for d in dims}
    unfused = {d: float(np.mean([s["apparent_ms"][d] for s in runs])) for d in dims}
    return {"workload": "the bench's cloud; dimensions 2-3 (the kernels that read the rank matrix from LDS)",
            "columns_per_dim": {d: runs[-1]["columns"][d] for d in dims},
            "fused_ms_per_dim": fused,
            "unfused_ms_per_dim": unfused,
            "unfused_over_fused": {d: unfused[d] / fused[d] for d in dims},
            "barcode_ms_fused": float(np.mean([s["total_ms"] for s in fused_stats])),
            "barcode_ms_unfused": float(np.mean([s["total_ms"] for s in runs]))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-boundary", action="store_true")
    ap.add_argument("--no-graphs", action="store_true")
    ap.add_argument("--no-full-sort", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (the reference for HBM counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch

        src = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                          "copies": 3}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "clouds, or the index ranges of one cloud's dimensions, would be split "
              "across GPUs with one process per GPU.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2502_05063_amd import synth, vrph

    n, max_dim = 192, 3
    X = synth.sphere(n, 3, seed=0)
    Xd = torch.from_numpy(X).cuda()
    ctx = vrph.Context(0)
    for i in range(args.warmup):
        # the first warm-up step runs the launch autotuner; its choice is cached
        # in the context and reused by every later step
        bc = ctx.barcode(X=Xd, max_dim=max_dim, autotune=(i == 0))
        print(f"warmup {i}: {bc.stats['total_ms']:.1f} ms", file=sys.stderr, flush=True)
    gc.collect()  # before, not inside, the timed steps (the collector stays on)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        bc = ctx.barcode(X=Xd, max_dim=max_dim)
        stats.append(bc.stats)
        print(f"step {i}: {bc.stats['total_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) / args.steps * 1e3
    s0 = stats[-1]
    simplices = sum(s0["candidates"])
    value = simplices / (ms / 1e3)

    # dominant kernel: the dimension-3 enumeration + apparent-pairs kernel.
    # It is bound by VALU instruction issue (integer compares, index
    # arithmetic and control of the apparent-pairs test on 64-wide waves), not
    # by HBM: its operands come from a rank matrix staged in LDS. Its roofline
    # is the 32-bit VALU lane-op rate, and `achieved` counts the integer
    # compares the apparent-pairs test needs (Lemma 5.3.6): C(d+1,2) per
    # candidate for its diameter, d+1 per cofacet the scan examines, C(d+1,2)
    # per facet whose diameter the second condition computes.
    d = max_dim
    k_ms = float(np.mean([s["apparent_ms"][d] for s in stats]))
    cand, cof, fac = s0["candidates"][d], s0["cofacets"][d], s0["facets"][d]
    cols, app, nonapp = s0["columns"][d], s0["apparent"][d], s0["reduced"][d]
    ops = cand * math.comb(d + 1, 2) + cof * (d + 1) + fac * math.comb(d + 1, 2)
    achieved_tops = ops / (k_ms / 1e3) / 1e12
    # Bytes an unfused design would move for the same result (Sec. 5.5: an
    # 8-byte key written by the enumeration and read back by the
    # apparent-pairs test per column, 16 bytes per apparent pair, 8 per
    # non-apparent column, 1 clearing bit per candidate and, when a next
    # dimension exists, per apparent pair). The fused kernel does not move
    # them: this is an equivalent rate, not HBM traffic.
    alg_bytes = (cand / 8 + cols * 8 + cols * 8 + app * 16 + nonapp * 8
                 + (app / 8 if d < max_dim else 0))
    equiv_gbs = alg_bytes / (k_ms / 1e3) / 1e9
    prof = profile_figures(s0["grid"][d])
    traffic = prof.get("hbm_bytes_per_launch")
    valu = prof.get("sq_insts_valu_per_launch")
    salu = prof.get("sq_insts_salu_per_launch")
    # issue capacity: one wave64 VALU instruction per SIMD every 4 cycles
    simd_cycles = SIMDS * CLOCK_HZ * (k_ms / 1e3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "simplices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sphere_3_192-like: 192 points on S^3 (seed 0), dims 0-3, full Rips",
                   "n": n, "max_dim": max_dim, "threshold": "inf"},
        "barcode_ms": ms,
        "kernel_ms_per_dim": [float(np.mean([s["apparent_ms"][k] for s in stats])) for k in range(d + 1)],
        "gpu_ms_per_dim": [float(np.mean([s["gpu_ms"][k] for s in stats])) for k in range(d + 1)],
        "host_ms_per_dim": [float(np.mean([s["host_ms"][k] for s in stats])) for k in range(d + 1)],
        "columns_per_dim": s0["columns"],
        "apparent_per_dim": s0["apparent"],
        "emergent_per_dim": s0["emergent"],
        "reduced_per_dim": s0["reduced"],
        "additions_per_dim": s0["additions"],
        "roofline": {"bound": "alu", "achieved": achieved_tops, "peak": ALU_PEAK_TOPS,
                     "unit": "TOP/s", "frac": achieved_tops / ALU_PEAK_TOPS, "traffic": traffic,
                     # the top dimension's variant: bitmap clearing set in, dense unit
                     # tables, no clearing set out and no pair output (mode bits 4)
                     "kernel": (f"enum_apparent_lds_kernel<{d}, 4>" if n <= LDS_MAX_N
                                else f"enum_apparent_kernel<{d}, 4>"), "kernel_ms": k_ms,
                     "ops_per_launch": ops,
                     "grid_workgroups": s0["grid"][d],
                     "valu_issue": ({"sq_insts_valu_per_launch": valu,
                                     "sq_insts_salu_per_launch": salu,
                                     "frac": valu * 4 / simd_cycles} if valu else None),
                     "hbm_measured": ({"gbs": traffic / (k_ms / 1e3) / 1e9,
                                       "frac": traffic / (k_ms / 1e3) / 1e9 / HBM_PEAK_GBS}
                                      if traffic else None),
                     "hbm_algorithmic_equivalent": {"bytes_per_launch": alg_bytes,
                                                    "gbs": equiv_gbs,
                                                    "frac": equiv_gbs / HBM_PEAK_GBS}},
    }
    if not args.no_batched:
        out["batched_fwd_bwd"] = batched_vs_plain(ctx, max(2, min(args.steps, 5)),
                                                  cpu_leg=not args.no_cpu_baseline)
    if not args.no_boundary:
        out["boundary_scan"] = boundary_scan(ctx)
    if not args.no_graphs:
        out["graph_extended"] = graph_extended(ctx)
    if not args.no_full_sort:
        out["full_sort_ab"] = full_sort_ab(ctx, Xd, max_dim, stats)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(X, max_dim)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
