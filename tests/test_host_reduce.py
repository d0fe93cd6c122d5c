"""The host submatrix reduction on its own (no GPU): host_reduce_driver.cpp
runs the product's reduce_dimension on columns it selects on the host, on
one thread and on several with every block forced onto all threads. The
pairs must be the same, in the same order, on any thread count (the
parallel pass makes exactly the sequential additions), and together with
the apparent pairs they must be the oracle's pairs of dimensions >= 1.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2502_05063_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2502_05063_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("drv") / "host_reduce_driver")
    cmd = [hipcc, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(HERE, "host_reduce_driver.cpp"), os.path.join(CSRC, "reduce.cpp"),
           "-lpthread", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def run(driver, path, max_dim, tau, threads, wide):
    r = subprocess.run([driver, path, str(max_dim), repr(float(tau)), str(threads),
                        "1" if wide else "0"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    return r.stdout


def as_set(text):
    out = set()
    for line in text.splitlines():
        d, b, t, bb, tb = (int(x) for x in line.split())
        ess = t == 2**64 - 1
        out.add((d, b, -1 if ess else t, bb, -1 if ess else tb))
    return out


def oracle_set(D, max_dim, thr):
    out = set()
    for p in oracle.barcode(D, max_dim, threshold=thr):
        if p["dim"] == 0:
            continue
        bb = int(np.float32(p["birth_diam"]).view(np.uint32))
        if p["essential"]:
            out.add((int(p["dim"]), int(p["birth"]), -1, bb, -1))
        else:
            tb = int(np.float32(p["death_diam"]).view(np.uint32))
            out.add((int(p["dim"]), int(p["birth"]), int(p["death"]), bb, tb))
    return out


CASES = [
    ("sphere", 56, 3, float("inf")),
    ("cube", 120, 2, float("inf")),
    ("o3", 90, 3, 1.9),
    ("torus", 200, 2, 1.2),
]


@pytest.mark.parametrize("name,n,max_dim,thr", CASES)
def test_thread_counts_agree_and_match_oracle(driver, tmp_path, name, n, max_dim, thr):
    if name == "sphere":
        X = synth.sphere(n, 3, seed=n)
    elif name == "cube":
        X = synth.uniform_cube(n, 3, seed=n)
    elif name == "o3":
        X = synth.orthogonal_3x3(n, seed=n)
    else:
        X = synth.torus(n, 2.0, 0.5, 0.05, np.random.default_rng(n))
    D = oracle.pdist(X)
    tau = min(thr, oracle.enclosing_radius(D))
    path = str(tmp_path / "m.bin")
    with open(path, "wb") as f:
        f.write(np.int32(n).tobytes())
        f.write(np.ascontiguousarray(D, np.float32).tobytes())
    one = run(driver, path, max_dim, tau, 1, False)
    assert one.strip(), "no pairs"
    # the threads race differently on every run: several runs per count
    for threads in (2, 8, 8, 16, 16, 16):
        assert run(driver, path, max_dim, tau, threads, True) == one, f"{threads} threads"
    assert run(driver, path, max_dim, tau, 8, False) == one
    assert as_set(one) == oracle_set(D, max_dim, thr)


# ---------------------------------------------------------------------------
# the explicit-matrix path's host part (reduce_explicit_columns)


@pytest.fixture(scope="module")
def explicit_driver(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("edrv") / "explicit_reduce_driver")
    cmd = [hipcc, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(HERE, "explicit_reduce_driver.cpp"), os.path.join(CSRC, "reduce.cpp"),
           "-lpthread", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def write_csc(path, ptr, rows):
    with open(path, "wb") as f:
        f.write(np.int64(len(ptr) - 1).tobytes())
        f.write(np.ascontiguousarray(ptr, np.int64).tobytes())
        f.write(np.ascontiguousarray(rows, np.int64).tobytes())


def run_explicit(drv, path, threads, wide, clearing, compression=False, counts=False):
    r = subprocess.run([drv, path, str(threads), "1" if wide else "0", "1" if clearing else "0",
                        "1" if compression else "0"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    low = np.array([int(x) for x in r.stdout.split()], np.int64)
    if not counts:
        return low
    info = {}
    for line in r.stderr.splitlines():
        w = line.split()
        if w[0] == "compression":
            info["compress_additions"], info["removed"] = int(w[2]), int(w[4])
        elif w[0] == "additions":
            info["additions"] = int(w[1])
    return low, info


@pytest.mark.parametrize("case", ["rips", "random"])
def test_explicit_thread_counts_agree_and_match_oracle(explicit_driver, tmp_path, case):
    if case == "rips":
        D = oracle.pdist(synth.uniform_cube(500, 3, seed=4))
        ptr, rows = synth.rips2_boundary_csc(D, 0.2)
        clearing = True
    else:  # any strictly upper triangular matrix, without clearing
        rng = np.random.default_rng(6)
        cols = []
        for j in range(6000):
            k = min(j, rng.binomial(j, 0.0006)) if j else 0
            cols.append(np.sort(rng.choice(j, size=k, replace=False)) if k else np.zeros(0, np.int64))
        ptr = np.concatenate([[0], np.cumsum([len(c) for c in cols])]).astype(np.int64)
        rows = np.concatenate(cols).astype(np.int64)
        clearing = False
    path = str(tmp_path / "m.bin")
    write_csc(path, ptr, rows)
    one = run_explicit(explicit_driver, path, 1, False, clearing)
    for threads in (2, 8, 16, 16):
        assert np.array_equal(run_explicit(explicit_driver, path, threads, True, clearing), one)
    cols = [rows[ptr[j]:ptr[j + 1]].tolist() for j in range(len(ptr) - 1)]
    assert np.array_equal(one, oracle.reduce_explicit(cols))


# Compression (Sec. 4.3.3, Alg. 8-9) must leave every pivot of Alg. 2 as it
# is: the pivots with compression, on any thread count, equal the oracle's
# plain Alg. 2 on the uncompressed matrix.
@pytest.mark.parametrize("n,tau,seed", [(500, 0.2, 4), (300, 0.35, 9), (120, 0.6, 2)])
def test_compression_keeps_the_pivots(explicit_driver, tmp_path, n, tau, seed):
    D = oracle.pdist(synth.uniform_cube(n, 3, seed=seed))
    ptr, rows = synth.rips2_boundary_csc(D, tau)
    path = str(tmp_path / "m.bin")
    write_csc(path, ptr, rows)
    cols = [rows[ptr[j]:ptr[j + 1]].tolist() for j in range(len(ptr) - 1)]
    ref = oracle.reduce_explicit(cols)
    plain, p_info = run_explicit(explicit_driver, path, 1, False, True, False, counts=True)
    comp, c_info = run_explicit(explicit_driver, path, 1, False, True, True, counts=True)
    assert np.array_equal(plain, ref)
    assert np.array_equal(comp, ref)
    for threads in (2, 8, 16):
        assert np.array_equal(run_explicit(explicit_driver, path, threads, True, True, True), ref)
    # the compression does work of its own and leaves the reduction less
    assert c_info["removed"] + c_info["compress_additions"] > 0
    assert c_info["additions"] <= p_info["additions"]
