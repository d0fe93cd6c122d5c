"""The host rank table built from a sorted finite-edge list (the path large
sparse clouds take) against the one built from the full weight matrix, over
a sequence of matrices: the same size twice in a row (only the previous
build's entries are reset), size changes both ways, ties (quantised
distances) and a size with the threaded fill (n >= 2048); and diameter
edges found from ranks alone against those found from the weights. No GPU.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2502_05063_amd", "csrc")
KINF = np.uint32(0xFFFFFFFF)  # the library's "beyond the threshold" weight


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("rt") / "rank_table_driver")
    cmd = [hipcc, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(HERE, "rank_table_driver.cpp"), os.path.join(CSRC, "reduce.cpp"),
           "-lpthread", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def weights(n, thr, seed, quantum=None):
    rng = np.random.default_rng(seed)
    X = rng.random((n, 3))
    D = np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)).astype(np.float32)
    if quantum:
        D = (np.round(D / quantum) * quantum).astype(np.float32)
    W = D.view(np.uint32).copy()
    W[D > np.float32(thr)] = KINF
    np.fill_diagonal(W, KINF)
    return W


def write(path, W):
    with open(path, "wb") as f:
        f.write(np.int32(W.shape[0]).tobytes())
        f.write(np.ascontiguousarray(W, np.uint32).tobytes())


def test_edge_list_table_matches_matrix_table(driver, tmp_path):
    seq = [(300, 0.30, 1, None), (300, 0.20, 2, None), (300, 0.35, 3, 0.05),
           (2100, 0.10, 4, None), (2100, 0.12, 5, None), (300, 0.25, 6, None),
           (40, 10.0, 7, None), (40, 0.3, 8, 0.1)]
    paths = []
    for i, (n, thr, seed, q) in enumerate(seq):
        p = str(tmp_path / f"w{i}.bin")
        write(p, weights(n, thr, seed, q))
        paths.append(p)
    r = subprocess.run([driver, *paths], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
