"""The host code and the oracle under the address and undefined-behaviour
sanitizers (no GPU): the host reduction (tests/host_reduce_driver.cpp), the
explicit-matrix reduction with compression
(tests/explicit_reduce_driver.cpp) and the rank table built from edge lists
(tests/rank_table_driver.cpp) over reduce.cpp, and the C oracle
(tests/oracle_driver.c), built with -fsanitize=address,undefined for the
host only and run on small inputs on several thread counts. A report from
either sanitizer (or a leak) fails the test; the results must still equal
the oracle's."""
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
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
# host-only sanitizers on the hipcc lines (the drivers hold no device code)
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]


def _hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        pytest.skip("hipcc not available")
    return exe


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    out = {}
    for name in ("host_reduce_driver", "explicit_reduce_driver", "rank_table_driver"):
        exe = str(d / name)
        cmd = [_hipcc(), "-O1", "-g", "-std=c++17", *HOST_SAN, "-I", os.path.join(ROOT, "include"),
               "-I", CSRC, os.path.join(HERE, name + ".cpp"), os.path.join(CSRC, "reduce.cpp"),
               "-lpthread", "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        out[name] = exe
    exe = str(d / "oracle_driver")
    cc = shutil.which("gcc") or "cc"
    r = subprocess.run([cc, "-O1", "-g", "-std=c11", "-ffp-contract=off",
                        "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                        "-I", os.path.join(ROOT, "oracle"), os.path.join(HERE, "oracle_driver.c"),
                        os.path.join(ROOT, "oracle", "vr_oracle.c"), "-lm", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out["oracle_driver"] = exe
    return out


def _run(args):
    r = subprocess.run(args, capture_output=True, text=True, timeout=600, env=SAN_ENV)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    return r.stdout


def _write_dist(path, D):
    with open(path, "wb") as f:
        f.write(np.int32(D.shape[0]).tobytes())
        f.write(np.ascontiguousarray(D, np.float32).tobytes())


def _pairs(text):
    return sorted(tuple(int(x) for x in line.split()) for line in text.splitlines())


@pytest.mark.parametrize("name,n,max_dim", [("torus", 60, 2), ("cube", 40, 3)])
def test_host_reduction_clean(drivers, tmp_path, name, n, max_dim):
    X = synth.torus_batch(1, n, 0.1, seed=3)[0] if name == "torus" else synth.uniform_cube(n, 3, 5)
    D = oracle.pdist(X)
    tau = float(oracle.enclosing_radius(D))
    path = str(tmp_path / "d.bin")
    _write_dist(path, D)
    one = _run([drivers["host_reduce_driver"], path, str(max_dim), repr(tau), "1", "0"])
    for threads in (4, 8):
        assert _pairs(_run([drivers["host_reduce_driver"], path, str(max_dim), repr(tau),
                            str(threads), "1"])) == _pairs(one)
    # the pairs of dimensions >= 1 (zero persistence included) are the oracle's
    ref = oracle.barcode(D, max_dim)
    ref = ref[ref["dim"] >= 1]
    got = _pairs(one)
    assert [(p[0], p[1]) for p in got] == sorted((int(r["dim"]), int(r["birth"])) for r in ref)


def test_explicit_reduction_clean(drivers, tmp_path):
    D = oracle.pdist(synth.uniform_cube(150, 3, seed=4))
    ptr, rows = synth.rips2_boundary_csc(D, 0.35)
    path = str(tmp_path / "m.bin")
    with open(path, "wb") as f:
        f.write(np.int64(len(ptr) - 1).tobytes())
        f.write(np.ascontiguousarray(ptr, np.int64).tobytes())
        f.write(np.ascontiguousarray(rows, np.int64).tobytes())
    cols = [rows[ptr[j]:ptr[j + 1]].tolist() for j in range(len(ptr) - 1)]
    ref = oracle.reduce_explicit(cols)
    for threads, wide, comp in ((1, "0", "0"), (8, "1", "0"), (1, "0", "1"), (8, "1", "1")):
        out = _run([drivers["explicit_reduce_driver"], path, str(threads), wide, "1", comp])
        assert np.array_equal(np.array([int(x) for x in out.split()]), ref)


@pytest.mark.parametrize("n,max_dim,thr", [(24, 2, "inf"), (24, 3, "0.6"), (30, 1, "inf")])
def test_oracle_clean(drivers, tmp_path, n, max_dim, thr):
    D = oracle.pdist(synth.uniform_cube(n, 3, seed=n))
    path = str(tmp_path / "d.bin")
    _write_dist(path, D)
    out = _run([drivers["oracle_driver"], path, str(max_dim), thr])
    assert int(out.split()[0]) == len(oracle.barcode(D, max_dim, float(thr)))


def test_rank_table_from_edges_clean(drivers, tmp_path):
    """The edge-list rank table over a sequence of matrices (same size twice,
    then a size change), checked against the matrix-built table."""
    paths = []
    for i, (n, thr, seed) in enumerate([(200, 0.3, 1), (200, 0.2, 2), (90, 0.5, 3)]):
        rng = np.random.default_rng(seed)
        X = rng.random((n, 3))
        D = np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1)).astype(np.float32)
        W = D.view(np.uint32).copy()
        W[D > np.float32(thr)] = np.uint32(0xFFFFFFFF)
        np.fill_diagonal(W, np.uint32(0xFFFFFFFF))
        p = str(tmp_path / f"w{i}.bin")
        with open(p, "wb") as f:
            f.write(np.int32(n).tobytes())
            f.write(W.tobytes())
        paths.append(p)
    assert _run([drivers["rank_table_driver"], *paths]).strip() == "ok"
