"""Error paths and determinism on the GPU.

- A batch plan whose buffers exceed the device's memory fails with
  VRPH_ENOMEM, frees what it had allocated, and the context keeps working.
- Calls that wait for their stream refuse, with VRPH_ESTATE, to run on a
  stream under capture (nothing is recorded into the caller's graph).
- Ten runs of the same input give byte-identical results: a single cloud
  (default and autotuned launches, all pairs reported) and batches (reduced
  on the device and on host threads).
"""
import numpy as np
import pytest

from paper_2502_05063_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2502_05063_amd import vrph

    assert torch.cuda.is_available()
    c = vrph.Context()
    yield c
    c.close()


def test_batch_plan_beyond_device_memory(ctx):
    import os

    import torch

    from paper_2502_05063_amd import vrph

    # 300 clouds of 4096 points: the device reduction's triangle bitmaps
    # alone are C(4096, 3) bits = 1.4 GB per cloud, 429 GB in all, more than
    # the device has: refused before anything is allocated
    free0, _ = torch.cuda.mem_get_info()
    with pytest.raises(vrph.VrphError) as ei:
        ctx.batch([4096] * 300, 3, max_dim=1)
    assert ei.value.status == vrph.ENOMEM
    # a cap below what a small plan needs
    clouds = synth.torus_batch(3, 80, 0.1, seed=1)
    os.environ["VRPH_WORKSPACE_CAP"] = "100000"
    try:
        with pytest.raises(vrph.VrphError) as ei:
            ctx.batch([len(c) for c in clouds], 3, max_dim=1)
        assert ei.value.status == vrph.ENOMEM
    finally:
        del os.environ["VRPH_WORKSPACE_CAP"]
    free1, _ = torch.cuda.mem_get_info()
    assert free1 >= free0 - (64 << 20), (free0, free1)
    # without the cap the same plan works
    b = ctx.batch([len(c) for c in clouds], 3, max_dim=1)
    res = b.forward(torch.from_numpy(np.concatenate(clouds)).cuda())
    assert len(res) == 3 and all(len(r.pairs) > 0 for r in res)
    b.close()


def test_calls_under_stream_capture_refuse(ctx):
    import torch

    from paper_2502_05063_amd import vrph

    clouds = synth.torus_batch(2, 60, 0.1, seed=2)
    X = torch.from_numpy(np.concatenate(clouds)).cuda()
    b = ctx.batch([len(c) for c in clouds], 3, max_dim=1)
    X1 = X[:60].contiguous()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    errors = []
    with torch.cuda.stream(s):
        g.capture_begin()
        try:
            for call in (lambda: b.forward(X), lambda: ctx.barcode(X=X1, max_dim=1)):
                try:
                    call()
                    errors.append(None)
                except vrph.VrphError as e:
                    errors.append(e.status)
        finally:
            g.capture_end()
    torch.cuda.synchronize()
    assert errors == [vrph.ESTATE, vrph.ESTATE]
    # and outside the capture both work
    assert len(b.forward(X)) == 2
    assert len(ctx.barcode(X=X1, max_dim=1).pairs) > 0
    b.close()


def _bytes(pairs):
    return np.ascontiguousarray(pairs).tobytes()


@pytest.mark.parametrize("autotune", [False, True], ids=["default", "autotuned"])
def test_single_cloud_ten_runs_identical(ctx, autotune):
    import torch

    X = torch.from_numpy(synth.sphere(120, 3, seed=5)).cuda()
    runs = {_bytes(ctx.barcode(X=X, max_dim=3, keep_zero=True, autotune=autotune).pairs)
            for _ in range(10)}
    assert len(runs) == 1


@pytest.mark.parametrize("host", [False, True], ids=["device_reduction", "host_reduction"])
def test_batch_ten_runs_identical(ctx, host):
    import torch

    clouds = synth.circle_or_torus_batch(24, 50, 200, 0.05, seed=9)
    b = ctx.batch([len(c) for c in clouds], 3, max_dim=1, keep_zero=True, host_reduction=host)
    X = torch.from_numpy(np.concatenate(clouds)).cuda()
    runs = set()
    for _ in range(10):
        res = b.forward(X)
        runs.add(b"".join(_bytes(r.pairs) for r in res))
    b.close()
    assert len(runs) == 1
