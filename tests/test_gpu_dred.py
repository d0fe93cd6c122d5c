"""The dimension-1 submatrix reduction on the device (batches) against the
host reduction of the same columns and against the oracle, and the split
forward (the clouds the cost model picks reduced on host threads while the
device reduces the others) against both.

Pairs (with their edges), the additions made and the columns paired without
any addition must be the same as on the host, which makes the same
additions as the column-by-column Alg. 2 with the reduction-matrix
technique; every cloud must also equal the oracle. Inputs cover ties (lattice
points: many equal distances), a finite threshold (essential classes in
dimension 1), graph replays with new data (the working bitmaps and counts
must return to zero), and the overflow paths (toggle log, V log, V arena:
the last hands the cloud to the host).
"""
import os

import numpy as np
import pytest

import oracle
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


def packed(clouds):
    import torch

    return torch.from_numpy(np.ascontiguousarray(np.concatenate(clouds), np.float32)).cuda()


def strip(pairs):
    out = np.empty(len(pairs), oracle.PAIR_DTYPE)
    for f in oracle.PAIR_DTYPE.names:
        out[f] = pairs[f]
    return out


def lattice(k, jitter_seed=None):
    g = np.stack(np.meshgrid(*[np.arange(k)] * 3, indexing="ij"), -1).reshape(-1, 3)
    X = g.astype(np.float32) * 0.25
    if jitter_seed is not None:
        rng = np.random.default_rng(jitter_seed)
        X = X[rng.permutation(len(X))]
    return np.ascontiguousarray(X)


def run_both(ctx, clouds, **kw):
    """Device-only and host-only reductions of the same batch; the split
    forward is checked against the host one here too."""
    sizes = [len(c) for c in clouds]
    dev = ctx.batch(sizes, 3, max_dim=1, device_reduction=True, **kw)
    host = ctx.batch(sizes, 3, max_dim=1, host_reduction=True, **kw)
    split = ctx.batch(sizes, 3, max_dim=1, **kw)
    try:
        Xp = packed(clouds)
        rd, rh = dev.forward(Xp), host.forward(Xp)
        for _ in range(2):  # the second forward uses the ratio the first measured
            check_split(split.forward(Xp), rh)
        return rd, rh
    finally:
        dev.close()
        host.close()
        split.close()


def check_split(rs, rh):
    for i, (a, b) in enumerate(zip(rs, rh)):
        assert np.array_equal(a.pairs, b.pairs), f"cloud {i}: pairs differ (split)"
        assert a.stats["reduced"] == b.stats["reduced"], i
        assert a.stats["additions"] == b.stats["additions"], i
        assert a.stats["emergent"] == b.stats["emergent"], i


def check_same(rd, rh, expect_device=True):
    for i, (a, b) in enumerate(zip(rd, rh)):
        assert np.array_equal(a.pairs, b.pairs), f"cloud {i}: pairs differ"
        assert a.stats["reduced"] == b.stats["reduced"], i
        assert a.stats["additions"] == b.stats["additions"], (i, a.stats["additions"],
                                                              b.stats["additions"])
        assert a.stats["emergent"] == b.stats["emergent"], i
        assert b.stats["device_reduced"] == 0
        if expect_device:
            assert a.stats["device_reduced"] == 1, i


@pytest.mark.parametrize("case", ["tori", "lattice", "threshold", "keep_zero"])
def test_device_matches_host_and_oracle(ctx, case):
    kw = {}
    if case == "tori":
        clouds = synth.circle_or_torus_batch(12, 30, 160, 0.05, seed=5)
    elif case == "lattice":
        clouds = [lattice(4), lattice(5, jitter_seed=1), lattice(3, jitter_seed=2)]
    elif case == "threshold":
        clouds = synth.torus_batch(5, 140, 0.1, seed=6)
        kw["threshold"] = 0.9
    else:
        clouds = synth.circle_or_torus_batch(6, 40, 120, 0.05, seed=7)
        kw["keep_zero"] = True
    rd, rh = run_both(ctx, clouds, **kw)
    check_same(rd, rh)
    thr = kw.get("threshold", float("inf"))
    for i, X in enumerate(clouds):
        ref = oracle.barcode(oracle.pdist(X), 1, thr)
        if not kw.get("keep_zero"):
            ref = oracle.nonzero(ref)
        assert np.array_equal(strip(rd[i].pairs), ref), f"cloud {i} vs oracle"
    if case == "threshold":
        # below the enclosing radius: dimension 1 keeps essential classes
        assert any(((r.dim(1)["essential"] == 1).any() for r in rd))


def test_replays_return_to_a_clean_state(ctx):
    sizes = [120, 45, 200, 80]
    dev = ctx.batch(sizes, 3, max_dim=1, device_reduction=True)
    host = ctx.batch(sizes, 3, max_dim=1, host_reduction=True)
    split = ctx.batch(sizes, 3, max_dim=1)
    try:
        for seed in range(4):
            rng = np.random.default_rng(100 + seed)
            clouds = [synth.torus(n, 2.0, 0.5, 0.1, rng) for n in sizes]
            Xp = packed(clouds)
            rd, rh = dev.forward(Xp), host.forward(Xp)
            check_same(rd, rh)
            check_split(split.forward(Xp), rh)
    finally:
        dev.close()
        host.close()
        split.close()


@pytest.mark.parametrize("caps,expect_device", [("16,4,0", True), ("0,0,8", False)],
                         ids=["logs_overflow", "arena_overflow"])
@pytest.mark.parametrize("device_only", [True, False], ids=["device", "split"])
def test_overflow_paths(ctx, caps, expect_device, device_only):
    """Tiny toggle and V logs: the bitmaps are cleared whole and V is read
    whole, still on the device. A tiny V arena: the clouds that outgrow it
    are reduced on the host. The pairs are the same either way, also when
    the split forward gives some clouds to host threads from the start."""
    clouds = synth.torus_batch(4, 150, 0.1, seed=8)
    os.environ["VRPH_DRED_TEST_CAPS"] = caps
    try:
        dev = ctx.batch([len(c) for c in clouds], 3, max_dim=1, device_reduction=device_only)
    finally:
        del os.environ["VRPH_DRED_TEST_CAPS"]
    host = ctx.batch([len(c) for c in clouds], 3, max_dim=1, host_reduction=True)
    try:
        Xp = packed(clouds)
        for _ in range(2):  # and the state left behind is clean for the next forward
            rd, rh = dev.forward(Xp), host.forward(Xp)
            if device_only:
                check_same(rd, rh, expect_device=expect_device)
            else:
                check_split(rd, rh)
            flags = [r.stats["device_reduced"] for r in rd]
            if expect_device and device_only:
                assert all(flags)
            elif not expect_device:
                assert not all(flags), "no cloud outgrew the 8-entry arena"
    finally:
        dev.close()
        host.close()


def test_c5_device_matches_host(ctx):
    """The differentiable workload at full size (64 tori x 500 points): the
    same pairs, additions and emergent counts on the device as on the host,
    and in the split forward, which gives some of the clouds to the host
    threads and leaves the others on the device."""
    clouds = synth.torus_batch(64, 500, 0.1, seed=0)
    rd, rh = run_both(ctx, clouds)
    check_same(rd, rh)
    split = ctx.batch([len(c) for c in clouds], 3, max_dim=1)
    try:
        rs = split.forward(packed(clouds))
        check_split(rs, rh)
        on_device = sum(r.stats["device_reduced"] for r in rs)
        assert 0 < on_device < len(clouds), on_device
    finally:
        split.close()


def test_batch_autotune(ctx, tmp_path):
    """The batch autotuner (VRPH_AUTOTUNE): the tuned plan gives the same
    pairs as the default one, writes its choice to the tuning file, and a new
    context reading that file uses it without tuning again."""
    import torch

    from paper_2502_05063_amd import vrph

    clouds = synth.circle_or_torus_batch(20, 40, 180, 0.05, seed=12)
    Xp = packed(clouds)
    sizes = [len(c) for c in clouds]
    path = str(tmp_path / "tuning.txt")
    os.environ["VRPH_TUNING_FILE"] = path
    try:
        c2 = vrph.Context()
        try:
            ref = ctx.batch(sizes, 3, max_dim=1, keep_zero=True)
            rr = ref.forward(Xp)
            tuned = c2.batch(sizes, 3, max_dim=1, keep_zero=True, autotune=True)
            rt = tuned.forward(Xp)
            for a, b in zip(rt, rr):
                assert np.array_equal(a.pairs, b.pairs)
            lines = [ln.split() for ln in open(path).read().splitlines()]
            batch_lines = [ln for ln in lines if ln[3] == "3"]
            assert len(batch_lines) == 1
            threads, mult = int(batch_lines[0][4]), int(batch_lines[0][5])
            assert threads in (256, 512, 1024) and mult >= 1
            assert rt[0].stats["grid"][1] == mult * torch.cuda.get_device_properties(0).multi_processor_count
            # a fresh context reads the choice and does not tune again
            c3 = vrph.Context()
            again = c3.batch(sizes, 3, max_dim=1, keep_zero=True, autotune=True)
            ra = again.forward(Xp)
            assert ra[0].stats["grid"][1] == rt[0].stats["grid"][1]
            assert len(open(path).read().splitlines()) == len(lines)
            for a, b in zip(ra, rr):
                assert np.array_equal(a.pairs, b.pairs)
            again.close()
            tuned.close()
            ref.close()
            c3.close()
        finally:
            c2.close()
    finally:
        del os.environ["VRPH_TUNING_FILE"]


@pytest.mark.parametrize("threads", [256, 512, 1024])
def test_every_workgroup_size_matches_host(tmp_path, threads):
    """Each workgroup size the autotuner may pick (forced through a tuning
    file line) gives the host reduction's pairs, additions and emergent
    counts."""
    import torch

    from paper_2502_05063_amd import vrph

    clouds = synth.circle_or_torus_batch(10, 60, 300, 0.05, seed=13)
    bucket = 1
    while bucket < max(len(c) for c in clouds):
        bucket <<= 1
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    path = str(tmp_path / "tuning.txt")
    with open(path, "w") as f:
        f.write(f"{arch} 1 {bucket} 3 {threads} 4\n")
    os.environ["VRPH_TUNING_FILE"] = path
    try:
        c = vrph.Context()
    finally:
        del os.environ["VRPH_TUNING_FILE"]
    try:
        rd, rh = run_both(c, clouds)
        check_same(rd, rh)
        assert rd[0].stats["grid"][1] == 4 * torch.cuda.get_device_properties(0).multi_processor_count
    finally:
        c.close()


def test_reduction_flags_exclude_each_other(ctx):
    from paper_2502_05063_amd import vrph

    with pytest.raises(vrph.VrphError) as ei:
        ctx.batch([50, 60], 3, max_dim=1, host_reduction=True, device_reduction=True)
    assert ei.value.status == vrph.EINVAL


@pytest.mark.parametrize("count", [1, 2, 3])
def test_split_small_batches(ctx, count):
    """Batches of one to three clouds: whatever the split picks (possibly
    every cloud on one side), three forwards in a row give the host
    reduction's pairs and counts."""
    clouds = synth.torus_batch(count, 300, 0.1, seed=20 + count)
    sizes = [len(c) for c in clouds]
    host = ctx.batch(sizes, 3, max_dim=1, host_reduction=True)
    split = ctx.batch(sizes, 3, max_dim=1)
    try:
        Xp = packed(clouds)
        rh = host.forward(Xp)
        for _ in range(3):
            check_split(split.forward(Xp), rh)
    finally:
        host.close()
        split.close()
