"""Merged launches (RK4IP_FLAG_MERGE_GROUPS): every pass kind of the 2D/3D groups of a plan
is one launch over all of them, through a work list of block offsets. Their arithmetic is the
per-group launches' with the merged schedule (radix 8, 256 threads, 2048/n lines or
columns), so a merged plan must equal, bitwise, a per-group plan forced to that schedule
(through the tune cache), eagerly and replayed from graphs; the profiler sees one launch
per pass kind, under the first group of each dimensionality."""
import json
import os

import numpy as np
import pytest

import oracle
from gpu_helpers import log, oprob, quantised, random_field, rel
from paper_1204_4255_amd import rk4ip
from paper_1204_4255_amd import workloads as W

pytestmark = pytest.mark.gpu

G = rk4ip.RK4IP_FLAG_GRAPH
MERGE = rk4ip.RK4IP_FLAG_MERGE_GROUPS

PASS_AXES = {2: [0, 1, 0, 0], 3: [0, 1, 2, 1, 0, 0]}


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    rk4ip.load()
    return t


def _forced_plan(probs, groups, flags, path):
    """A per-group plan whose passes use the merged schedule (written into a tune cache)."""
    cache = {}
    for g in groups:
        n3 = tuple(g.n) + (1,) * (3 - len(g.n))
        base = f"gfx950|n={n3[0]},{n3[1]},{n3[2]}|b={g.batch}"
        if len(g.n) == 1:
            cache[f"{base}|pass=0"] = [0, 0, 16, 0]
            continue
        for i, ax in enumerate(PASS_AXES[len(g.n)]):
            cache[f"{base}|pass={i}"] = [2048 // g.n[ax], 0, 8, 0]
    with open(path, "w") as fh:
        json.dump(cache, fh)
    old = os.environ.get("RK4IP_TUNE_CACHE")
    os.environ["RK4IP_TUNE_CACHE"] = str(path)
    try:
        plan = rk4ip.Plan(probs, flags=flags | rk4ip.RK4IP_FLAG_AUTOTUNE)
    finally:
        if old is None:
            del os.environ["RK4IP_TUNE_CACHE"]
        else:
            os.environ["RK4IP_TUNE_CACHE"] = old
    return plan


def _groups():
    rng = np.random.Generator(np.random.PCG64(8))
    gs = [W.Group(n=(128, 128), lo=(-8, -8), hi=(8, 8), batch=5, gnl=100.0, trap=(1, 1, 0), sigma=0.01, seed=6),
          W.Group(n=(256, 256), lo=(-8, -8), hi=(8, 8), batch=3, gnl=20.0, trap=(1, 1, 0), seed=6, id_base=5),
          W.Group(n=(128,), lo=(-8,), hi=(8,), batch=4, gnl=1.0, trap=(1, 0, 0), sigma=0.01, seed=6, id_base=8),
          W.Group(n=(256, 128), lo=(-8, -4), hi=(8, 4), batch=1, gnl=50.0, trap=(1, 2, 0), gamma=0.02, seed=6,
                  id_base=12),
          W.Group(n=(128, 128, 256), lo=(-5, -5, -6), hi=(5, 5, 6), batch=1, gnl=20.0, trap=(1, 1, 1), sigma=0.005,
                  seed=6, id_base=13)]
    for g in gs[:2]:
        g.Vgrid = (0.01 * rng.standard_normal((g.batch, g.M))).astype(np.float32)
    return gs


@pytest.mark.parametrize("flags", [0, G], ids=["eager", "graph"])
def test_merged_equals_per_group_launches(torch, tmp_path, flags):
    gs = _groups()
    fields = [quantised(0.5 * random_field(g, 40 + i)) for i, g in enumerate(gs)]
    w = W.Workload("merged", gs, 1e-3, 37, fields)
    probs, keep = rk4ip.problems_from_workload(w)
    merged = rk4ip.Plan(probs, flags=flags | MERGE)
    ref = _forced_plan(probs, gs, flags, tmp_path / "tune.json")
    names_m = [[merged.schedule(i, k) for k in range(merged.num_passes(i))] for i in range(len(gs))]
    names_r = [[ref.schedule(i, k) for k in range(ref.num_passes(i))] for i in range(len(gs))]
    log(f"merged {flags}: " + " | ".join(" ".join(n) for n in names_m))
    assert names_m == names_r
    a = rk4ip.field_to_device(w)
    b = rk4ip.field_to_device(w)
    merged.run(a, 37, step0=4)
    ref.run(b, 37, step0=4)
    torch.cuda.synchronize()
    assert torch.isfinite(torch.view_as_real(a)).all()
    assert torch.equal(a, b)
    # and the physics: one noisy instance of the 2D group against the oracle
    g0 = gs[0]
    g1 = W.Group(n=g0.n, lo=g0.lo, hi=g0.hi, batch=1, gnl=g0.gnl, trap=g0.trap, sigma=g0.sigma, seed=g0.seed,
                 id_base=g0.id_base + 2)
    g1.Vgrid = g0.Vgrid[2:3]
    r, _, _ = oracle.run(oprob(g1, w.h), fields[0][2:3], 37, step0=4)
    got = a[2 * g0.M:3 * g0.M].cpu().numpy().astype(np.complex128)
    err = rel(got, r)
    log(f"  instance 2 of the 128^2 group vs oracle: {err:.2e}")
    assert err < 1e-5
    merged.destroy()
    ref.destroy()


def test_merged_launch_counts(torch):
    """Eager merged run of 6 steps: each 2D/3D pass kind is timed once per launch under the
    first group of its dimensionality; the other groups of that dimensionality see none."""
    gs = _groups()
    fields = [quantised(0.5 * random_field(g, 40 + i)) for i, g in enumerate(gs)]
    w = W.Workload("merged", gs, 1e-3, 6, fields)
    probs, keep = rk4ip.problems_from_workload(w)
    plan = rk4ip.Plan(probs, flags=MERGE)
    d = rk4ip.field_to_device(w)
    plan.profile(True)
    plan.run(d, 6)
    counts = [[plan.profile_read(i, k)[0] for k in range(plan.num_passes(i))] for i in range(len(gs))]
    log(f"  launches per (group, pass): {counts}")
    # 2D: FIRST, LF, XF, LAST2 -> 1, 6, 5, 1 under group 0; 3D the same pattern under group 4
    assert counts[0] == [1, 6, 5, 1] and counts[1] == [0, 0, 0, 0] and counts[3] == [0, 0, 0, 0]
    assert counts[4] == [1, 6, 6, 6, 5, 1]
    assert counts[2] == [6]  # the 1D group: one launch per step
    plan.destroy()


def test_merged_uneven_batch_full_shapes(torch, tmp_path):
    """The adjoint workload's uneven batch (32 x 128^2 + 32 x 256^2, each instance with its
    own potential grid), 20 steps from graphs: merged equals per-group launches bitwise."""
    w = W.adjoint2d(nsteps=20)
    probs, keep = rk4ip.problems_from_workload(w)
    merged = rk4ip.Plan(probs, flags=G | MERGE)
    ref = _forced_plan(probs, w.groups, G, tmp_path / "tune.json")
    a = rk4ip.field_to_device(w)
    b = rk4ip.field_to_device(w)
    merged.run(a, 20)
    ref.run(b, 20)
    torch.cuda.synchronize()
    log(f"  adjoint2d shapes merged vs per-group: bitwise {bool(torch.equal(a, b))}")
    assert torch.equal(a, b)
    merged.destroy()
    ref.destroy()
