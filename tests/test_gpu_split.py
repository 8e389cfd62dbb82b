"""The split-field schedule (one thread per field; field order 3 in the tune cache) forced on
every pass of noisy 2D and 3D lattices with a potential grid and the noise in the potential,
in both precision forms. Each thread of a split workgroup runs the same arithmetic on its
field as a thread of the joint schedule does on that field, so the runs must equal the
joint schedule's bitwise, eagerly and replayed from graphs, and match the FP64 oracle."""
import json
import os

import numpy as np
import pytest

import oracle
from gpu_helpers import log, quantised, rel
from paper_1204_4255_amd import rk4ip, workloads as W

pytestmark = pytest.mark.gpu

# axis of each pass: FIRST, LF, XF, LAST2 (2D); FIRST, D2, LF, D2, XF, LAST2 (3D)
PASS_AXES = {2: [0, 1, 0, 0], 3: [0, 1, 2, 1, 0, 0]}
# the LF and XF passes (split also at radix 16)
PASS_LFXF = {2: [1, 2], 3: [2, 4]}


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    rk4ip.load()
    return t


def _forced(probs, g, seq, f64, flags, path, slines=4, rr=8):
    """A plan whose passes all take radix `rr` with `seq` (0 joint, 3 split): half the
    default lines on the contiguous axis, `slines` columns on the strided ones. At radix 16
    only LF and XF take the split schedule (the others stay joint)."""
    n3 = tuple(g.n) + (1,) * (3 - len(g.n))
    base = f"gfx950|n={n3[0]},{n3[1]},{n3[2]}|b={g.batch}"
    cache = {}
    for i, ax in enumerate(PASS_AXES[len(g.n)]):
        N = g.n[ax]
        lines = (4096 // N) // 2 if ax == 0 else slines
        sq = seq if (rr == 8 or i in PASS_LFXF[len(g.n)]) else 0
        cache[f"{base}|pass={i}{'|f64' if f64 else ''}"] = [lines, sq, rr, 0]
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


@pytest.mark.parametrize("n,batch", [((256, 128), 2), ((128, 128, 128), 1)])
@pytest.mark.parametrize("f64", [False, True])
def test_split_schedule_equals_joint_and_oracle(torch, tmp_path, n, batch, f64):
    log(f"split schedule: n={n} batch={batch} f64={f64}")
    _compare(torch, tmp_path, n, batch, f64, [(0, 4), (3, 4)])


@pytest.mark.parametrize("n,batch", [((128, 256), 2), ((128, 256, 256), 1)])
@pytest.mark.parametrize("f64", [False, True])
def test_narrow_strided_tiles_equal_wide_and_oracle(torch, tmp_path, n, batch, f64):
    """Strided tiles of two columns (the narrow schedules of lattices with few lines) must
    equal four-column tiles bitwise, with both fields at once and split."""
    log(f"narrow strided tiles: n={n} batch={batch} f64={f64}")
    _compare(torch, tmp_path, n, batch, f64, [(0, 4), (0, 2), (3, 2)])


@pytest.mark.parametrize("n,batch", [((256, 128), 2), ((128, 256, 256), 1)])
def test_radix16_split_equals_joint_and_oracle(torch, tmp_path, n, batch):
    """LF and XF split at radix 16 (complex64 only) equal the joint radix-16 schedule."""
    log(f"radix-16 split: n={n} batch={batch}")
    _compare(torch, tmp_path, n, batch, False, [(0, 4), (3, 4)], rr=16)


def _compare(torch, tmp_path, n, batch, f64, schedules, rr=8):
    """Runs of one noisy problem (potential grid, noise in the potential) under each forced
    (field order, strided columns) schedule: bitwise equal, one of them graph-replayed, and
    within 2e-6 of the oracle."""
    nd = len(n)
    g = W.Group(n=n, lo=(-6.0,) * nd, hi=(6.0,) * nd, batch=batch, gnl=3.0, trap=(1.0, 1.3, 0.7), gamma=0.02,
                sigma=0.01, seed=41, id_base=2)
    x = g.mesh()
    env = np.exp(-sum(X ** 2 for X in x) / 2)
    f0 = quantised(np.broadcast_to(env * np.exp(0.3j * x[0]), g.shape))
    rng = np.random.Generator(np.random.PCG64(43))
    Vg = (0.2 * rng.standard_normal((batch,) + tuple(n))).astype(np.float32)
    Vt = torch.tensor(Vg.reshape(-1), device="cuda")
    h, sv = 1e-3, 0.3
    p = rk4ip.make_problem(g.n, g.lo, g.hi, h, batch=batch, alpha=g.alpha, gamma=g.gamma, g_nl=g.gnl, trap=g.trap,
                           V_grid=Vt, sigma=g.sigma, seed=g.seed, id_base=g.id_base, sigma_V=sv)
    op = oracle.Problem(n=g.n, lo=g.lo, hi=g.hi, h=h, batch=batch, alpha=g.alpha, gamma=g.gamma, gnl=g.gnl,
                        trap=g.trap, Vgrid=Vg.astype(np.float64), sigma=g.sigma, seed=g.seed, id_base=g.id_base,
                        sigma_V=sv)
    flags = rk4ip.RK4IP_FLAG_FP64_TRANSFORMS if f64 else 0
    plans = []
    for k, (seq, sl) in enumerate(schedules):
        plans.append(_forced([p], g, seq, f64, flags, tmp_path / f"s{k}.json", sl, rr))
        for i in range(plans[-1].num_passes(0)):
            sq = seq if (rr == 8 or i in PASS_LFXF[nd]) else 0
            assert (":split:" if sq == 3 else ":joint:") in plans[-1].schedule(0, i)
            assert f":r{rr}" in plans[-1].schedule(0, i)
        strided = [plans[-1].schedule(0, i) for i in range(plans[-1].num_passes(0)) if ":strided:" in
                   plans[-1].schedule(0, i)]
        assert all(f":lines{sl}:" in x for x in strided), strided
    seq, sl = schedules[-1]
    plans.append(_forced([p], g, seq, f64, flags | rk4ip.RK4IP_FLAG_GRAPH, tmp_path / "g.json", sl, rr))
    nsteps = 6
    fields = []
    for plan in plans:
        d = torch.tensor(f0.astype(np.complex64).reshape(-1), device="cuda")
        plan.run(d, nsteps, step0=5)
        fields.append(d)
    torch.cuda.synchronize()
    assert all(torch.equal(fields[0], x) for x in fields[1:])
    ref, _, _ = oracle.run(op, f0, nsteps, step0=5)
    err = rel(fields[-1].cpu().numpy().astype(np.complex128).reshape(g.shape), ref)
    log(f"  {nsteps} steps: schedules {schedules} bitwise equal, rel L2 vs oracle {err:.2e}")
    assert err < 2e-6
