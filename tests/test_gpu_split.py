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


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    rk4ip.load()
    return t


def _forced(probs, g, seq, f64, flags, path):
    """A plan whose passes all take radix 8 with `seq` (0 joint, 3 split): half the default
    lines on the contiguous axis, 4 columns on the strided ones (compiled for both)."""
    n3 = tuple(g.n) + (1,) * (3 - len(g.n))
    base = f"gfx950|n={n3[0]},{n3[1]},{n3[2]}|b={g.batch}"
    cache = {}
    for i, ax in enumerate(PASS_AXES[len(g.n)]):
        N = g.n[ax]
        lines = (4096 // N) // 2 if ax == 0 else 4
        cache[f"{base}|pass={i}{'|f64' if f64 else ''}"] = [lines, seq, 8, 0]
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
    joint = _forced([p], g, 0, f64, flags, tmp_path / "joint.json")
    split = _forced([p], g, 3, f64, flags, tmp_path / "split.json")
    splitg = _forced([p], g, 3, f64, flags | rk4ip.RK4IP_FLAG_GRAPH, tmp_path / "split.json")
    assert all(":split:" in split.schedule(0, i) for i in range(split.num_passes(0)))
    assert all(":joint:" in joint.schedule(0, i) for i in range(joint.num_passes(0)))
    nsteps = 6
    fields = []
    for plan in (joint, split, splitg):
        d = torch.tensor(f0.astype(np.complex64).reshape(-1), device="cuda")
        plan.run(d, nsteps, step0=5)
        fields.append(d)
    torch.cuda.synchronize()
    assert torch.equal(fields[0], fields[1]) and torch.equal(fields[1], fields[2])
    ref, _, _ = oracle.run(op, f0, nsteps, step0=5)
    err = rel(fields[1].cpu().numpy().astype(np.complex128).reshape(g.shape), ref)
    log(f"  {nsteps} steps: split == joint bitwise, rel L2 vs oracle {err:.2e}")
    assert err < 2e-6
