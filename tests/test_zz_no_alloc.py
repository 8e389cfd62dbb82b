"""rk4ip_step_noalloc (the step without a plan or a workspace, its tables and work fields in
the library's static device buffer) against rk4ip_step on a plan built with flags 0, through
the C ABI: the same launches on tables computed with the same expressions, so the results
agree to rounding (relative 1e-6; in practice bitwise). Two calls in a row, the second with
a smaller input, so that the buffer's leftovers from the first call cannot leak into the
second."""
import numpy as np
import pytest

from gpu_helpers import log, quantised, random_field
from paper_1204_4255_amd import rk4ip
from paper_1204_4255_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    rk4ip.load()
    return t


def _case(torch, groups, step, extra=()):
    """groups: workload groups; extra: (problem, field) pairs appended after them."""
    fields = [quantised(random_field(g, 11 + i)) for i, g in enumerate(groups)]
    w = W.Workload("noalloc", groups, 1e-3, 1, fields)
    probs, _keep = rk4ip.problems_from_workload(w)
    probs += [p for p, _ in extra]
    flat = np.concatenate([np.asarray(f, np.complex64).reshape(-1) for f in fields + [f for _, f in extra]])
    ref = torch.tensor(flat, device="cuda")
    plan = rk4ip.Plan(probs, flags=0)
    plan.step(ref, step)
    got = torch.tensor(flat, device="cuda")
    rk4ip.step_noalloc(probs, got, step)
    torch.cuda.synchronize()
    plan.destroy()
    err = float(torch.linalg.vector_norm(got - ref) / torch.linalg.vector_norm(ref))
    same = bool(torch.equal(got, ref))
    log(f"  groups {[g.n for g in groups]}: rel diff {err:.3e}, bitwise {same}")
    assert torch.isfinite(got).all()
    assert err < 1e-6


def _big():
    # 3D + 2D + 1D (noisy, trapped, damped), about 1.2 M points
    return [W.Group(n=(64, 64, 128), lo=(-6, -6, -8), hi=(6, 6, 8), batch=2, gnl=50.0, trap=(1, 1.5, 2), gamma=0.02,
                    sigma=0.01, seed=3),
            W.Group(n=(256, 128), lo=(-8, -6), hi=(8, 6), batch=3, gnl=20.0, trap=(1, 1, 0), sigma=0.02, seed=3,
                    id_base=2),
            W.Group(n=(1024,), lo=(-16,), hi=(16,), batch=64, gnl=1.0, trap=(1, 0, 0), gamma=0.01, sigma=1e-3,
                    seed=3, id_base=5)]


def _small(torch):
    """A small 2D group with a potential grid, then a cosine-basis line and a noisy line."""
    g = W.Group(n=(32, 16), lo=(-4, -4), hi=(4, 4), batch=2, gnl=5.0, trap=(1, 1, 0), sigma=0.01, seed=7)
    rng = np.random.Generator(np.random.PCG64(4))
    g.Vgrid = (0.1 * rng.standard_normal((2, g.M))).astype(np.float32)
    x = (np.arange(128) + 0.5) * 7.0 / 128
    cos_line = rk4ip.make_problem((128,), (0,), (7,), 1e-3, batch=3, g_nl=2.0, trap=(1, 0, 0), basis=1, seed=7,
                                  id_base=2)
    f_cos = quantised(np.broadcast_to(np.exp(-x ** 2 / 2), (3, 128)))
    line = rk4ip.make_problem((64,), (-4,), (4,), 1e-3, batch=5, g_nl=1.0, trap=(1, 0, 0), sigma=0.05, seed=7,
                              id_base=5)
    f_line = quantised(random_field(W.Group(n=(64,), lo=(-4,), hi=(4,), batch=5), 3))
    return [g], [(cos_line, f_cos), (line, f_line)]


def test_noalloc_step_matches_plan_step_twice(torch):
    """A large mixed plan, then a smaller one (its tables land where the first call's work
    fields were)."""
    log("rk4ip_step_noalloc: large mixed groups, then small groups")
    _case(torch, _big(), 17)
    groups, extra = _small(torch)
    _case(torch, groups, 3, extra)


def test_noalloc_refuses_what_does_not_fit(torch):
    too_big = rk4ip.make_problem((256, 256, 128), (0, 0, 0), (1, 1, 1), 1e-3)  # 8.4 M points, 134 MB
    psi = torch.zeros(256 * 256 * 128, dtype=torch.complex64, device="cuda")
    with pytest.raises(rk4ip.Rk4ipError) as e:
        rk4ip.step_noalloc([too_big], psi, 0)
    assert e.value.status == rk4ip.RK4IP_ERR_WORKSPACE_TOO_SMALL
    K = np.ones(64)
    conv = rk4ip.make_problem((64,), (0,), (1,), 1e-3, conv_K=K)
    psi = torch.zeros(64, dtype=torch.complex64, device="cuda")
    with pytest.raises(rk4ip.Rk4ipError) as e:
        rk4ip.step_noalloc([conv], psi, 0)
    assert e.value.status == rk4ip.RK4IP_ERR_INVALID_ARG
