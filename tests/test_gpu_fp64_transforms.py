"""GPU parity of the FP64-transform precision form (RK4IP_FLAG_FP64_TRANSFORMS): the
propagator and the step against the FP64 oracle, and its determinism under graph replay,
autotuned schedules and resumed runs. With the transforms in FP64, a single operation is
within the rounding of its complex64 result (a few 1e-8)."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, oprob, quantised, random_field, rel, rel_per_instance
from paper_1204_4255_amd import rk4ip
from paper_1204_4255_amd import workloads as W

pytestmark = pytest.mark.gpu

F64 = rk4ip.RK4IP_FLAG_FP64_TRANSFORMS


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    rk4ip.load()
    return t


def _plan(w, flags):
    probs, keep = rk4ip.problems_from_workload(w)
    plan = rk4ip.Plan(probs, flags=flags)
    plan._keep_V = keep
    return plan


def _dev(torch, a):
    return torch.tensor(np.asarray(a, dtype=np.complex64).reshape(-1), device="cuda")


def _host(t, shape):
    return t.cpu().numpy().astype(np.complex128).reshape(shape)


@pytest.mark.parametrize("n,batch", [((8,), 3), ((1024,), 5), ((64, 8), 2), ((16, 128), 1), ((512, 32), 1),
                                     ((8, 16, 32), 2), ((64, 64, 64), 1), ((1024, 8, 8), 1)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_apply_D_fp64(torch, n, batch, adjoint):
    log(f"apply_D fp64 n={n} batch={batch} adjoint={adjoint}")
    nd = len(n)
    g = W.Group(n=n, lo=(-3.0,) * nd, hi=(4.0,) * nd, batch=batch, gamma=0.3, alpha=0.7)
    f = quantised(random_field(g, 5))
    w = W.Workload("d", [g], 0.05, 1, [f])
    plan = _plan(w, F64)
    d = _dev(torch, f)
    plan.apply_D(d, adjoint)
    ref = oracle.apply_D(oprob(g, 0.05), f, adjoint=adjoint)
    err = rel(_host(d, g.shape), ref)
    log(f"  rel {err:.2e}")
    # one FP32 rounding of the result per axis
    assert err < 1.5e-7 * nd


STEP_CASES = [
    ((8,), 3), ((16,), 130), ((64,), 5), ((256,), 9), ((1024,), 3), ((2048,), 2),
    ((8, 8), 2), ((64, 32), 3), ((32, 128), 1), ((512, 16), 1), ((16, 1024), 1),
    ((8, 8, 8), 3), ((32, 16, 8), 2), ((16, 32, 64), 1), ((128, 8, 16), 1),
]


@pytest.mark.parametrize("n,batch", STEP_CASES)
def test_one_step_fp64(torch, n, batch):
    log(f"one step fp64 n={n} batch={batch}")
    nd = len(n)
    g = W.Group(n=n, lo=(-5.0,) * nd, hi=(5.0,) * nd, batch=batch, gnl=2.5, trap=(1.0, 1.3, 0.7), gamma=0.05,
                sigma=0.02, seed=77, id_base=3)
    rng = np.random.Generator(np.random.PCG64(9))
    g.Vgrid = (0.1 * rng.standard_normal((batch, g.M))).astype(np.float32)
    f = quantised(random_field(g, 3))
    w = W.Workload("s", [g], 2e-3, 1, [f])
    plan = _plan(w, F64)
    d = _dev(torch, f)
    plan.step(d, 41)
    torch.cuda.synchronize()
    ref = oracle.step(oprob(g, 2e-3), f, 41)
    err = rel_per_instance(_host(d, g.shape), ref, batch)
    log(f"  max rel {np.max(err):.2e}")
    assert np.max(err) < 5e-7, err


@pytest.mark.parametrize("extra", [0, rk4ip.RK4IP_FLAG_GRAPH, rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_FUSE_1D,
                                   rk4ip.RK4IP_FLAG_AUTOTUNE])
def test_fp64_determinism_resume_and_graph(torch, extra):
    """Eager, graph-replayed, autotuned and resumed runs of mixed 1D/2D/3D groups agree:
    bitwise where the schedules are the same, within 1e-6 where the autotuner picks others."""
    log(f"fp64 determinism flags={extra}")
    gs = [W.Group(n=(64, 16), lo=(-6, -6), hi=(6, 6), batch=2, gnl=5.0, trap=(1, 1, 0), sigma=0.01, seed=9),
          W.Group(n=(256,), lo=(-8,), hi=(8,), batch=5, gnl=1.0, trap=(1, 0, 0), sigma=0.01, seed=9, id_base=2),
          W.Group(n=(16, 8, 32), lo=(-4, -4, -4), hi=(4, 4, 4), batch=1, gnl=2.0, trap=(1, 1, 1), sigma=0.01,
                  seed=9, id_base=7)]
    fields = [quantised(random_field(g, 30 + i)) for i, g in enumerate(gs)]
    w = W.Workload("det", gs, 1e-3, 41, fields)
    base = _plan(w, F64)
    a = rk4ip.field_to_device(w)
    base.run(a, 41, step0=100)
    plan = _plan(w, F64 | extra)
    b = rk4ip.field_to_device(w)
    plan.run(b, 41, step0=100)
    c = rk4ip.field_to_device(w)
    plan.run(c, 20, step0=100)
    plan.run(c, 21, step0=120)
    torch.cuda.synchronize()
    if extra & rk4ip.RK4IP_FLAG_AUTOTUNE:
        assert float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(a)) < 1e-6
    else:
        assert torch.equal(a, b)
    assert torch.equal(b, c)
    # and the run itself against the oracle, group by group
    off = 0
    for g, f in zip(gs, fields):
        n = g.batch * g.M
        ref, _, _ = oracle.run(oprob(g, 1e-3), f, 41, step0=100)
        err = rel(_host(b[off:off + n], g.shape), ref)
        log(f"  group n={g.n}: rel {err:.2e}")
        assert err < 2e-6
        off += n
