"""GPU parity of the semi-implicit integrator (RK4IP_FLAG_SEMI_IMPLICIT: Sec. 3.5's
semi-implicit method in the midpoint interaction picture) and of the noise substeps
(noise_substeps, the shared Wiener path of Sec. 3.5's strong-convergence test) against
the FP64 oracle: one step on every lattice kind, runs through graphs, fused 1D launches,
autotuned schedules and the FP64-transform form, and the strong convergence of a
stochastic GPE measured on both sides."""
import numpy as np
import pytest

import oracle
from gpu_helpers import assert_same_runs, log, oprob, plan_for, quantised, random_field, rel, rel_per_instance
from paper_1204_4255_amd import rk4ip
from paper_1204_4255_amd import workloads as W

pytestmark = pytest.mark.gpu

SI = rk4ip.RK4IP_FLAG_SEMI_IMPLICIT
F64 = rk4ip.RK4IP_FLAG_FP64_TRANSFORMS


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    rk4ip.load()
    return t


def _dev(torch, a):
    return torch.tensor(np.asarray(a, dtype=np.complex64).reshape(-1), device="cuda")


def _host(t, shape):
    return t.cpu().numpy().astype(np.complex128).reshape(shape)


def _group(n, batch, **kw):
    nd = len(n)
    base = dict(n=n, lo=(-5.0,) * nd, hi=(5.0,) * nd, batch=batch, gnl=2.5, trap=(1.0, 1.3, 0.7), gamma=0.05,
                sigma=0.02, seed=77, id_base=3)
    base.update(kw)
    g = W.Group(**base)
    rng = np.random.Generator(np.random.PCG64(9))
    g.Vgrid = (0.1 * rng.standard_normal((batch, g.M))).astype(np.float32)
    return g


STEP_CASES = [
    ((8,), 3), ((16,), 130), ((64,), 5), ((256,), 9), ((1024,), 3), ((2048,), 2), ((4096,), 1),
    ((8, 8), 2), ((64, 32), 3), ((32, 128), 1), ((512, 16), 1), ((16, 1024), 1),
    ((8, 8, 8), 3), ((32, 16, 8), 2), ((16, 32, 64), 1), ((128, 8, 16), 1), ((64, 64, 64), 1),
]


@pytest.mark.parametrize("S", [1, 4])
@pytest.mark.parametrize("n,batch", STEP_CASES)
def test_si_one_step_matches_oracle(torch, n, batch, S):
    log(f"semi-implicit step n={n} batch={batch} substeps={S}")
    g = _group(n, batch)
    f = quantised(random_field(g, 3))
    w = W.Workload("si", [g], 2e-3, 1, [f])
    plan = plan_for(w, SI, noise_substeps=S)
    d = _dev(torch, f)
    plan.step(d, 41)
    torch.cuda.synchronize()
    ref = oracle.step(oprob(g, 2e-3, integrator=1, noise_substeps=S), f, 41)
    err = rel_per_instance(_host(d, g.shape), ref, batch)
    log(f"  max rel {np.max(err):.2e}")
    assert np.max(err) < 1e-6, err


@pytest.mark.parametrize("S", [2, 8, 1024])
def test_noise_substeps_match_oracle(torch, S):
    log(f"noise with {S} substeps")
    g = W.Group(n=(64, 16), lo=(-3, -3), hi=(3, 3), batch=3, sigma=1.0, seed=0x1234_5678_9ABC, id_base=11)
    w = W.Workload("nz", [g], 1e-3, 1, [np.zeros(g.shape, complex)])
    plan = plan_for(w, 0, noise_substeps=S)
    for step in (0, 5, (1 << 30) + 3):
        xi = plan.noise(0, step).cpu().numpy().astype(np.complex128)
        ref = oracle.noise(oprob(g, 1e-3, noise_substeps=S), step).reshape(g.batch, -1)
        # a sum of S single-precision draws
        assert np.max(np.abs(xi - ref)) <= 2e-6 * np.sqrt(S) * np.max(np.abs(ref)), step


def _mixed_groups():
    return [W.Group(n=(64, 16), lo=(-6, -6), hi=(6, 6), batch=2, gnl=5.0, trap=(1, 1, 0), gamma=0.1, sigma=0.01,
                    seed=9),
            W.Group(n=(256,), lo=(-8,), hi=(8,), batch=5, gnl=1.0, trap=(1, 0, 0), sigma=0.01, seed=9, id_base=2),
            W.Group(n=(16, 8, 32), lo=(-4, -4, -4), hi=(4, 4, 4), batch=1, gnl=2.0, trap=(1, 1, 1), sigma=0.01,
                    seed=9, id_base=7)]


@pytest.mark.parametrize("extra", [0, rk4ip.RK4IP_FLAG_GRAPH, rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_FUSE_1D,
                                   F64, F64 | rk4ip.RK4IP_FLAG_GRAPH])
@pytest.mark.parametrize("S", [1, 4])
def test_si_runs_resume_graph_and_oracle(torch, extra, S):
    """Eager, graph-replayed (one axis-0 pass applying the half step twice between steps),
    fused and resumed runs of mixed 1D/2D/3D groups are bitwise equal, and agree with the
    oracle's run."""
    log(f"semi-implicit runs flags={extra} substeps={S}")
    gs = _mixed_groups()
    fields = [quantised(random_field(g, 30 + i)) for i, g in enumerate(gs)]
    w = W.Workload("det", gs, 1e-3, 41, fields)
    base = plan_for(w, SI | (extra & F64), noise_substeps=S)
    a = rk4ip.field_to_device(w)
    base.run(a, 41, step0=100)
    plan = plan_for(w, SI | extra, noise_substeps=S)
    b = rk4ip.field_to_device(w)
    plan.run(b, 41, step0=100)
    c = rk4ip.field_to_device(w)
    plan.run(c, 20, step0=100)
    plan.run(c, 21, step0=120)
    torch.cuda.synchronize()
    assert_same_runs(torch, gs, a, b, c, kspace_lines=not extra & F64)
    off = 0
    for g, f in zip(gs, fields):
        n = g.batch * g.M
        ref, _, _ = oracle.run(oprob(g, 1e-3, integrator=1, noise_substeps=S), f, 41, step0=100)
        err = rel(_host(b[off:off + n], g.shape), ref)
        log(f"  group n={g.n}: rel {err:.2e}")
        assert err < (2e-6 if extra & F64 else 5e-6)
        off += n


def test_si_graph_replays_with_work_between(torch):
    log("semi-implicit graph replays interleaved with eager torch work")
    g = W.Group(n=(32, 16, 8), lo=(-4, -4, -4), hi=(4, 4, 4), batch=2, gnl=3.0, trap=(1, 1, 1), gamma=0.2,
                sigma=0.01, seed=4)
    f = quantised(random_field(g, 40))
    w = W.Workload("gr", [g], 1e-3, 33, [f])
    eager = plan_for(w, SI)
    graph = plan_for(w, SI | rk4ip.RK4IP_FLAG_GRAPH)
    a = _dev(torch, f)
    b = _dev(torch, f)
    for rep in range(4):
        eager.run(a, 33, step0=33 * rep)
        graph.run(b, 33, step0=33 * rep)
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(a, b), rep


@pytest.mark.parametrize("extra", [0, F64])
def test_si_autotuned_schedules_match_oracle(torch, extra):
    log(f"semi-implicit autotuned schedules flags={extra} (3D 256x32x64, 2D 512x128, 1D 1024)")
    for n in ((256, 32, 64), (512, 128), (1024,)):
        nd = len(n)
        g = W.Group(n=n, lo=(-5.0,) * nd, hi=(5.0,) * nd, batch=2 if nd == 1 else 1, gnl=10.0, trap=(1, 1, 1),
                    gamma=0.05, sigma=0.01, seed=2)
        f = quantised(random_field(g, 50))
        w = W.Workload("t", [g], 1e-3, 3, [f])
        tuned = plan_for(w, SI | extra | rk4ip.RK4IP_FLAG_AUTOTUNE)
        log("  " + " ".join(tuned.schedule(0, i) for i in range(tuned.num_passes(0))))
        b = _dev(torch, f)
        tuned.run(b, 3)
        torch.cuda.synchronize()
        ref, _, _ = oracle.run(oprob(g, 1e-3, integrator=1), f, 3)
        err = rel(_host(b, g.shape), ref)
        log(f"  rel {err:.2e}")
        assert err < 2e-6


def test_si_adjoint_is_rejected(torch):
    g = W.Group(n=(16, 16), lo=(-2, -2), hi=(2, 2), gnl=1.0)
    f = quantised(random_field(g, 1))
    plan = plan_for(W.Workload("a", [g], 1e-3, 4, [f]), SI)
    d = _dev(torch, f)
    _, ck = plan.run(d, 4, ckpt_every=2)
    with pytest.raises(rk4ip.Rk4ipError) as e:
        plan.adjoint(ck, 4, 2, torch.ones_like(d))
    assert e.value.status == rk4ip.RK4IP_ERR_INVALID_ARG


def test_si_strong_convergence_matches_oracle(torch):
    """A stochastic damped GPE (32 paths, 64 points on [-8, 8)) integrated to T = 0.64 with
    h = 2^l h_f and 2^l noise substeps, so every run samples one Wiener path; the error of
    each level against the h_f run, per path, averaged over paths. The steps keep the
    fixed-point iteration contracting (h max V / 2 < 1) and the fastest mode resolved
    (h k_max^2 / 2 < 1). The GPU's errors equal the oracle's to a few percent and fall
    at least as h^0.8 (strong order one; the oracle measures 1.04)."""
    g = W.Group(n=(64,), lo=(-8.0,), hi=(8.0,), batch=32, gnl=10.0, gamma=0.05, sigma=0.1, trap=(1.0, 0, 0),
                seed=21)
    x = g.axis(0)
    psi0 = np.broadcast_to(np.pi ** -0.25 * np.exp(-x ** 2 / 2), g.shape).astype(np.complex64).astype(np.complex128)
    hf, T = 2.5e-4, 0.64
    nf = int(round(T / hf))
    levels = (16, 8, 4)

    def gpu_run(S):
        w = W.Workload("sc", [g], hf * S, nf // S, [psi0])
        plan = plan_for(w, SI | rk4ip.RK4IP_FLAG_GRAPH | F64, noise_substeps=S)
        d = _dev(torch, psi0)
        plan.run(d, nf // S)
        torch.cuda.synchronize()
        return _host(d, g.shape)

    def ora_run(S):
        out, _, _ = oracle.run(oprob(g, hf * S, integrator=1, noise_substeps=S), psi0, nf // S)
        return out

    def perr(a, b):
        return float(np.mean(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))

    gfine, ofine = gpu_run(1), ora_run(1)
    log(f"  fine runs differ by {perr(gfine, ofine):.2e}")
    assert perr(gfine, ofine) < 1e-5
    ge, oe = [], []
    for S in levels:
        gr, orr = gpu_run(S), ora_run(S)
        assert perr(gr, orr) < 1e-5
        ge.append(perr(gr, gfine))
        oe.append(perr(orr, ofine))
        log(f"  h = {hf * S:.4g}: strong error gpu {ge[-1]:.4e} oracle {oe[-1]:.4e}")
    assert np.allclose(ge, oe, rtol=0.03)
    orders = [np.log2(ge[i] / ge[i + 1]) for i in range(len(ge) - 1)]
    log(f"  orders {orders}")
    assert all(o > 0.8 for o in orders), orders
