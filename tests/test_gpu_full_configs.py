"""GPU parity of the five workloads at their full sizes and run lengths, in the launch
configuration the benchmark uses (hipGraph replay, autotuned schedules, several 1D steps
per launch). Where the oracle cannot follow the whole workload in seconds, it follows
sampled instances one by one, and properties that hold at any size cover the rest.
"Relative L2 over the run" is the maximum over the sample times of the workload."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, oprob, quantised, rel, rel_per_instance
from paper_1204_4255_amd import rk4ip
from paper_1204_4255_amd import workloads as W

pytestmark = pytest.mark.gpu

BENCH_FLAGS = rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_AUTOTUNE
F64 = rk4ip.RK4IP_FLAG_FP64_TRANSFORMS

# Precision forms: on gpe2d the complex64 form accumulates the FP32 rounding of the
# per-axis transforms (the same every step, so it adds up linearly) to about 1e-5 over
# 2000 steps, at the target, so the FP64-transform form (FFTs, propagator multiply and
# delta add in FP64, fields complex64) is the form this workload is claimed in and is held
# to 1e-5. The complex64 run is kept as a measurement with a bound that only guards
# against regressions; it is not claimed at 1e-5. The 1D lines of sgpe1d keep their state
# in k-space and hold 1e-5 in complex64.


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


def _host(t, shape):
    return t.cpu().numpy().astype(np.complex128).reshape(shape)


@pytest.mark.parametrize("flags,bound", [(rk4ip.RK4IP_FLAG_GRAPH | F64, 1e-5), (BENCH_FLAGS | F64, 1e-5),
                                         (BENCH_FLAGS, 1.5e-5)],
                         ids=["fp64-default", "fp64-autotuned", "c64-autotuned-unclaimed"])
def test_gpe2d_512_full_run(torch, flags, bound):
    """512^2, 2000 steps: error over the run (every 100 steps) and FP64 diagnostics. The
    kinetic energy weights the field error by k^2 (FP32 rounding sits at high k), so it
    gets 1e-4; N, E_pot and E_int get 1e-5."""
    w = W.gpe2d()
    g = w.groups[0]
    log(f"gpe2d 512^2, {w.nsteps} steps, samples every {w.sample_every}, flags {flags}")
    f = quantised(w.psi0[0])
    plan = _plan(w, flags)
    d = torch.tensor(f.astype(np.complex64).reshape(-1), device="cuda")
    ref = f.copy()
    p = oprob(g, w.h)
    errs = []
    for s in range(0, w.nsteps, w.sample_every):
        plan.run(d, w.sample_every, step0=s)
        ref, _, _ = oracle.run(p, ref, w.sample_every, step0=s)
        errs.append(rel(_host(d, g.shape), ref))
    gdiag = plan.diagnostics(d).cpu().numpy()[0]
    rdiag = oracle.diag(p, ref)[0]
    log("  rel L2 at samples: " + " ".join(f"{e:.2e}" for e in errs))
    log(f"  diagnostics rel diff (N, E_kin, E_pot, E_int): {np.abs(gdiag / rdiag - 1)}")
    assert max(errs) < bound
    assert np.all(np.abs(gdiag / rdiag - 1) < np.array([1e-5, 1e-4, 1e-5, 1e-5]))


@pytest.mark.parametrize("flags,bound", [(0, 1e-5), (F64, 1e-5)], ids=["c64", "fp64"])
def test_sgpe1d_full_length(torch, flags, bound):
    """2048 paths x 1024, 5000 steps, several steps per launch from a graph: 16 sampled
    paths against the oracle one by one over the run, and the ensemble norm of all paths
    against its expectation. The Hamiltonian part keeps N pathwise and damping is uniform,
    so only the noise feeds N. For a forcing held constant over a step the scheme integrates
    e^{L(h - s)} with Simpson weights S_k = (e^{L_k h} + 4 e^{L_k h/2} + 1)/6 (the stages with
    G constant), so each step adds h sigma^2 sum_k |S_k|^2 to E[N] on average. Modes that turn
    by several radians per step get less than the white-noise rate sigma^2 M (here on
    average 74% of it), so the continuum value sigma^2 M / (2 gamma) does not apply."""
    w = W.sgpe1d()
    g = w.groups[0]
    log(f"sgpe1d {g.batch} paths x {g.n[0]}, {w.nsteps} steps, flags {flags}")
    plan = _plan(w, rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_FUSE_1D | flags)
    f = quantised(w.psi0[0])
    d = torch.tensor(f.astype(np.complex64).reshape(-1), device="cuda")
    sample = np.linspace(0, g.batch - 1, 16).astype(int)
    refs = {int(b): f[b:b + 1].copy() for b in sample}
    worst = np.zeros(len(sample))
    for s in range(0, w.nsteps, w.sample_every):
        plan.run(d, w.sample_every, step0=s)
        got = _host(d, g.shape)
        for i, b in enumerate(sample):
            gb = W.Group(n=g.n, lo=g.lo, hi=g.hi, batch=1, gnl=g.gnl, gamma=g.gamma, sigma=g.sigma, trap=g.trap,
                         seed=g.seed, id_base=g.id_base + int(b))
            refs[int(b)], _, _ = oracle.run(oprob(gb, w.h), refs[int(b)], w.sample_every, step0=s)
            worst[i] = max(worst[i], rel_per_instance(got[b:b + 1], refs[int(b)], 1)[0])
    log(f"  sampled paths, max rel L2 over the run: max {worst.max():.3e} median {np.median(worst):.3e}")
    assert worst.max() < bound
    # ensemble norm against the expectation of the discrete scheme
    diag = plan.diagnostics(d).cpu().numpy()
    N = diag[:, 0]
    N0 = float(np.sum(np.abs(f[0]) ** 2) * g.dV)
    t = w.h * w.nsteps
    m = np.arange(g.n[0])
    k = 2 * np.pi / (g.hi[0] - g.lo[0]) * np.where(m < g.n[0] // 2, m, m - g.n[0])
    Lk = -1j * g.alpha * k * k - g.gamma
    Sk = (np.exp(Lk * w.h) + 4 * np.exp(Lk * w.h / 2) + 1) / 6
    per_step = w.h * g.sigma ** 2 * np.sum(np.abs(Sk) ** 2)
    B = per_step / (1 - np.exp(-2 * g.gamma * w.h))   # stationary noise norm
    A = N0 - B
    EN = A * np.exp(-2 * g.gamma * t) + B
    VN = 2 * g.sigma ** 2 * (A * (np.exp(-2 * g.gamma * t) - np.exp(-4 * g.gamma * t)) / (2 * g.gamma)
                             + B * (1 - np.exp(-4 * g.gamma * t)) / (4 * g.gamma))
    z = (np.mean(N) - EN) / np.sqrt(VN / g.batch)
    zv = (np.var(N, ddof=1) - VN) / (VN * np.sqrt(2.0 / (g.batch - 1)))
    log(f"  E[N] {np.mean(N):.6f} vs {EN:.6f} (z {z:.2f}); Var N {np.var(N, ddof=1):.3e} vs {VN:.3e} (z {zv:.2f})")
    assert abs(z) < 4 and abs(zv) < 4


def test_gpe3d_256_eight_steps_full_size(torch):
    """256^3 with the benchmark's flags: the whole field after 8 steps vs the oracle."""
    w = W.gpe3d(nsteps=8)
    g = w.groups[0]
    log("gpe3d 256^3, 8 steps, graph + autotune, full field vs oracle")
    f = quantised(w.psi0[0])
    plan = _plan(w, BENCH_FLAGS)
    d = torch.tensor(f.astype(np.complex64).reshape(-1), device="cuda")
    plan.run(d, 8)
    ref, _, _ = oracle.run(oprob(g, w.h), f, 8)
    err = rel(_host(d, g.shape), ref)
    log(f"  rel L2 after 8 steps: {err:.3e}")
    assert err < 1e-6


def test_gpe3d_256_full_run_conserves(torch):
    """256^3, 500 steps (the oracle cannot follow it in seconds): no damping and no noise,
    so norm and energy are invariants of the dynamics; the scheme keeps them to O(h^4)
    and FP32 rounding must not move them by more than 1e-5 over the run."""
    w = W.gpe3d()
    log(f"gpe3d 256^3, {w.nsteps} steps, diagnostics every {w.sample_every}")
    plan = _plan(w, BENCH_FLAGS)
    d = rk4ip.field_to_device(w)
    diag, _ = plan.run(d, w.nsteps, sample_every=w.sample_every)
    dg = diag.cpu().numpy()[:, 0, :]
    N = dg[:, 0]
    E = dg[:, 1] + dg[:, 2] + dg[:, 3]
    dN = np.max(np.abs(N / N[0] - 1))
    dE = np.max(np.abs(E / E[0] - 1))
    log(f"  N {N[0]:.9f} -> {N[-1]:.9f} (max drift {dN:.2e}); E {E[0]:.6f} -> {E[-1]:.6f} (max drift {dE:.2e})")
    assert np.all(np.isfinite(dg))
    assert dN < 1e-5 and dE < 1e-5


def test_gpe3d_256_hundred_steps_vs_oracle(torch):
    """256^3 with the benchmark's flags over 100 steps: the whole field against the oracle
    every 25 steps (the graph replays 32-step blocks, so the samples fall inside and
    across replays)."""
    w = W.gpe3d(nsteps=100)
    g = w.groups[0]
    log("gpe3d 256^3, 100 steps, graph + autotune, whole field vs oracle every 25 steps")
    f = quantised(w.psi0[0])
    plan = _plan(w, BENCH_FLAGS)
    d = torch.tensor(f.astype(np.complex64).reshape(-1), device="cuda")
    ref = f.copy()
    p = oprob(g, w.h)
    errs = []
    for s in range(0, 100, 25):
        plan.run(d, 25, step0=s)
        ref, _, _ = oracle.run(p, ref, 25, step0=s)
        errs.append(rel(_host(d, g.shape), ref))
        log(f"  step {s + 25}: rel L2 {errs[-1]:.3e}")
    assert max(errs) < 1e-5


def test_adjoint2d_full_length(torch):
    """The 64-instance uneven batch, 1000 steps, checkpoint every 50, loss
    sum_b 1 - |<phi|psi_b(T)>|^2: psi(T) and both gradients of four instances of each
    size (spread over the group, each with its own id and potential grid) against the
    oracle's forward run and discrete adjoint."""
    from paper_1204_4255_amd.autograd import RK4IPSolver

    w = W.adjoint2d()
    M = w.ckpt_every
    log(f"adjoint2d full batch, {w.nsteps} steps, checkpoint every {M}")
    probs, _k = rk4ip.problems_from_workload(w)
    solver = RK4IPSolver(probs, w.nsteps, M)
    psi0 = rk4ip.field_to_device(w).requires_grad_(True)
    V = torch.tensor(np.concatenate([g.Vgrid.reshape(-1) for g in w.groups]).astype(np.float32), device="cuda",
                     requires_grad=True)
    out = solver(psi0, V)
    loss, off = 0, 0
    for g, phi in zip(w.groups, w.target):
        n = g.batch * g.M
        t = torch.tensor(phi.astype(np.complex64).reshape(-1), device="cuda")
        c = g.dV * torch.sum(torch.conj(t)[None] * out[off:off + n].reshape(g.batch, -1), dim=1)
        loss = loss + torch.sum(1 - torch.abs(c) ** 2)
        off += n
    loss.backward()
    outs = out.detach().cpu().numpy().astype(np.complex128)
    g_psi = psi0.grad.cpu().numpy().astype(np.complex128)
    g_V = V.grad.cpu().numpy().astype(np.float64)
    off = 0
    for g, phi, f in zip(w.groups, w.target, w.psi0):
        for b in (0, 10, 21, g.batch - 1):
            # instance b of the group alone (its own id and potential grid)
            g1 = W.Group(n=g.n, lo=g.lo, hi=g.hi, batch=1, gnl=g.gnl, trap=g.trap, seed=g.seed,
                         id_base=g.id_base + b)
            g1.Vgrid = np.asarray(g.Vgrid[b:b + 1], np.float32).astype(np.float64)
            p = oprob(g1, w.h)
            f1 = quantised(f[b:b + 1])
            ref_T, _, _ = oracle.run(p, f1, w.nsteps)
            c = oracle.overlap(p, phi, ref_T)
            lamT = -2 * g.dV * c[:, None, None] * phi[None]
            ref_g, ref_V = oracle.adjoint(p, f1, lamT, nsteps=w.nsteps, ckpt_every=M)
            sl = slice(off + b * g.M, off + (b + 1) * g.M)
            e0 = rel(outs[sl], ref_T)
            e1 = rel(g_psi[sl], ref_g)
            e2 = rel(g_V[sl], ref_V)
            log(f"  n={g.n} instance {b}: psi_T rel {e0:.2e}, grad_psi0 rel {e1:.2e}, grad_V rel {e2:.2e}")
            assert e0 < 1e-5 and e1 < 1e-5 and e2 < 1e-5
        off += g.batch * g.M


# ----------------------------------------------------------------------------- the semi-implicit form

SI = rk4ip.RK4IP_FLAG_SEMI_IMPLICIT


def test_gpe3d_256_semi_implicit_eight_steps_full_size(torch):
    """256^3 with the benchmark's flags and the semi-implicit step: the whole field after 8
    steps vs the oracle's semi-implicit step."""
    w = W.gpe3d(nsteps=8)
    g = w.groups[0]
    log("gpe3d 256^3, semi-implicit, 8 steps, graph + autotune, full field vs oracle")
    f = quantised(w.psi0[0])
    plan = _plan(w, BENCH_FLAGS | SI)
    d = torch.tensor(f.astype(np.complex64).reshape(-1), device="cuda")
    plan.run(d, 8)
    ref, _, _ = oracle.run(oprob(g, w.h, integrator=1), f, 8)
    err = rel(_host(d, g.shape), ref)
    log(f"  rel L2 after 8 steps: {err:.3e}")
    assert err < 1e-6


@pytest.mark.parametrize("flags,bound", [(0, 1e-5), (F64, 1e-5)], ids=["c64", "fp64"])
def test_sgpe1d_semi_implicit_full_length(torch, flags, bound):
    """2048 paths x 1024, 5000 semi-implicit steps, several steps per launch from a graph:
    16 sampled paths against the oracle's semi-implicit run one by one over the run."""
    w = W.sgpe1d()
    g = w.groups[0]
    log(f"sgpe1d semi-implicit {g.batch} paths x {g.n[0]}, {w.nsteps} steps, flags {flags}")
    plan = _plan(w, rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_FUSE_1D | SI | flags)
    f = quantised(w.psi0[0])
    d = torch.tensor(f.astype(np.complex64).reshape(-1), device="cuda")
    sample = np.linspace(0, g.batch - 1, 16).astype(int)
    refs = {int(b): f[b:b + 1].copy() for b in sample}
    worst = np.zeros(len(sample))
    for s in range(0, w.nsteps, w.sample_every):
        plan.run(d, w.sample_every, step0=s)
        got = _host(d, g.shape)
        for i, b in enumerate(sample):
            gb = W.Group(n=g.n, lo=g.lo, hi=g.hi, batch=1, gnl=g.gnl, gamma=g.gamma, sigma=g.sigma, trap=g.trap,
                         seed=g.seed, id_base=g.id_base + int(b))
            refs[int(b)], _, _ = oracle.run(oprob(gb, w.h, integrator=1), refs[int(b)], w.sample_every, step0=s)
            worst[i] = max(worst[i], rel_per_instance(got[b:b + 1], refs[int(b)], 1)[0])
    log(f"  sampled paths, max rel L2 over the run: max {worst.max():.3e} median {np.median(worst):.3e}")
    assert worst.max() < bound
