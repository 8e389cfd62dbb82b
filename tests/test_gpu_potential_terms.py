"""GPU parity of the potential's extra terms against the FP64 oracle: the real Wiener noise
in the potential (the stochastics example of Sec. 4; 1D, 2D and 3D) and the non-local
potential, a convolution of the density with a kernel (the non-local example of Sec. 4;
1D), under the RK4IP and the semi-implicit step, in both precision forms, through graphs,
fused launches and resumed runs."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, quantised, rel, rel_per_instance
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


def _kernel(n, L, a=1.0):
    # a softened Coulomb kernel 1/sqrt(d^2 + a^2) at the lattice offsets (d >= n/2 wraps)
    d = np.arange(n)
    d = np.where(d < n // 2, d, d - n) * (L / n)
    return 1.0 / np.sqrt(d ** 2 + a ** 2)


def _case(n, batch, sigma_V, conv, sigma=0.01, L=16.0, seed=31):
    g = W.Group(n=(n,), lo=(-L / 2,), hi=(L / 2,), batch=batch, gnl=1.0, trap=(1.0, 0, 0), gamma=0.05,
                sigma=sigma, seed=seed, id_base=4)
    x = g.axis(0)
    shift = np.linspace(-1.0, 1.0, batch)[:, None]
    f0 = quantised(np.pi ** -0.25 * np.exp(-(x[None] - shift) ** 2 / 2) * np.exp(0.3j * x[None]))
    K = _kernel(n, L) if conv else None
    return g, f0, K


def _plans(g, h, K, sigma_V, flags, S=1):
    p = rk4ip.make_problem(g.n, g.lo, g.hi, h, batch=g.batch, alpha=g.alpha, gamma=g.gamma, g_nl=g.gnl, trap=g.trap,
                           sigma=g.sigma, seed=g.seed, id_base=g.id_base, noise_substeps=S, sigma_V=sigma_V,
                           conv_K=K)
    plan = rk4ip.Plan([p], flags=flags)
    op = oracle.Problem(n=g.n, lo=g.lo, hi=g.hi, h=h, batch=g.batch, alpha=g.alpha, gamma=g.gamma, gnl=g.gnl,
                        trap=g.trap, sigma=g.sigma, seed=g.seed, id_base=g.id_base, noise_substeps=S,
                        sigma_V=sigma_V, convK=K, integrator=1 if flags & SI else 0)
    return plan, op


def _dev(torch, a):
    return torch.tensor(np.asarray(a, dtype=np.complex64).reshape(-1), device="cuda")


def _host(t, shape):
    return t.cpu().numpy().astype(np.complex128).reshape(shape)


@pytest.mark.parametrize("sigma_V,conv", [(0.5, False), (0.0, True), (0.5, True)])
@pytest.mark.parametrize("n,batch", [(8, 3), (64, 5), (256, 9), (1024, 2), (4096, 1)])
@pytest.mark.parametrize("si", [False, True])
def test_one_step_matches_oracle(torch, n, batch, sigma_V, conv, si):
    log(f"potential terms: n={n} batch={batch} sigma_V={sigma_V} conv={conv} si={si}")
    g, f0, K = _case(n, batch, sigma_V, conv)
    plan, op = _plans(g, 2e-3, K, sigma_V, SI if si else 0)
    d = _dev(torch, f0)
    plan.step(d, 17)
    torch.cuda.synchronize()
    ref = oracle.step(op, f0, 17)
    err = rel_per_instance(_host(d, g.shape), ref, batch)
    log(f"  max rel {np.max(err):.2e}")
    assert np.max(err) < 1e-6, err


@pytest.mark.parametrize("extra", [0, rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_FUSE_1D, F64,
                                   F64 | rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_FUSE_1D])
@pytest.mark.parametrize("si", [False, True])
@pytest.mark.parametrize("S", [1, 2])
def test_runs_resume_and_oracle(torch, extra, si, S):
    """Eager, graph-replayed and fused, and resumed runs agree bitwise and with the oracle's
    run (a noisy trapped GPE with the non-local potential, 60 steps)."""
    log(f"potential terms runs: flags={extra} si={si} substeps={S}")
    g, f0, K = _case(256, 4, 0.3, True, sigma=0.02)
    base, op = _plans(g, 1e-3, K, 0.3, (SI if si else 0) | (extra & F64), S)
    plan, _ = _plans(g, 1e-3, K, 0.3, (SI if si else 0) | extra, S)
    a = _dev(torch, f0)
    base.run(a, 60, step0=7)
    b = _dev(torch, f0)
    plan.run(b, 60, step0=7)
    c = _dev(torch, f0)
    plan.run(c, 25, step0=7)
    plan.run(c, 35, step0=32)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(b, c)
    ref, _, _ = oracle.run(op, f0, 60, step0=7)
    err = rel(_host(b, g.shape), ref)
    log(f"  rel {err:.2e}")
    assert err < (2e-6 if extra & F64 else 5e-6)


@pytest.mark.parametrize("n,batch", [((64, 32), 2), ((16, 128), 1), ((32, 16, 8), 2), ((128, 8, 16), 1)])
@pytest.mark.parametrize("si", [False, True])
def test_noisy_potential_on_lattices(torch, n, batch, si):
    """The noise in the potential on 2D and 3D lattices (the per-axis passes): one step and
    a graph-replayed run that splits and resumes, against the oracle."""
    log(f"noisy potential: n={n} batch={batch} si={si}")
    nd = len(n)
    g = W.Group(n=n, lo=(-4.0,) * nd, hi=(4.0,) * nd, batch=batch, gnl=2.0, trap=(1.0, 1.2, 0.8), gamma=0.05,
                sigma=0.01, seed=23, id_base=1)
    x = g.mesh()
    env = np.exp(-sum(X ** 2 for X in x) / 2)
    f0 = quantised(np.broadcast_to(env * np.exp(0.2j * x[0]), g.shape))
    h, sv = 1e-3, 0.4
    flags = SI if si else 0
    p = rk4ip.make_problem(g.n, g.lo, g.hi, h, batch=batch, alpha=g.alpha, gamma=g.gamma, g_nl=g.gnl, trap=g.trap,
                           sigma=g.sigma, seed=g.seed, id_base=g.id_base, sigma_V=sv)
    op = oracle.Problem(n=g.n, lo=g.lo, hi=g.hi, h=h, batch=batch, alpha=g.alpha, gamma=g.gamma, gnl=g.gnl,
                        trap=g.trap, sigma=g.sigma, seed=g.seed, id_base=g.id_base, sigma_V=sv,
                        integrator=1 if si else 0)
    plan = rk4ip.Plan([p], flags=flags)
    d = _dev(torch, f0)
    plan.step(d, 9)
    torch.cuda.synchronize()
    err = rel_per_instance(_host(d, g.shape), oracle.step(op, f0, 9), batch)
    log(f"  one step max rel {np.max(err):.2e}")
    assert np.max(err) < 1e-6
    graph = rk4ip.Plan([p], flags=flags | rk4ip.RK4IP_FLAG_GRAPH)
    a = _dev(torch, f0)
    graph.run(a, 40, step0=3)
    b = _dev(torch, f0)
    plan.run(b, 17, step0=3)
    plan.run(b, 23, step0=20)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    ref, _, _ = oracle.run(op, f0, 40, step0=3)
    err = rel(_host(a, g.shape), ref)
    log(f"  40 steps rel {err:.2e}")
    assert err < 5e-6


@pytest.mark.parametrize("n,si", [((256,), False), ((256,), True), ((32, 16), False), ((16, 8, 8), False),
                                  ((16, 8, 8), True)])
def test_potential_noise_is_the_oracles(torch, n, si):
    """A step with only the noisy potential (alpha = 0, g = 0, V = 0) multiplies every
    point by the RK4 factor of e^{-i h sigma_V eta} (the semi-implicit step: by
    1 + z + z^2/2 + z^3/4), with eta the oracle's real noise at that step and point."""
    batch, h, sv = 4, 0.01, 0.2
    nd = len(n)
    g = W.Group(n=n, lo=(-4.0,) * nd, hi=(4.0,) * nd, batch=batch, alpha=0.0, seed=12)
    p = rk4ip.make_problem(g.n, g.lo, g.hi, h, batch=batch, alpha=0.0, seed=12, sigma_V=sv)
    plan = rk4ip.Plan([p], flags=SI if si else 0)
    f0 = np.ones(g.shape, complex)
    d = _dev(torch, f0)
    plan.step(d, 5)
    got = _host(d, g.shape).reshape(batch, -1)
    op = oracle.Problem(n=g.n, lo=g.lo, hi=g.hi, h=h, batch=batch, alpha=0.0, seed=12, sigma_V=sv)
    eta = oracle.vnoise(op, 5)
    z = -1j * h * sv * eta
    factor = 1 + z + z ** 2 / 2 + (z ** 3 / 4 if si else z ** 3 / 6 + z ** 4 / 24)
    err = np.max(np.abs(got - factor))
    log(f"noisy potential alone n={n} si={si}: max |step - closed form| {err:.2e}, max |z| {np.max(np.abs(z)):.2f}")
    assert err < 1e-6


def test_unsupported_combinations_are_rejected(torch):
    with pytest.raises(rk4ip.Rk4ipError):
        rk4ip.Plan([rk4ip.make_problem((16, 16), (0, 0), (1, 1), 1e-3, conv_K=np.ones(16))])
    g, f0, K = _case(64, 2, 0.2, True)
    plan, _ = _plans(g, 1e-3, K, 0.2, 0)
    d = _dev(torch, f0)
    _, ck = plan.run(d, 4, ckpt_every=2)
    with pytest.raises(rk4ip.Rk4ipError) as e:
        plan.adjoint(ck, 4, 2, torch.ones_like(d))
    assert e.value.status == rk4ip.RK4IP_ERR_INVALID_ARG
    h = torch.full((2,), 1e-3, dtype=torch.float64, device="cuda")
    with pytest.raises(rk4ip.Rk4ipError) as e:
        plan.ark45(d, 0.1, 1e-6, h)  # noisy: the adaptive integrator is deterministic
    assert e.value.status == rk4ip.RK4IP_ERR_INVALID_ARG
