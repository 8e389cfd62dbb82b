"""GPU parity of the cosine and sine bases on a half domain (Sec. 3.1: even and odd
boundary conditions; the half-interval example of Sec. 4 runs the trapped 1D GPE on
(0, 7) with the cosine transform and half the points) against the FP64 oracle, which
applies the propagator through the DCT-II / DST-II sums themselves."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, quantised, rel, rel_per_instance
from paper_1204_4255_amd import rk4ip

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


def _case(n, batch, basis, L=7.0, sigma=0.01):
    x = (np.arange(n) + 0.5) * L / n
    w = np.linspace(0.8, 1.2, batch)[:, None]
    g = np.exp(-(w * x[None]) ** 2 / 2) * np.exp(0.3j * x[None] ** 2)
    f0 = quantised(g if basis == 1 else x[None] * g)
    kw = dict(h=1e-3, gnl=2.0, trap=(1.0, 0, 0), gamma=0.05, sigma=sigma, seed=19, id_base=6)
    return f0, kw


def _plan(n, batch, basis, kw, flags, L=7.0, Vgrid=None):
    p = rk4ip.make_problem((n,), (0.0,), (L,), kw["h"], batch=batch, gamma=kw["gamma"], g_nl=kw["gnl"],
                           trap=kw["trap"], sigma=kw["sigma"], seed=kw["seed"], id_base=kw["id_base"], basis=basis,
                           V_grid=Vgrid)
    return rk4ip.Plan([p], flags=flags)


def _oprob(n, batch, basis, kw, flags, L=7.0, Vgrid=None):
    return oracle.Problem(n=(n,), lo=(0.0,), hi=(L,), batch=batch, basis=basis,
                          integrator=1 if flags & SI else 0,
                          Vgrid=None if Vgrid is None else Vgrid.cpu().numpy().astype(np.float64), **kw)


@pytest.mark.parametrize("basis", [1, 2])
@pytest.mark.parametrize("n,batch", [(8, 3), (64, 5), (256, 2), (1024, 2), (2048, 1)])
@pytest.mark.parametrize("si", [False, True])
def test_one_step_matches_oracle(torch, basis, n, batch, si):
    log(f"basis {basis}: one step n={n} batch={batch} si={si}")
    f0, kw = _case(n, batch, basis)
    rng = np.random.Generator(np.random.PCG64(2))
    Vg = torch.tensor((0.1 * rng.standard_normal((batch, n))).astype(np.float32), device="cuda")
    flags = SI if si else 0
    plan = _plan(n, batch, basis, kw, flags, Vgrid=Vg)
    d = _dev(torch, f0)
    plan.step(d, 23)
    torch.cuda.synchronize()
    ref = oracle.step(_oprob(n, batch, basis, kw, flags, Vgrid=Vg), f0, 23)
    err = rel_per_instance(_host(d, f0.shape), ref, batch)
    log(f"  max rel {np.max(err):.2e}")
    assert np.max(err) < 1e-6, err


@pytest.mark.parametrize("basis", [1, 2])
@pytest.mark.parametrize("extra", [0, rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_FUSE_1D, F64,
                                   rk4ip.RK4IP_FLAG_AUTOTUNE | rk4ip.RK4IP_FLAG_GRAPH])
@pytest.mark.parametrize("si", [False, True])
def test_runs_resume_and_oracle(torch, basis, extra, si):
    log(f"basis {basis}: runs flags={extra} si={si}")
    n, batch = 256, 4
    f0, kw = _case(n, batch, basis)
    flags = (SI if si else 0) | extra
    plan = _plan(n, batch, basis, kw, flags)
    b = _dev(torch, f0)
    plan.run(b, 50, step0=11)
    c = _dev(torch, f0)
    plan.run(c, 21, step0=11)
    plan.run(c, 29, step0=32)
    torch.cuda.synchronize()
    assert torch.equal(b, c)
    ref, _, _ = oracle.run(_oprob(n, batch, basis, kw, flags), f0, 50, step0=11)
    err = rel(_host(b, f0.shape), ref)
    log(f"  rel {err:.2e}")
    assert err < (2e-6 if extra & F64 else 5e-6)


def test_half_domain_cosine_equals_the_full_domain(torch):
    """The half-interval example's point: the trapped 1D GPE on (0, 7) with 256 cosine
    points gives, on the GPU, the right half of the same problem on (-7, 7) with 512
    Fourier points at the mirrored cell centres (deterministic, 400 steps)."""
    n, L, h, S = 256, 7.0, 1e-3, 400
    dx = L / n
    x = (np.arange(n) + 0.5) * dx
    f_half = quantised(np.pi ** -0.25 * np.exp(-x ** 2 / 2) * np.exp(0.2j * x ** 2))[None]
    half = rk4ip.Plan([rk4ip.make_problem((n,), (0.0,), (L,), h, g_nl=5.0, trap=(1.0, 0, 0), basis=1)],
                      flags=rk4ip.RK4IP_FLAG_GRAPH)
    full = rk4ip.Plan([rk4ip.make_problem((2 * n,), (-L + dx / 2,), (L + dx / 2,), h, g_nl=5.0, trap=(1.0, 0, 0))],
                      flags=rk4ip.RK4IP_FLAG_GRAPH)
    f_full = np.concatenate([f_half[0][::-1], f_half[0]])[None]
    a = _dev(torch, f_half)
    b = _dev(torch, f_full)
    half.run(a, S)
    full.run(b, S)
    ha = _host(a, (1, n))[0]
    hb = _host(b, (1, 2 * n))[0]
    # each complex64 run against its FP64 oracle (the two oracles agree to 1e-12), then
    # the two independent runs against each other
    oh, _, _ = oracle.run(oracle.Problem(n=(n,), lo=(0.0,), hi=(L,), h=h, gnl=5.0, trap=(1.0, 0, 0), basis=1),
                          f_half, S)
    of, _, _ = oracle.run(oracle.Problem(n=(2 * n,), lo=(-L + dx / 2,), hi=(L + dx / 2,), h=h, gnl=5.0,
                                         trap=(1.0, 0, 0)), f_full, S)
    e_half, e_full, err = rel(ha, oh[0]), rel(hb, of[0]), rel(ha, hb[n:])
    log(f"  after {S} steps: half-domain cosine vs oracle {e_half:.2e}, full-domain Fourier vs oracle "
        f"{e_full:.2e}, half vs full {err:.2e}")
    assert rel(oh[0], of[0, n:]) < 1e-12
    assert e_half < 5e-6 and e_full < 5e-6
    assert err < 1e-5


def test_other_entry_points_refuse_basis_plans(torch):
    f0, kw = _case(64, 2, 1)
    plan = _plan(64, 2, 1, kw, 0)
    d = _dev(torch, f0)
    for call in (lambda: plan.diagnostics(d), lambda: plan.run(d, 4, sample_every=2), lambda: plan.moments(0, d),
                 lambda: plan.overlap(0, d[:64], d), lambda: plan.apply_D(d)):
        with pytest.raises(rk4ip.Rk4ipError):
            call()
    h = torch.full((2,), 1e-3, dtype=torch.float64, device="cuda")
    with pytest.raises(rk4ip.Rk4ipError):
        plan.ark45(d, 0.1, 1e-6, h)
