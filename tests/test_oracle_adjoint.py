"""Pins of the oracle's tangent-linear model and discrete adjoint.

The paper has no adjoint; these tests pin the oracle's hand-derived transpose of the
RK4IP step to independent facts: (1) the dot-product identity between the tangent and
adjoint models, (2) central finite differences of the FP64 forward run, (3) PyTorch's
CPU autograd through an independently written torch-op RK4IP, (4) the result not
depending on the checkpoint spacing.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1204_4255_amd import workloads as W


def _prob(g, h):
    return oracle.Problem(n=g.n, lo=g.lo, hi=g.hi, h=h, batch=g.batch, alpha=g.alpha, gamma=g.gamma,
                          gnl=g.gnl, trap=g.trap, sigma=g.sigma, seed=g.seed, id_base=g.id_base, Vgrid=g.Vgrid)


def _case(n=(16, 8), batch=2, sigma=0.05, gamma=0.1, seed=4):
    g = W.Group(n=n, lo=(-4.0,) * len(n), hi=(4.0,) * len(n), batch=batch, gnl=3.0, trap=(1.0, 0.7, 0.0),
                gamma=gamma, sigma=sigma, seed=seed)
    r = np.random.Generator(np.random.PCG64(seed))
    g.Vgrid = 0.3 * r.standard_normal((batch, g.M))
    grids = g.mesh()
    env = np.exp(-sum(X ** 2 for X in grids) / 4)
    psi0 = (env * (r.standard_normal(g.shape) + 1j * r.standard_normal(g.shape))).astype(complex)
    return g, psi0, r


def _inner(a, b):
    return float(np.sum(np.real(np.conj(a) * b)))


def test_dot_product_identity():
    g, psi0, r = _case()
    p = _prob(g, 0.02)
    S = 6
    dpsi = r.standard_normal(g.shape) + 1j * r.standard_normal(g.shape)
    dV = r.standard_normal((g.batch, g.M))
    _, dpsiS = oracle.tangent(p, psi0, dpsi, dV, nsteps=S, step0=3)
    lamS = r.standard_normal(g.shape) + 1j * r.standard_normal(g.shape)
    lam0, Vbar = oracle.adjoint(p, psi0, lamS, nsteps=S, ckpt_every=4, step0=3)
    lhs = _inner(lamS, dpsiS)
    rhs = _inner(lam0, dpsi) + float(np.sum(Vbar.reshape(g.batch, -1) * dV))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def _loss(p, psi0, phi, S, step0=0):
    out, _, _ = oracle.run(p, psi0, S, step0=step0)
    dV = np.prod([(p.hi[a] - p.lo[a]) / p.n[a] for a in range(p.ndim)])
    c = dV * np.sum(np.conj(phi)[None] * out, axis=tuple(range(1, out.ndim)))
    return float(np.sum(1 - np.abs(c) ** 2)), c, dV


def test_central_finite_differences():
    g, psi0, r = _case(sigma=0.0)
    S = 5
    grids = g.mesh()
    phi = np.exp(-((grids[0] - 0.5) ** 2 + grids[1] ** 2) / 2).astype(complex)
    p = _prob(g, 0.02)
    _, c, dV = _loss(p, psi0, phi, S)
    lamS = (-2 * dV * c[:, None, None]) * phi[None]
    grad, Vbar = oracle.adjoint(p, psi0, lamS, nsteps=S, ckpt_every=2)
    eps = 1e-4
    for trial in range(3):
        d = r.standard_normal(g.shape) + 1j * r.standard_normal(g.shape)
        lp, _, _ = _loss(p, psi0 + eps * d, phi, S)
        lm, _, _ = _loss(p, psi0 - eps * d, phi, S)
        fd = (lp - lm) / (2 * eps)
        an = _inner(grad, d)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (fd, an)
    # potential grid: random direction and a single entry
    base_V = g.Vgrid.copy()
    for trial in range(2):
        if trial == 0:
            dv = r.standard_normal(base_V.shape)
        else:
            dv = np.zeros_like(base_V)
            dv[1, g.M // 2 + 3] = 1.0
        g.Vgrid = base_V + eps * dv
        lp, _, _ = _loss(_prob(g, 0.02), psi0, phi, S)
        g.Vgrid = base_V - eps * dv
        lm, _, _ = _loss(_prob(g, 0.02), psi0, phi, S)
        g.Vgrid = base_V
        fd = (lp - lm) / (2 * eps)
        an = float(np.sum(Vbar.reshape(dv.shape) * dv))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-6), (fd, an)


def _torch_rk4ip(psi0, V, xi_steps, k2, h, gnl, gamma, sigma, alpha, dims):
    """An independent torch-op RK4IP with the same midpoint-origin reading."""
    E = torch.exp((-1j * alpha * k2 - gamma) * h / 2)

    def D(f):
        return torch.fft.ifftn(E * torch.fft.fftn(f, dim=dims), dim=dims)

    def hG(f, xi):
        return h * (-1j * (V + gnl * (f.real ** 2 + f.imag ** 2)) * f + sigma * xi)

    psi = psi0
    for xi in xi_steps:
        a = D(psi)
        k1 = D(hG(psi, xi))
        k2_ = hG(a + k1 / 2, xi)
        k3 = hG(a + k2_ / 2, xi)
        k4 = hG(D(a + k3), xi)
        psi = D(a + k1 / 6 + k2_ / 3 + k3 / 3) + k4 / 6
    return psi


def test_matches_torch_cpu_autograd():
    torch.manual_seed(0)
    g, psi0, r = _case(n=(16, 16), batch=2, sigma=0.1, gamma=0.05)
    h, S, step0 = 0.02, 4, 2
    p = _prob(g, h)
    grids = g.mesh()
    phi = np.exp(-((grids[0] - 0.5) ** 2 + grids[1] ** 2) / 2).astype(complex)
    # wavenumbers on the spectral lattice
    ks = [2 * np.pi / (g.hi[a] - g.lo[a]) * np.fft.fftfreq(g.n[a], d=1.0 / g.n[a]) for a in range(2)]
    KY, KX = np.meshgrid(ks[1], ks[0], indexing="ij")
    k2 = torch.tensor(KX ** 2 + KY ** 2)
    X, Y = grids
    V = torch.tensor(0.5 * (g.trap[0] * X ** 2 + g.trap[1] * Y ** 2))[None] + torch.tensor(
        g.Vgrid.reshape(g.shape), requires_grad=False)
    Vg = torch.tensor(g.Vgrid.reshape(g.shape), requires_grad=True)
    Vt = V - V.detach() + torch.tensor(0.5 * (g.trap[0] * X ** 2 + g.trap[1] * Y ** 2))[None] + Vg
    xi_steps = [torch.tensor(oracle.noise(p, step0 + s)) for s in range(S)]
    x0 = torch.tensor(psi0, requires_grad=True)
    out = _torch_rk4ip(x0, Vt, xi_steps, k2, h, g.gnl, g.gamma, g.sigma, 0.5, (-2, -1))
    ref_out, _, _ = oracle.run(p, psi0, S, step0=step0)
    assert np.max(np.abs(out.detach().numpy() - ref_out)) < 1e-12
    dV = g.dV
    c = dV * torch.sum(torch.conj(torch.tensor(phi))[None] * out, dim=(-2, -1))
    loss = torch.sum(1 - torch.abs(c) ** 2)
    loss.backward()
    lamS = (-2 * dV * c.detach().numpy()[:, None, None]) * phi[None]
    grad, Vbar = oracle.adjoint(p, psi0, lamS, nsteps=S, ckpt_every=3, step0=step0)
    gt = x0.grad.numpy()
    assert np.linalg.norm(grad - gt) <= 1e-10 * np.linalg.norm(gt)
    vt = Vg.grad.numpy()
    assert np.linalg.norm(Vbar - vt) <= 1e-10 * np.linalg.norm(vt)


def test_torch_gradient_convention():
    z = torch.tensor(1.0 + 1.0j, requires_grad=True)
    (z.real ** 2 + z.imag ** 2).backward()
    assert complex(z.grad) == 2 + 2j   # d/dRe + i d/dIm


def test_checkpoint_spacing_does_not_change_result():
    g, psi0, r = _case(n=(8, 8), batch=1)
    p = _prob(g, 0.03)
    lamS = r.standard_normal(g.shape) + 1j * r.standard_normal(g.shape)
    ref = oracle.adjoint(p, psi0, lamS, nsteps=7, ckpt_every=7)
    for M in (1, 2, 3, 10):
        out = oracle.adjoint(p, psi0, lamS, nsteps=7, ckpt_every=M)
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1])


@pytest.mark.parametrize("n", [(32,), (8, 8, 4)])
def test_dot_product_identity_1d_3d(n):
    g, psi0, r = _case(n=n, batch=1)
    p = _prob(g, 0.02)
    dpsi = r.standard_normal(g.shape) + 1j * r.standard_normal(g.shape)
    dV = r.standard_normal((1, g.M))
    _, dpsiS = oracle.tangent(p, psi0, dpsi, dV, nsteps=3)
    lamS = r.standard_normal(g.shape) + 1j * r.standard_normal(g.shape)
    lam0, Vbar = oracle.adjoint(p, psi0, lamS, nsteps=3, ckpt_every=2)
    lhs = _inner(lamS, dpsiS)
    rhs = _inner(lam0, dpsi) + float(np.sum(Vbar.reshape(1, -1) * dV))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
