"""Pin of the oracle's noise handling in both integrators by a closed form: for
d psi/dt = L psi + sigma xi with xi constant over a step (V = 0, g = 0) every stage is
linear, and one RK4IP step is exactly psi <- e^{Lh} psi + h sigma (e^{Lh} + 4 e^{Lh/2} + 1)
xi / 6 (Simpson's rule), one semi-implicit step psi <- e^{Lh} psi + h sigma e^{Lh/2} xi
(the midpoint rule). A wrong stage weight, a noise term missing from a stage, or xi
drawn at the wrong step breaks the equality."""
import numpy as np
import pytest

import oracle
from closed_forms import non_local_case, plane_wave_amplitude


@pytest.mark.parametrize("dims", [1, 2])
@pytest.mark.parametrize("integrator", [0, 1])
def test_linear_sde_step_is_simpson_or_midpoint(dims, integrator):
    n = (64,) if dims == 1 else (16, 8)
    lo, hi = (-8.0,) * dims, (8.0,) * dims
    batch, h, S, sig, gam, alpha = 2, 1e-3, 12, 0.2, 0.05, 0.5
    op = oracle.Problem(n=n, lo=lo, hi=hi, h=h, batch=batch, alpha=alpha, gamma=gam, sigma=sig, seed=77,
                        id_base=2, integrator=integrator)
    ax = [lo[a] + np.arange(n[a]) * (hi[a] - lo[a]) / n[a] for a in range(dims)]
    env = np.exp(-ax[0] ** 2 / 2) if dims == 1 else np.exp(-ax[0][None, :] ** 2 / 2 - ax[1][:, None] ** 2 / 2)
    psi0 = np.broadcast_to(env, (batch,) + env.shape).astype(complex)
    ks = [2 * np.pi * np.fft.fftfreq(n[a], d=(hi[a] - lo[a]) / n[a]) for a in range(dims)]
    k2 = ks[0] ** 2 if dims == 1 else ks[0][None, :] ** 2 + ks[1][:, None] ** 2
    Lk = -1j * alpha * k2 - gam
    fax = tuple(range(1, dims + 1))
    E1, Eh = np.exp(Lk * h), np.exp(Lk * h / 2)
    w = h * sig * ((E1 + 4 * Eh + 1) / 6 if integrator == 0 else Eh)
    f = np.fft.fftn(psi0, axes=fax)
    for s in range(S):
        f = E1 * f + w * np.fft.fftn(oracle.noise(op, 5 + s), axes=fax)
    exact = np.fft.ifftn(f, axes=fax)
    ref, _, _ = oracle.run(op, psi0, S, step0=5)
    assert np.linalg.norm(ref - exact) / np.linalg.norm(exact) < 1e-13
    # the other integrator's weights do not fit: the pin tells the two apart
    w2 = h * sig * (Eh if integrator == 0 else (E1 + 4 * Eh + 1) / 6)
    g = np.fft.fftn(psi0, axes=fax)
    for s in range(S):
        g = E1 * g + w2 * np.fft.fftn(oracle.noise(op, 5 + s), axes=fax)
    assert np.linalg.norm(ref - np.fft.ifftn(g, axes=fax)) / np.linalg.norm(exact) > 1e-8


@pytest.mark.parametrize("integrator", [0, 1])
def test_non_local_potential_on_plane_waves(integrator):
    """A plane wave's density is uniform, so the non-local potential is the constant
    |A|^2 dV sum_d K(d): the oracle's run equals the same step applied to the scalar
    amplitude equation, and differs from the run without the non-local term."""
    gam, alpha, h, S = 0.05, 0.5, 2e-3, 40
    n, L, gnl, dx, K, qs, amps, psi0 = non_local_case()
    op = oracle.Problem(n=(n,), lo=(-L / 2,), hi=(L / 2,), h=h, batch=len(qs), alpha=alpha, gamma=gam, gnl=gnl,
                        convK=K, integrator=integrator)
    ref, _, _ = oracle.run(op, psi0, S)
    for i, q in enumerate(qs):
        E = np.exp((-1j * alpha * (2 * np.pi * q / L) ** 2 - gam) * h / 2)
        A0 = psi0[i, 0]
        want = plane_wave_amplitude(A0, S, h, E, gnl + dx * K.sum(), integrator) / A0 * psi0[i]
        local = plane_wave_amplitude(A0, S, h, E, gnl, integrator) / A0 * psi0[i]
        assert np.linalg.norm(ref[i] - want) / np.linalg.norm(want) < 1e-13
        assert np.linalg.norm(ref[i] - local) / np.linalg.norm(want) > 1e-2
