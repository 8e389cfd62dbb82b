"""Pins of the oracle's cosine and sine bases on a half domain (Sec. 3.1: even and odd
boundary conditions; the half-interval example of Sec. 4 uses the cosine transform).

They rest on the Fourier oracle, pinned on its own: a problem symmetric about the origin
and integrated on the full domain with the Fourier basis, on a lattice whose points are
the mirror images of the half domain's cell centres, must give on the right half exactly
what the cosine (even data) or sine (odd data) basis gives on the half domain alone; and
on a single cosine mode, whose free evolution is a closed form."""
import numpy as np
import pytest

import oracle


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def _half_and_full(n, L, basis, integrator, **kw):
    dx = L / n
    half = oracle.Problem(n=(n,), lo=(0.0,), hi=(L,), basis=basis, integrator=integrator, **kw)
    # the full periodic domain of length 2L whose lattice points are +-(j + 1/2) dx
    full = oracle.Problem(n=(2 * n,), lo=(-L + dx / 2,), hi=(L + dx / 2,), integrator=integrator, **kw)
    xh = (np.arange(n) + 0.5) * dx
    xf = -L + dx / 2 + np.arange(2 * n) * dx
    return half, full, xh, xf


@pytest.mark.parametrize("integrator", [0, 1])
@pytest.mark.parametrize("basis", [1, 2])
def test_half_domain_equals_the_mirrored_full_domain(basis, integrator):
    n, L = 64, 7.0
    kw = dict(h=2e-3, gnl=3.0, trap=(1.0, 0, 0), gamma=0.1)
    half, full, xh, xf = _half_and_full(n, L, basis, integrator, **kw)

    def f0(x):
        g = np.exp(-(x ** 2) / 2) * np.exp(0.4j * x ** 2)
        return g if basis == 1 else x * g  # even or odd about the origin

    a, _, _ = oracle.run(half, f0(xh)[None], 40)
    b, _, _ = oracle.run(full, f0(xf)[None], 40)
    assert np.allclose(xf[n:], xh)
    assert rel(a[0], b[0, n:]) < 1e-12
    # and the left half of the full run is the mirror image
    sign = 1.0 if basis == 1 else -1.0
    assert rel(b[0, :n][::-1] * sign, b[0, n:]) < 1e-12


@pytest.mark.parametrize("m", [0, 3, 17])
def test_a_cosine_mode_evolves_by_its_closed_form(m):
    # G = 0: cos(k_m x) with k_m = pi m / L is an eigenfunction of L, so after S steps it
    # is exp((-i alpha k_m^2 - gamma) S h) cos(k_m x)
    n, L, h, S, gam = 32, 5.0, 0.01, 25, 0.2
    p = oracle.Problem(n=(n,), lo=(0.0,), hi=(L,), h=h, gamma=gam, basis=1)
    x = (np.arange(n) + 0.5) * L / n
    k = np.pi * m / L
    out, _, _ = oracle.run(p, np.cos(k * x)[None] + 0j, S)
    assert rel(out[0], np.exp((-0.5j * k * k - gam) * S * h) * np.cos(k * x)) < 1e-12


def test_the_highest_sine_mode_is_kept():
    # the sine basis carries k = pi n / L (the alternating sequence on the cell centres)
    n, L, h = 16, 3.0, 0.01
    p = oracle.Problem(n=(n,), lo=(0.0,), hi=(L,), h=h, basis=2)
    x = (np.arange(n) + 0.5) * L / n
    k = np.pi * n / L
    out, _, _ = oracle.run(p, np.sin(k * x)[None] + 0j, 3)
    assert rel(out[0], np.exp(-0.5j * k * k * 3 * h) * np.sin(k * x)) < 1e-12


def test_bases_are_one_dimensional_and_local():
    with pytest.raises(ValueError):
        oracle.step(oracle.Problem(n=(8, 8), lo=(0, 0), hi=(1, 1), h=0.01, basis=1), np.ones((1, 8, 8), complex))
    with pytest.raises(ValueError):
        oracle.step(oracle.Problem(n=(8,), lo=(0,), hi=(1,), h=0.01, basis=1, convK=np.ones(8)), np.ones((1, 8), complex))
