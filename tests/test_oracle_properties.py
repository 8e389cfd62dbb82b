"""Property pins of the oracle's propagator D = e^{L h/2} (Sec. 3.6), over random lattices,
parameters and fields (hypothesis): without damping it is unitary in every basis and its
transpose undoes it; its transpose is its adjoint for the complex inner product; on a
Fourier lattice it commutes with translations by lattice vectors; without the kinetic
term it is the damping factor alone."""
import numpy as np
from hypothesis import given, settings, strategies as st

import oracle

SETTINGS = settings(max_examples=25, deadline=None)


def _field(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@st.composite
def lattices(draw, bases=(0,)):
    basis = draw(st.sampled_from(bases))
    nd = 1 if basis else draw(st.integers(1, 3))
    n = tuple(2 ** draw(st.integers(1, 5 if nd < 3 else 3)) for _ in range(nd))
    L = tuple(draw(st.floats(1.0, 20.0)) for _ in range(nd))
    lo = tuple(draw(st.floats(-10.0, 0.0)) for _ in range(nd))
    h = draw(st.floats(1e-3, 0.5))
    alpha = draw(st.floats(0.1, 2.0))
    batch = draw(st.integers(1, 3))
    seed = draw(st.integers(0, 2 ** 31))
    return dict(n=n, lo=lo, hi=tuple(a + b for a, b in zip(lo, L)), h=h, alpha=alpha, batch=batch,
                basis=basis), seed


@SETTINGS
@given(lattices(bases=(0, 1, 2)))
def test_undamped_propagator_is_unitary_and_its_transpose_undoes_it(case):
    kw, seed = case
    p = oracle.Problem(**kw)
    f = _field(np.random.Generator(np.random.PCG64(seed)), p.shape)
    d = oracle.apply_D(p, f)
    assert abs(np.linalg.norm(d) / np.linalg.norm(f) - 1) < 1e-12
    back = oracle.apply_D(p, d, adjoint=True)
    assert np.linalg.norm(back - f) < 1e-11 * np.linalg.norm(f)


@SETTINGS
@given(lattices(bases=(0, 1, 2)), st.floats(0.0, 3.0))
def test_transpose_is_the_adjoint(case, gamma):
    kw, seed = case
    p = oracle.Problem(gamma=gamma, **kw)
    rng = np.random.Generator(np.random.PCG64(seed))
    f, g = _field(rng, p.shape), _field(rng, p.shape)
    lhs = np.vdot(g, oracle.apply_D(p, f))
    rhs = np.vdot(oracle.apply_D(p, g, adjoint=True), f)
    assert abs(lhs - rhs) < 1e-11 * np.linalg.norm(f) * np.linalg.norm(g)


@SETTINGS
@given(lattices(), st.integers(-7, 7))
def test_fourier_propagator_commutes_with_lattice_translations(case, shift):
    kw, seed = case
    p = oracle.Problem(**kw)
    f = _field(np.random.Generator(np.random.PCG64(seed)), p.shape)
    axis = p.ndim  # the last numpy axis is lattice axis 0
    a = oracle.apply_D(p, np.roll(f, shift, axis=axis))
    b = np.roll(oracle.apply_D(p, f), shift, axis=axis)
    assert np.linalg.norm(a - b) < 1e-11 * np.linalg.norm(f)


@SETTINGS
@given(lattices(bases=(0, 1, 2)), st.floats(0.01, 3.0))
def test_without_the_kinetic_term_only_the_damping_is_left(case, gamma):
    kw, seed = case
    kw = dict(kw, alpha=0.0)
    p = oracle.Problem(gamma=gamma, **kw)
    f = _field(np.random.Generator(np.random.PCG64(seed)), p.shape)
    d = oracle.apply_D(p, f)
    assert np.linalg.norm(d - np.exp(-gamma * kw["h"] / 2) * f) < 1e-12 * np.linalg.norm(f)


@SETTINGS
@given(lattices(bases=(0, 1, 2)), st.floats(-5.0, 5.0), st.floats(0.0, 2.0 * np.pi), st.sampled_from([0, 1]))
def test_a_global_phase_commutes_with_the_step(case, gnl, phase, integrator):
    # G depends on |psi|^2 only, so without noise step(e^{i c} psi) = e^{i c} step(psi)
    kw, seed = case
    kw = dict(kw, h=min(kw["h"], 0.05))
    p = oracle.Problem(gnl=gnl, trap=(1.0, 0.5, 0.3), gamma=0.1, integrator=integrator, **kw)
    f = 0.5 * _field(np.random.Generator(np.random.PCG64(seed)), p.shape)
    a = oracle.step(p, np.exp(1j * phase) * f)
    b = np.exp(1j * phase) * oracle.step(p, f)
    assert np.linalg.norm(a - b) < 1e-11 * np.linalg.norm(b)
