"""Pins of the oracle's adaptive Cash-Karp RK4(5) in the interaction picture (Sec. 3.5's
adaptive fourth-fifth order Runge-Kutta, Sec. 3.6's interaction picture).

Each test rests on something other than the oracle's own code: the Runge-Kutta order
conditions that the published pair must satisfy, the local error orders on a problem
with a closed-form solution, the exact free evolution (where the error estimate must
vanish and the step grow by the controller's maximum factor), the exact NLSE soliton,
and the property the paper's step-count figure shows: with the interaction picture the
number of steps does not grow with the spatial resolution."""
import numpy as np
import pytest

import oracle
from paper_1204_4255_amd import workloads as W


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def _prob(g, **kw):
    return oracle.Problem(n=g.n, lo=g.lo, hi=g.hi, h=1e-3, batch=g.batch, alpha=g.alpha, gamma=g.gamma, gnl=g.gnl,
                          trap=g.trap, **kw)


def test_cash_karp_pair_satisfies_its_order_conditions():
    # Butcher's order conditions up to order 5 for the propagated weights b, up to 4 for
    # the embedded b*, with b* failing the first fifth-order one (else the estimate is 0)
    c, A, b, bs = oracle.ck_tableau()
    a = np.zeros((6, 6))
    a[:, :5] = A
    assert np.allclose(a.sum(axis=1), c, atol=1e-15)
    ac = a @ c
    ac2 = a @ c ** 2
    ac3 = a @ c ** 3
    aac = a @ ac
    conds4 = [(lambda w: w.sum(), 1), (lambda w: w @ c, 1 / 2), (lambda w: w @ c ** 2, 1 / 3),
              (lambda w: w @ ac, 1 / 6), (lambda w: w @ c ** 3, 1 / 4), (lambda w: w @ (c * ac), 1 / 8),
              (lambda w: w @ ac2, 1 / 12), (lambda w: w @ aac, 1 / 24)]
    conds5 = [(lambda w: w @ c ** 4, 1 / 5), (lambda w: w @ (c ** 2 * ac), 1 / 10), (lambda w: w @ (c * ac2), 1 / 15),
              (lambda w: w @ (c * aac), 1 / 30), (lambda w: w @ ac ** 2, 1 / 20), (lambda w: w @ ac3, 1 / 20),
              (lambda w: w @ (a @ (c * ac)), 1 / 40), (lambda w: w @ (a @ ac2), 1 / 60),
              (lambda w: w @ (a @ aac), 1 / 120)]
    for f, v in conds4 + conds5:
        assert abs(f(b) - v) < 1e-14
    for f, v in conds4:
        assert abs(f(bs) - v) < 1e-14
    assert abs(conds5[0][0](bs) - 1 / 5) > 1e-4


def test_ck_step_local_orders_on_a_plane_wave():
    # G = -i c psi (constant potential) on a plane wave: the exact step is
    # e^{(L(k) - i c) h} psi. The fifth-order result's local error falls as h^6, the
    # embedded difference (the estimate) as h^5.
    n, L, cv, gam, m = 32, 10.0, 1.7, 0.2, 5
    g = W.Group(n=(n,), lo=(-L / 2,), hi=(L / 2,), gamma=gam)
    x = g.axis(0)
    k = 2 * np.pi * m / L
    p = _prob(g, Vgrid=np.full((1, n), cv))
    psi = np.exp(1j * k * x)[None]
    errs, ests = [], []
    for h in (0.2, 0.1, 0.05):
        out, est = oracle.ck_step(p, psi, h)
        exact = np.exp((-0.5j * k * k - gam - 1j * cv) * h) * psi
        errs.append(rel(out, exact))
        ests.append(est[0])
    for i in range(2):
        assert 5.6 < np.log2(errs[i] / errs[i + 1]) < 6.4, errs
        assert 4.6 < np.log2(ests[i] / ests[i + 1]) < 5.4, ests


def test_free_gaussian_is_exact_and_the_step_grows_by_five():
    # with G = 0 every stage vanishes: the estimate is 0, each step is e^{L h} exactly,
    # and the controller grows the step by its maximum factor until the end cuts it
    n, L, s0, x0, k0 = 256, 40.0, 1.3, 0.5, 1.0
    g = W.Group(n=(n,), lo=(-L / 2,), hi=(L / 2,))
    x = g.axis(0)

    def free(t):
        cc = 1 + 1j * t / s0 ** 2
        return ((np.pi * s0 ** 2) ** -0.25 * cc ** -0.5
                * np.exp(-(x - x0 - k0 * t) ** 2 / (2 * s0 ** 2 * cc) + 1j * k0 * x - 0.5j * k0 ** 2 * t))

    T, h0 = 1.7, 0.01
    out, hn, st, log, done = oracle.ark45(_prob(g), free(0.0)[None], T, 1e-9, h0, log_cap=16)
    assert done and st[0, 1] == 0
    assert rel(out[0], free(T)) < 1e-12
    steps = log[0, :st[0, 0]]
    assert np.allclose(steps[:-1], h0 * 5.0 ** np.arange(len(steps) - 1), rtol=1e-15)
    assert abs(steps.sum() - T) < 1e-15 * T


def _soliton(n, T, tol, h0=1e-3, log_cap=0):
    g = W.Group(n=(n,), lo=(-20.0,), hi=(20.0,), gnl=-1.0)
    x = g.axis(0)
    psi0 = (1 / np.cosh(x) * np.exp(0.5j * x))[None]
    exact = 1 / np.cosh(x - 0.5 * T) * np.exp(1j * (0.5 * x + 0.375 * T))
    out, hn, st, log, done = oracle.ark45(_prob(g), psi0, T, tol, h0, log_cap=log_cap)
    assert done
    return rel(out[0], exact), st[0], log


def test_soliton_error_follows_the_tolerance():
    # the exact soliton sech(x - v t) e^{i(v x + (1 - v^2) t / 2)}, v = 1/2
    errs, counts = [], []
    for tol in (1e-5, 1e-7, 1e-9):
        e, st, _ = _soliton(256, 2.0, tol)
        errs.append(e)
        counts.append(st[0])
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-8
    # a local tolerance 100x tighter costs about 100^(1/5) = 2.5x the steps
    assert all(1.8 < counts[i + 1] / counts[i] < 3.2 for i in range(2)), counts


def test_step_count_does_not_grow_with_resolution():
    # the interaction picture solves the kinetic term exactly, so the step is set by G
    # alone: the same steps at every resolution (the paper's step-count figure)
    counts = [_soliton(n, 2.0, 1e-8, log_cap=64)[1][0] for n in (128, 256, 512, 1024)]
    assert max(counts) - min(counts) <= 1, counts


def test_rejected_steps_and_the_accepted_ones_meet_the_tolerance():
    # a first trial step far too large is rejected until it fits; replaying the accepted
    # steps one by one gives the same field, and each one's estimate is within tol
    tol, T = 1e-7, 1.0
    g = W.Group(n=(128,), lo=(-20.0,), hi=(20.0,), gnl=-1.0)
    x = g.axis(0)
    psi0 = (1 / np.cosh(x) * np.exp(0.5j * x))[None]
    p = _prob(g)
    out, hn, st, log, done = oracle.ark45(p, psi0, T, tol, 0.8, log_cap=256)
    assert done and st[0, 1] >= 1
    f = psi0.astype(complex)
    for h in log[0, :st[0, 0]]:
        f, est = oracle.ck_step(p, f, h)
        assert est[0] <= tol
    assert rel(f, out) < 1e-14
    assert np.all(log[0, 1:st[0, 0] - 1] / log[0, :st[0, 0] - 2] <= 5.0 + 1e-12)


def test_instances_adapt_independently():
    # a batch of solitons of different amplitudes: every instance equals its own run
    g = W.Group(n=(128,), lo=(-20.0,), hi=(20.0,), gnl=-1.0, batch=3)
    x = g.axis(0)
    amps = np.array([0.5, 1.0, 2.0])
    psi0 = amps[:, None] / np.cosh(amps[:, None] * x[None]) + 0j
    out, hn, st, log, done = oracle.ark45(_prob(g), psi0, 1.0, 1e-7, 1e-3)
    assert done and len(set(st[:, 0])) == 3
    for b in range(3):
        gb = W.Group(n=(128,), lo=(-20.0,), hi=(20.0,), gnl=-1.0)
        ob, hb, sb, _, _ = oracle.ark45(_prob(gb), psi0[b:b + 1], 1.0, 1e-7, 1e-3)
        assert np.array_equal(ob[0], out[b]) and np.array_equal(sb[0], st[b]) and hb[0] == hn[b]


def test_noise_is_rejected():
    g = W.Group(n=(16,), lo=(0.0,), hi=(1.0,))
    with pytest.raises(ValueError):
        oracle.ark45(_prob(g, sigma=0.1), np.ones((1, 16), complex), 1.0, 1e-6, 0.1)


def test_explicit_method_steps_grow_with_resolution():
    # the comparison of Sec. 3.6 (the step-count figure): with the kinetic term in the
    # stages the stable step falls as 1/k_max^2, so doubling the points costs about 4x the
    # steps; the interaction picture keeps the count
    ip_counts, ex_counts = [], []
    for n in (128, 256, 512):
        g = W.Group(n=(n,), lo=(-20.0,), hi=(20.0,), gnl=-1.0)
        x = g.axis(0)
        psi0 = (1 / np.cosh(x) * np.exp(0.5j * x))[None]
        for ip, counts in ((True, ip_counts), (False, ex_counts)):
            _, _, st, _, done = oracle.ark45(_prob(g), psi0, 1.0, 1e-7, 1e-3, ip=ip)
            assert done
            counts.append(int(st[0, 0]))
    assert max(ip_counts) - min(ip_counts) <= 1, ip_counts
    assert ex_counts[2] / ex_counts[1] > 3 and ex_counts[1] / ex_counts[0] > 3, ex_counts


def test_explicit_method_on_the_free_gaussian():
    # with G = 0 the explicit method integrates L psi alone: the closed form to the tolerance
    n, L, s0, x0, k0 = 128, 40.0, 1.3, 0.5, 1.0
    g = W.Group(n=(n,), lo=(-L / 2,), hi=(L / 2,))
    x = g.axis(0)

    def free(t):
        cc = 1 + 1j * t / s0 ** 2
        return ((np.pi * s0 ** 2) ** -0.25 * cc ** -0.5
                * np.exp(-(x - x0 - k0 * t) ** 2 / (2 * s0 ** 2 * cc) + 1j * k0 * x - 0.5j * k0 ** 2 * t))

    out, _, st, _, done = oracle.ark45(_prob(g), free(0.0)[None], 1.0, 1e-9, 1e-3, ip=False)
    assert done and st[0, 0] > 10  # not exact in one step, unlike the interaction picture
    assert rel(out[0], free(1.0)) < 1e-6
