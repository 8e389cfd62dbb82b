"""GPU parity of the adaptive Cash-Karp RK4(5) in the interaction picture (rk4ip_ark45:
Sec. 3.5's adaptive fourth-fifth order Runge-Kutta on eq. (6) of Sec. 3.6) against the
FP64 oracle.

Accepting a step is a floating-point decision that the GPU takes on its own complex64
estimate, so near the tolerance the two sides may choose different steps; both runs are
then correct. The tests therefore compare what is unique and check that the rest is
valid: the oracle replays the GPU's logged accepted steps and must reach the same field
(element by element), every accepted step must meet the tolerance by the oracle's FP64
estimate, every step change must follow the controller from that estimate, and the step
counts must match the oracle's own adaptive run."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, quantised, rel
from paper_1204_4255_amd import rk4ip
from paper_1204_4255_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    rk4ip.load()
    return t


def _oprob(g, convK=None):
    return oracle.Problem(n=g.n, lo=g.lo, hi=g.hi, h=1e-3, batch=1, alpha=g.alpha, gamma=g.gamma, gnl=g.gnl,
                          trap=g.trap, convK=convK)


def _plan(gs, torch):
    probs = [rk4ip.make_problem(g.n, g.lo, g.hi, 1e-3, batch=g.batch, alpha=g.alpha, gamma=g.gamma, g_nl=g.gnl,
                                trap=g.trap) for g in gs]
    return rk4ip.Plan(probs)


def _dev(torch, a):
    return torch.tensor(np.asarray(a, dtype=np.complex64).reshape(-1), device="cuda")


def _factor(err, tol):
    if not np.isfinite(err):
        return 0.2
    if err == 0.0:
        return 5.0
    return min(5.0, max(0.2, 0.9 * (tol / err) ** 0.2))


def _replay_check(g, f0, steps, tol, h_first, span, rejected, slack=0.1, convK=None, ip=True):
    """Replay the accepted steps of one instance on the oracle; check each one meets tol
    by the oracle's estimate and that the step changes follow the controller. Returns the
    replayed field."""
    p = _oprob(g, convK)
    f = np.asarray(f0, complex)[None]
    errs = []
    for h in steps:
        f, e = oracle.ck_step(p, f, h, ip=ip)
        errs.append(e[0])
    errs = np.array(errs)
    assert np.all(errs <= tol * (1 + slack)), (errs.max(), tol)
    # the next trial after an accepted step is h f(err); a rejection only shrinks it, and
    # the last step may have been cut to the end of the interval
    bound = steps[:-1] * np.array([_factor(e, tol) for e in errs[:-1]])
    assert np.all(steps[1:-1] <= bound[:-1] * (1 + 5 * slack)), "a step grew faster than the controller allows"
    if rejected == 0 and len(steps) > 2:
        # without rejections each step is h f(err); where err is far below tol it sits near
        # the complex64 rounding floor of the GPU's own estimate, so only steps whose FP64
        # estimate is at least tol/10 are held to it
        firm = errs[:-2] >= 0.1 * tol
        assert np.allclose(steps[1:-1][firm], bound[:-1][firm], rtol=slack), "a step differs from h f(err)"
    # the first trial is the given step, cut to the interval when it would pass its end
    assert rejected > 0 or steps[0] == (h_first if h_first < span else span)
    return f[0]


def _solitons(n, amps, L=20.0):
    g = W.Group(n=(n,), lo=(-L,), hi=(L,), gnl=-1.0, batch=len(amps))
    x = g.axis(0)
    a = np.asarray(amps, float)[:, None]
    f0 = a / np.cosh(a * x[None]) * np.exp(0.5j * x[None])
    return g, quantised(f0)


@pytest.mark.parametrize("n,amps", [(64, [1.0]), (256, [0.5, 1.0, 1.5, 2.0, 1.2]), (1024, [1.0, 2.0]),
                                    (4096, [1.0])])
def test_ark45_replay_matches_oracle(torch, n, amps):
    tol, T, h0 = 1e-6, 1.0, 1e-3
    log(f"ark45 solitons n={n} amps={amps}")
    g, f0 = _solitons(n, amps)
    plan = _plan([g], torch)
    d = _dev(torch, f0)
    h = torch.full((g.batch,), h0, dtype=torch.float64, device="cuda")
    stats, hl = plan.ark45(d, T, tol, h, log_cap=400)
    torch.cuda.synchronize()
    stats = stats.cpu().numpy()
    hl = hl.cpu().numpy()
    out = d.cpu().numpy().astype(np.complex128).reshape(g.shape)
    assert np.all(stats[:, 2] == 1)
    for b in range(g.batch):
        acc, rej = int(stats[b, 0]), int(stats[b, 1])
        steps = hl[b, :acc]
        assert abs(steps.sum() - T) < 1e-12
        ref = _replay_check(g, f0[b], steps, tol, h0, T, rej)
        err = rel(out[b], ref)
        # the oracle's own adaptive run takes about the same steps
        gb = W.Group(n=(n,), lo=g.lo, hi=g.hi, gnl=g.gnl)
        _, _, ost, _, _ = oracle.ark45(_oprob(gb), f0[b:b + 1], T, tol, h0)
        log(f"  amp {amps[b]}: {acc} accepted, {rej} rejected (oracle {ost[0, 0]}, {ost[0, 1]}); replay rel {err:.2e}")
        assert err < 1e-5
        assert abs(acc - ost[0, 0]) <= 2


def test_ark45_free_evolution_is_exact(torch):
    n, L, s0, x0, k0 = 256, 40.0, 1.3, 0.5, 1.0
    g = W.Group(n=(n,), lo=(-L / 2,), hi=(L / 2,), gamma=0.05)
    x = g.axis(0)

    def free(t):
        c = 1 + 1j * t / s0 ** 2
        return (np.exp(-0.05 * t) * (np.pi * s0 ** 2) ** -0.25 * c ** -0.5
                * np.exp(-(x - x0 - k0 * t) ** 2 / (2 * s0 ** 2 * c) + 1j * k0 * x - 0.5j * k0 ** 2 * t))

    T, h0 = 1.7, 0.01
    plan = _plan([g], torch)
    d = _dev(torch, free(0.0))
    h = torch.full((1,), h0, dtype=torch.float64, device="cuda")
    stats, hl = plan.ark45(d, T, 1e-9, h, log_cap=16)
    stats = stats.cpu().numpy()[0]
    steps = hl.cpu().numpy()[0, :stats[0]]
    assert stats[1] == 0 and stats[2] == 1
    assert np.array_equal(steps[:-1], h0 * 5.0 ** np.arange(len(steps) - 1))
    assert rel(d.cpu().numpy().astype(np.complex128), free(T)) < 2e-6


def test_ark45_step_count_independent_of_resolution(torch):
    counts = []
    for n in (256, 512, 1024, 2048):
        g, f0 = _solitons(n, [1.0])
        plan = _plan([g], torch)
        d = _dev(torch, f0)
        h = torch.full((1,), 1e-3, dtype=torch.float64, device="cuda")
        stats, _ = plan.ark45(d, 2.0, 1e-7, h)
        counts.append(int(stats[0, 0]))
    log(f"  accepted steps at n = 256..2048: {counts}")
    assert max(counts) - min(counts) <= 1


def test_ark45_trap_period_in_samples(torch):
    """The 1D trapped GPE over one trap period in 50 intervals (the shape of the paper's
    first example), continuing each interval from the step the last one proposed; each
    interval is replayed on the oracle from the GPU's state at its start. The domain keeps
    h max V inside the pair's stability interval on the imaginary axis (|R(i y)| exceeds 1
    by 2% at y = 2 and 9% at y = 2.6): the potential is not in the interaction picture, and
    edge modes outside that interval would amplify each side's own rounding."""
    g = W.Group(n=(128,), lo=(-8.0,), hi=(8.0,), gnl=1.0, trap=(1.0, 0, 0), batch=3)
    x = g.axis(0)
    shifts = np.array([0.0, 0.5, 1.0])
    f0 = quantised(np.pi ** -0.25 * np.exp(-(x[None] - shifts[:, None]) ** 2 / 2))
    plan = _plan([g], torch)
    d = _dev(torch, f0)
    h = torch.full((3,), 1e-2, dtype=torch.float64, device="cuda")
    tol, span = 1e-6, 2 * np.pi / 50
    worst, total = 0.0, 0
    for s in range(50):
        start = d.cpu().numpy().astype(np.complex128).reshape(g.shape)
        h_in = h.cpu().numpy().copy()
        stats, hl = plan.ark45(d, span, tol, h, log_cap=64)
        stats = stats.cpu().numpy()
        hl = hl.cpu().numpy()
        out = d.cpu().numpy().astype(np.complex128).reshape(g.shape)
        assert np.all(stats[:, 2] == 1)
        for b in range(3):
            steps = hl[b, :stats[b, 0]]
            ref = _replay_check(g, start[b], steps, tol, h_in[b], span, int(stats[b, 1]))
            worst = max(worst, rel(out[b], ref))
            total += int(stats[b, 0])
    log(f"  50 intervals: {total} accepted steps over 3 instances, worst interval replay rel {worst:.2e}")
    assert worst < 2e-6


def test_ark45_with_the_non_local_potential(torch):
    """Solitons with a softened Coulomb non-local potential (the non-local example of Sec. 4
    integrated adaptively, as the paper's 1D examples are): replayed on the oracle."""
    tol, T, h0 = 1e-6, 1.0, 1e-3
    n, L = 256, 40.0
    g, f0 = _solitons(n, [0.8, 1.0, 1.3])
    d_ = np.arange(n)
    d_ = np.where(d_ < n // 2, d_, d_ - n) * (L / n)
    K = 0.2 / np.sqrt(d_ ** 2 + 1.0)
    p = rk4ip.make_problem(g.n, g.lo, g.hi, 1e-3, batch=g.batch, alpha=g.alpha, g_nl=g.gnl, conv_K=K)
    plan = rk4ip.Plan([p])
    d = _dev(torch, f0)
    h = torch.full((g.batch,), h0, dtype=torch.float64, device="cuda")
    stats, hl = plan.ark45(d, T, tol, h, log_cap=400)
    stats = stats.cpu().numpy()
    hl = hl.cpu().numpy()
    out = d.cpu().numpy().astype(np.complex128).reshape(g.shape)
    assert np.all(stats[:, 2] == 1)
    for b in range(g.batch):
        acc, rej = int(stats[b, 0]), int(stats[b, 1])
        ref = _replay_check(g, f0[b], hl[b, :acc], tol, h0, T, rej, convK=K)
        gb = W.Group(n=(n,), lo=g.lo, hi=g.hi, gnl=g.gnl)
        _, _, ost, _, _ = oracle.ark45(_oprob(gb, K), f0[b:b + 1], T, tol, h0)
        err = rel(out[b], ref)
        log(f"  non-local, instance {b}: {acc} accepted, {rej} rejected (oracle {ost[0, 0]}, {ost[0, 1]}); "
            f"replay rel {err:.2e}")
        assert err < 1e-5
        assert abs(acc - ost[0, 0]) <= 2


@pytest.mark.parametrize("n", [128, 256])
def test_ark45_explicit_method_replay(torch, n):
    """The explicit comparison method (the linear part in the stages): replayed on the
    oracle's explicit steps, with the oracle's own step counts. The controller keeps this
    method at its stability limit, where the pair amplifies the highest modes a little
    each step; the soliton has no content there, but the complex64 run carries its
    rounding floor in them, which the FP64 run does not. So the fields are compared on
    the modes below half the Nyquist wavenumber (1e-5, the bar of every other replay), and
    the rounding-driven remainder in the highest modes is reported."""
    tol, T, h0 = 1e-6, 1.0, 1e-3
    g, f0 = _solitons(n, [0.8, 1.0])
    plan = _plan([g], torch)
    d = _dev(torch, f0)
    h = torch.full((g.batch,), h0, dtype=torch.float64, device="cuda")
    stats, hl = plan.ark45(d, T, tol, h, log_cap=2048, explicit=True)
    stats = stats.cpu().numpy()
    hl = hl.cpu().numpy()
    out = d.cpu().numpy().astype(np.complex128).reshape(g.shape)
    assert np.all(stats[:, 2] == 1)
    for b in range(g.batch):
        acc, rej = int(stats[b, 0]), int(stats[b, 1])
        ref = _replay_check(g, f0[b], hl[b, :acc], tol, h0, T, rej, ip=False)
        gb = W.Group(n=(n,), lo=g.lo, hi=g.hi, gnl=g.gnl)
        _, _, ost, _, _ = oracle.ark45(_oprob(gb), f0[b:b + 1], T, tol, h0, ip=False)
        err = rel(out[b], ref)
        k = np.fft.fftfreq(n) * n
        low = np.abs(k) < n // 4

        def lowpass(f):
            return np.fft.ifft(np.where(low, np.fft.fft(f), 0))

        err_low = rel(lowpass(out[b]), lowpass(ref))
        log(f"  explicit n={n}, instance {b}: {acc} accepted, {rej} rejected (oracle {ost[0, 0]}, {ost[0, 1]}); "
            f"replay rel {err:.2e}, below half the Nyquist wavenumber {err_low:.2e}")
        assert err_low < 1e-5
        assert abs(acc - ost[0, 0]) <= max(2, 0.02 * ost[0, 0])


def test_ark45_explicit_steps_grow_with_resolution(torch):
    """The paper's step-count comparison on the GPU: the explicit method's accepted steps
    grow about fourfold per doubling of the points, the interaction picture's do not."""
    ip, ex = [], []
    for n in (128, 256, 512):
        g, f0 = _solitons(n, [1.0])
        plan = _plan([g], torch)
        for explicit, counts in ((False, ip), (True, ex)):
            d = _dev(torch, f0)
            h = torch.full((1,), 1e-3, dtype=torch.float64, device="cuda")
            stats, _ = plan.ark45(d, 1.0, 1e-7, h, explicit=explicit)
            assert int(stats[0, 2]) == 1
            counts.append(int(stats[0, 0]))
    log(f"  accepted steps at n = 128, 256, 512: interaction picture {ip}, explicit {ex}")
    assert max(ip) - min(ip) <= 1
    assert ex[2] / ex[1] > 3 and ex[1] / ex[0] > 3


def test_ark45_stops_after_max_attempts(torch):
    g, f0 = _solitons(128, [1.0, 2.0])
    plan = _plan([g], torch)
    d = _dev(torch, f0)
    h = torch.full((2,), 1e-5, dtype=torch.float64, device="cuda")
    stats, hl = plan.ark45(d, 1.0, 1e-6, h, max_attempts=3, log_cap=8)
    stats = stats.cpu().numpy()
    assert np.all(stats[:, 2] == 0) and np.all(stats[:, 0] + stats[:, 1] == 3)
    hl = hl.cpu().numpy()
    out = d.cpu().numpy().astype(np.complex128).reshape(g.shape)
    for b in range(2):
        f = f0[b:b + 1]
        for hh in hl[b, :stats[b, 0]]:
            f, _ = oracle.ck_step(_oprob(W.Group(n=(128,), lo=g.lo, hi=g.hi, gnl=g.gnl)), f, hh)
        assert rel(out[b], f[0]) < 1e-6


def test_ark45_rejects_what_it_does_not_cover(torch):
    g2 = W.Group(n=(16, 16), lo=(-1, -1), hi=(1, 1))
    plan = rk4ip.Plan([rk4ip.make_problem(g2.n, g2.lo, g2.hi, 1e-3)])
    d = torch.zeros(256, dtype=torch.complex64, device="cuda")
    h = torch.full((1,), 1e-3, dtype=torch.float64, device="cuda")
    with pytest.raises(rk4ip.Rk4ipError) as e:
        plan.ark45(d, 1.0, 1e-6, h)
    assert e.value.status == rk4ip.RK4IP_ERR_UNSUPPORTED_SHAPE
    noisy = rk4ip.Plan([rk4ip.make_problem((64,), (-1,), (1,), 1e-3, sigma=0.1)])
    d1 = torch.zeros(64, dtype=torch.complex64, device="cuda")
    for kw in (dict(), dict(tol=0.0)):
        with pytest.raises(rk4ip.Rk4ipError) as e:
            (noisy if not kw else _plan([W.Group(n=(64,), lo=(-1,), hi=(1,))], torch)).ark45(
                d1, 1.0, kw.get("tol", 1e-6), h)
        assert e.value.status == rk4ip.RK4IP_ERR_INVALID_ARG
