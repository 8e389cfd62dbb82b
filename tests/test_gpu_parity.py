"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same seeded
inputs. Bar: Philox integers bit-exact; fields within relative L2 1e-5 over whole runs
(the target of the workloads), 1e-6 for single operations."""
import os

import numpy as np
import pytest

import oracle
from gpu_helpers import assert_same_runs, log, oprob, plan_for, quantised, random_field, rel, rel_per_instance
from paper_1204_4255_amd import rk4ip
from paper_1204_4255_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


# ----------------------------------------------------------------------------- noise


def test_philox_bit_exact(torch):
    log("philox: known answers + 65536 random counters")
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(t, 16) for t in line.split()])
    for r in rows:
        ctr = torch.tensor(np.array(r[0:4], dtype=np.uint32).view(np.int32), device="cuda")
        out = torch.empty(4, dtype=torch.int32, device="cuda")
        seed = r[4] | (r[5] << 32)
        rk4ip.rk4ip_debug_philox(seed, ctr, out)
        assert out.cpu().numpy().view(np.uint32).tolist() == r[6:10]
    rng = np.random.Generator(np.random.PCG64(1))
    ctr = rng.integers(0, 2 ** 32, size=(65536, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0xDEADBEEF12345678
    d_ctr = torch.tensor(ctr.view(np.int32), device="cuda")
    d_out = torch.empty_like(d_ctr)
    rk4ip.rk4ip_debug_philox(seed, d_ctr, d_out)
    got = d_out.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle.philox_batch(ctr, seed))


@pytest.mark.parametrize("step", [0, 7, (1 << 33) + 5])
def test_noise_field_matches_oracle(torch, step):
    log(f"noise field step {step}")
    g = W.Group(n=(64, 32), lo=(-4, -2), hi=(4, 2), batch=3, sigma=1.0, seed=0x1234_5678_9ABC, id_base=11)
    plan = plan_for(W.Workload("n", [g], 1e-3, 1, [np.zeros(g.shape)]))
    xi = _host(plan.noise(0, step), g.shape)
    ref = oracle.noise(oprob(g, 1e-3), step)
    # same Philox words on both sides; Box-Muller in FP32 vs FP64
    assert np.max(np.abs(xi - ref)) <= 2e-6 * np.max(np.abs(ref))


# ----------------------------------------------------------------------------- FFT engine


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft_engine(torch, n, sign):
    log(f"fft n={n} sign={sign}")
    g = W.Group(n=(n,), lo=(0.0,), hi=(1.0,), batch=1)
    plan = plan_for(W.Workload("f", [g], 1e-3, 1, [np.zeros(g.shape)]))
    nlines = 37
    rng = np.random.Generator(np.random.PCG64(n))
    x = quantised(rng.standard_normal((nlines, n)) + 1j * rng.standard_normal((nlines, n)))
    y = _host(plan.fft(0, 0, _dev(torch, x), sign), (nlines, n))
    ref = np.stack([oracle.fft(x[i], sign) for i in range(nlines)])
    assert rel(y, ref) < 3e-7 * max(1.0, np.log2(n) / 4)


# ----------------------------------------------------------------------------- propagator


@pytest.mark.parametrize("n,batch", [((8,), 3), ((1024,), 5), ((64, 8), 2), ((16, 128), 1), ((512, 32), 1),
                                     ((8, 16, 32), 2), ((64, 64, 64), 1), ((1024, 8, 8), 1)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_apply_D(torch, n, batch, adjoint):
    log(f"apply_D n={n} batch={batch} adjoint={adjoint}")
    nd = len(n)
    g = W.Group(n=n, lo=(-3.0,) * nd, hi=(4.0,) * nd, batch=batch, gamma=0.3, alpha=0.7)
    f = quantised(random_field(g, 5))
    w = W.Workload("d", [g], 0.05, 1, [f])
    plan = plan_for(w)
    d = _dev(torch, f)
    plan.apply_D(d, adjoint)
    ref = oracle.apply_D(oprob(g, 0.05), f, adjoint=adjoint)
    assert rel(_host(d, g.shape), ref) < 1e-6


# ----------------------------------------------------------------------------- one step


STEP_CASES = [
    ((8,), 3), ((16,), 130), ((64,), 5), ((256,), 9), ((1024,), 3), ((2048,), 2), ((4096,), 1),
    ((8, 8), 2), ((64, 32), 3), ((32, 128), 1), ((512, 16), 1), ((16, 1024), 1),
    ((8, 8, 8), 3), ((32, 16, 8), 2), ((16, 32, 64), 1), ((128, 8, 16), 1),
]


@pytest.mark.parametrize("n,batch", STEP_CASES)
def test_one_step_matches_oracle(torch, n, batch):
    log(f"one step n={n} batch={batch}")
    nd = len(n)
    g = W.Group(n=n, lo=(-5.0,) * nd, hi=(5.0,) * nd, batch=batch, gnl=2.5, trap=(1.0, 1.3, 0.7), gamma=0.05,
                sigma=0.02, seed=77, id_base=3)
    rng = np.random.Generator(np.random.PCG64(9))
    g.Vgrid = (0.1 * rng.standard_normal((batch, g.M))).astype(np.float32)
    f = quantised(random_field(g, 3))
    w = W.Workload("s", [g], 2e-3, 1, [f])
    plan = plan_for(w)
    d = _dev(torch, f)
    plan.step(d, 41)
    torch.cuda.synchronize()
    ref = oracle.step(oprob(g, 2e-3), f, 41)
    err = rel_per_instance(_host(d, g.shape), ref, batch)
    assert np.max(err) < 1e-6, err


def test_uneven_groups_in_one_plan(torch):
    log("uneven groups: 3x16x16 + 2x32x32 + 4x64 (1D)")
    rng = np.random.Generator(np.random.PCG64(2))
    gs = []
    base = 0
    for n, b in (((16, 16), 3), ((32, 32), 2)):
        g = W.Group(n=n, lo=(-6.0, -6.0), hi=(6.0, 6.0), batch=b, gnl=10.0, trap=(1, 1, 0), sigma=0.01, seed=5,
                    id_base=base)
        g.Vgrid = (0.01 * rng.standard_normal((b, g.M))).astype(np.float32)
        gs.append(g)
        base += b
    g1 = W.Group(n=(64,), lo=(-8.0,), hi=(8.0,), batch=4, gnl=1.0, trap=(1, 0, 0), seed=5, id_base=base, sigma=0.01)
    gs.append(g1)
    fields = [quantised(random_field(g, i)) for i, g in enumerate(gs)]
    w = W.Workload("u", gs, 1e-3, 5, fields)
    plan = plan_for(w)
    d = rk4ip.field_to_device(w)
    plan.run(d, 5, step0=2)
    got = d.cpu().numpy().astype(np.complex128)
    off = 0
    for g, f in zip(gs, fields):
        ref, _, _ = oracle.run(oprob(g, 1e-3), f, 5, step0=2)
        part = got[off:off + g.batch * g.M].reshape(g.shape)
        off += g.batch * g.M
        assert np.max(rel_per_instance(part, ref, g.batch)) < 1e-5


# ----------------------------------------------------------------------------- diagnostics


@pytest.mark.parametrize("n,batch", [((256,), 3), ((64, 32), 2), ((32, 16, 8), 2), ((1024,), 1)])
def test_diagnostics_match_oracle(torch, n, batch):
    log(f"diagnostics n={n}")
    nd = len(n)
    g = W.Group(n=n, lo=(-5.0,) * nd, hi=(5.0,) * nd, batch=batch, gnl=3.0, trap=(1.0, 2.0, 0.5))
    rng = np.random.Generator(np.random.PCG64(4))
    g.Vgrid = (0.2 * rng.standard_normal((batch, g.M))).astype(np.float32)
    f = quantised(random_field(g, 8))
    plan = plan_for(W.Workload("g", [g], 1e-3, 1, [f]))
    out = plan.diagnostics(_dev(torch, f)).cpu().numpy()
    ref = oracle.diag(oprob(g, 1e-3), f)
    assert np.allclose(out, ref, rtol=2e-6, atol=1e-9 * np.abs(ref).max())
    # bit-reproducible
    out2 = plan.diagnostics(_dev(torch, f)).cpu().numpy()
    assert np.array_equal(out, out2)


def test_overlap_and_moments(torch):
    log("overlap and moments")
    g = W.Group(n=(32, 16), lo=(-4, -4), hi=(4, 4), batch=6)
    f = quantised(random_field(g, 12))
    phi = quantised(random_field(W.Group(n=(32, 16), lo=(-4, -4), hi=(4, 4)), 13)[0])
    plan = plan_for(W.Workload("o", [g], 1e-3, 1, [f]))
    c = plan.overlap(0, _dev(torch, phi), _dev(torch, f)).cpu().numpy()
    ref = oracle.overlap(oprob(g, 1e-3), phi, f)
    assert np.allclose(c[:, 0] + 1j * c[:, 1], ref, rtol=1e-12, atol=1e-12)
    mean, var = plan.moments(0, _dev(torch, f))
    rm, rv = oracle.moments(oprob(g, 1e-3), f)
    assert np.allclose(mean.cpu().numpy(), rm.reshape(-1), rtol=1e-12)
    assert np.allclose(var.cpu().numpy(), rv.reshape(-1), rtol=1e-10, atol=1e-14)


def test_nonfinite_is_reported(torch):
    log("non-finite detection")
    g = W.Group(n=(16, 16), lo=(-4, -4), hi=(4, 4), batch=2)
    f = quantised(random_field(g, 1))
    f[1, 3, 4] = np.nan
    plan = plan_for(W.Workload("x", [g], 1e-3, 1, [f]))
    assert plan.status() == rk4ip.RK4IP_OK
    plan.diagnostics(_dev(torch, f))
    assert plan.status() == rk4ip.RK4IP_ERR_NONFINITE
    assert plan.status() == rk4ip.RK4IP_OK


# ----------------------------------------------------------------------------- runs and determinism


def test_run_samples_and_checkpoints(torch):
    log("run with samples and checkpoints")
    g = W.Group(n=(32, 32), lo=(-6, -6), hi=(6, 6), batch=2, gnl=20.0, trap=(1, 1, 0), sigma=0.005, seed=3)
    f = quantised(random_field(g, 21))
    w = W.Workload("r", [g], 1e-3, 10, [f])
    plan = plan_for(w)
    d = _dev(torch, f)
    diag, ck = plan.run(d, 10, step0=4, sample_every=4, ckpt_every=3)
    ref, rdiag, rck = oracle.run(oprob(g, 1e-3), f, 10, step0=4, sample_every=4, ckpt_every=3)
    # about 7e-7 of FP32 rounding per step on this rough random field
    assert rel(_host(d, g.shape), ref) < 1e-5
    assert np.allclose(diag.cpu().numpy(), rdiag, rtol=1e-5, atol=1e-9)
    assert ck.shape[0] == 4
    for c in range(4):
        assert rel(_host(ck[c], g.shape), rck[c]) < 1e-5


@pytest.mark.parametrize("flags", [0, rk4ip.RK4IP_FLAG_GRAPH, rk4ip.RK4IP_FLAG_FUSE_1D,
                                   rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_FUSE_1D])
def test_determinism_resume_and_graph(torch, flags):
    log(f"determinism flags={flags}")
    gs = [W.Group(n=(64, 16), lo=(-6, -6), hi=(6, 6), batch=2, gnl=5.0, trap=(1, 1, 0), sigma=0.01, seed=9),
          W.Group(n=(256,), lo=(-8,), hi=(8,), batch=5, gnl=1.0, trap=(1, 0, 0), sigma=0.01, seed=9, id_base=2)]
    fields = [quantised(random_field(g, 30 + i)) for i, g in enumerate(gs)]
    w = W.Workload("det", gs, 1e-3, 23, fields)
    base = plan_for(w, 0)
    a = rk4ip.field_to_device(w)
    base.run(a, 23, step0=100)
    plan = plan_for(w, flags)
    b = rk4ip.field_to_device(w)
    plan.run(b, 23, step0=100)
    c = rk4ip.field_to_device(w)
    plan.run(c, 11, step0=100)
    plan.run(c, 12, step0=111)
    torch.cuda.synchronize()
    assert_same_runs(torch, gs, a, b, c)


def test_graph_replays_match_eager_with_work_between(torch):
    log("graph replays interleaved with eager torch work")
    g = W.Group(n=(32, 16, 8), lo=(-4, -4, -4), hi=(4, 4, 4), batch=2, gnl=3.0, trap=(1, 1, 1), sigma=0.01, seed=4)
    f = quantised(random_field(g, 40))
    w = W.Workload("gr", [g], 1e-3, 33, [f])
    eager = plan_for(w, 0)
    graph = plan_for(w, rk4ip.RK4IP_FLAG_GRAPH)
    a = _dev(torch, f)
    b = _dev(torch, f)
    for rep in range(4):
        eager.run(a, 33, step0=33 * rep)
        graph.run(b, 33, step0=33 * rep)   # FIRST, one replay of the 32-step graph, LAST2
        junk = torch.randn(1 << 16, device="cuda").sum()  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(a, b), rep


def test_autotuned_schedules_match_oracle(torch):
    """Every schedule the autotuner may pick computes the same step: with 16 values per
    thread the per-line arithmetic is identical (bitwise equal to the default), with 8
    it differs only by rounding."""
    log("autotuned schedules vs default and oracle (3D 256x32x64, 2D 512x128)")
    for n in ((256, 32, 64), (512, 128)):
        nd = len(n)
        g = W.Group(n=n, lo=(-5.0,) * nd, hi=(5.0,) * nd, batch=1, gnl=10.0, trap=(1, 1, 1), sigma=0.01, seed=2)
        f = quantised(random_field(g, 50))
        w = W.Workload("t", [g], 1e-3, 3, [f])
        base = plan_for(w, 0)
        tuned = plan_for(w, rk4ip.RK4IP_FLAG_AUTOTUNE)
        names = [tuned.schedule(0, i) for i in range(tuned.num_passes(0))]
        log("  " + " ".join(names))
        a = _dev(torch, f)
        b = _dev(torch, f)
        base.run(a, 3)
        tuned.run(b, 3)
        torch.cuda.synchronize()
        ref, _, _ = oracle.run(oprob(g, 1e-3), f, 3)
        assert rel(_host(b, g.shape), ref) < 2e-6
        if all(nm.endswith(":r16") for nm in names):
            assert torch.equal(a, b)
        else:
            assert rel(_host(b, g.shape), _host(a, g.shape)) < 2e-6


# ----------------------------------------------------------------------------- the workloads


def test_nlse_soliton_full_run(torch):
    log("nlse1d n=256, 1000 steps")
    w = W.nlse1d()
    g = w.groups[0]
    f = quantised(w.psi0[0])
    plan = plan_for(w)
    d = _dev(torch, f)
    diag, _ = plan.run(d, w.nsteps, sample_every=w.sample_every)
    ref, rdiag, _ = oracle.run(oprob(g, w.h), f, w.nsteps, sample_every=w.sample_every)
    got = _host(d, g.shape)
    err = rel(got, ref)
    log(f"  rel L2 vs oracle at T: {err:.3e}")
    assert err < 1e-5
    x = g.axis(0)
    exact = 1 / np.cosh(x - 0.5) * np.exp(1j * (0.5 * x + 0.375))
    assert rel(got[0], exact) < 1e-5
    N = diag.cpu().numpy()[:, 0, 0]
    assert np.max(np.abs(N - 2.0)) < 2e-5
    assert np.allclose(diag.cpu().numpy(), rdiag, rtol=2e-5, atol=1e-7)


def test_gpe2d_512_parity(torch):
    nsteps = 200
    log(f"gpe2d 512^2, {nsteps} steps")
    w = W.gpe2d(nsteps=nsteps)
    g = w.groups[0]
    f = quantised(w.psi0[0])
    plan = plan_for(w)
    d = _dev(torch, f)
    plan.run(d, nsteps)
    ref, _, _ = oracle.run(oprob(g, w.h), f, nsteps)
    err = rel(_host(d, g.shape), ref)
    log(f"  rel L2 vs oracle: {err:.3e}")
    assert err < 1e-5


def test_sgpe1d_paths_and_moments(torch):
    P, nsteps = 64, 500
    log(f"sgpe1d {P} paths x 1024, {nsteps} steps")
    w = W.sgpe1d(paths=P, nsteps=nsteps)
    g = w.groups[0]
    f = quantised(w.psi0[0])
    plan = plan_for(w, rk4ip.RK4IP_FLAG_FUSE_1D)
    d = _dev(torch, f)
    plan.run(d, nsteps)
    ref, _, _ = oracle.run(oprob(g, w.h), f, nsteps)
    got = _host(d, g.shape)
    err = rel_per_instance(got, ref, P)
    log(f"  pathwise rel L2: max {err.max():.3e} median {np.median(err):.3e}")
    assert err.max() < 1e-5
    mean, var = plan.moments(0, d)
    # the reduction on the GPU's own fields against the FP64 definition: rounding only
    gm, gv = oracle.moments(oprob(g, w.h), got)
    assert np.allclose(mean.cpu().numpy(), gm.reshape(-1), rtol=1e-12)
    assert np.allclose(var.cpu().numpy(), gv.reshape(-1), rtol=1e-10, atol=1e-14)
    # against the oracle's own run: the mean to the fields' error; the variance is the
    # spread of paths that differ only through a weak noise (sigma = 1e-3), so the fields'
    # relative error of ~1e-6 is amplified by the mean over that spread
    rm, rv = oracle.moments(oprob(g, w.h), ref)
    assert rel(mean.cpu().numpy(), rm) < 1e-5
    assert rel(var.cpu().numpy(), rv) < 1e-3


def test_gpe3d_256_two_steps_full_size(torch):
    log("gpe3d 256^3, 2 steps, full field vs oracle")
    w = W.gpe3d(nsteps=2)
    g = w.groups[0]
    f = quantised(w.psi0[0])
    plan = plan_for(w)
    d = _dev(torch, f)
    plan.run(d, 2)
    got = _host(d, g.shape)
    ref, _, _ = oracle.run(oprob(g, w.h), f, 2)
    err = rel(got, ref)
    log(f"  rel L2 vs oracle after 2 steps: {err:.3e}")
    assert err < 1e-6


@pytest.mark.parametrize("n,batch", [((8,), 5), ((64,), 3), ((256,), 4), ((1024,), 3), ((2048,), 2), ((4096,), 1)])
def test_line_step_radix8_matches_oracle(torch, n, batch, tmp_path, monkeypatch):
    """The 1D whole-line kernel with 8 values per thread (picked through the tune cache)
    against the oracle: one step, and 12 steps fused per launch with noise on a rough
    random field (about 2e-7 of FP32 rounding per step), next to the 16-value kernel."""
    log(f"line step radix 8 n={n} batch={batch}")
    g = W.Group(n=n, lo=(-5.0,), hi=(5.0,), batch=batch, gnl=2.5, trap=(1.0, 0, 0), gamma=0.05, sigma=0.02,
                seed=77, id_base=3)
    f = quantised(random_field(g, 3))
    w = W.Workload("s", [g], 2e-3, 12, [f])
    ref1 = oracle.step(oprob(g, 2e-3), f, 41)
    ref12, _, _ = oracle.run(oprob(g, 2e-3), f, 12, step0=41)
    errs = {}
    for rr in (8, 16):
        cache = tmp_path / f"tune{rr}.json"
        cache.write_text('{ "gfx950|n=%d,1,1|b=%d|pass=0": [0, 0, %d] }\n' % (n[0], batch, rr))
        monkeypatch.setenv("RK4IP_TUNE_CACHE", str(cache))
        plan = plan_for(w, rk4ip.RK4IP_FLAG_AUTOTUNE | rk4ip.RK4IP_FLAG_FUSE_1D)
        assert plan.schedule(0, 0).endswith(f":r{rr}"), plan.schedule(0, 0)
        d = _dev(torch, f)
        plan.step(d, 41)
        e1 = np.max(rel_per_instance(_host(d, g.shape), ref1, batch))
        d = _dev(torch, f)
        plan.run(d, 12, step0=41)
        e12 = np.max(rel_per_instance(_host(d, g.shape), ref12, batch))
        errs[rr] = (e1, e12)
    log(f"  radix 8: {errs[8][0]:.2e} / {errs[8][1]:.2e}; radix 16: {errs[16][0]:.2e} / {errs[16][1]:.2e}")
    assert errs[8][0] < 1e-6 and errs[8][1] < 5e-6
    assert errs[8][1] < 2 * errs[16][1] + 1e-7
