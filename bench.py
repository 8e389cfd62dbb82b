#!/usr/bin/env python3
"""Benchmark of the RK4IP step on one MI355X: the 3D Gross-Pitaevskii workload on a
256^3 complex64 lattice (trap 1/2(x^2 + 1.5 y^2 + 2 z^2), g = 2000, dt = 2e-4).

Prints ONE JSON line: grid-point-steps/s over exactly --steps timed steps (after
--warmup untimed ones, inputs resident in HBM), the HBM roofline of the dominant kernel
(algorithmic bytes per launch / mean launch time measured with HIP events on the launch
stream), and the FP64 CPU oracle timed on a bounded sample on this host's cores.

    python bench.py [--gpus 1] [--steps 500] [--warmup 20] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "RK4IP grid-point-steps/s + % HBM roofline; batched/adjoint vs plain at 1e-5"
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per lattice point of each pass kind (complex64 = 8 B): FIRST
# reads psi and writes two fields; D2, LF and XF read and write two; LAST2 reads two and
# writes psi. A steady-state 3D step is D2, LF, D2, XF = 128 B per point (a run adds one
# FIRST and swaps its last XF for LAST2); a 1D line step reads and writes psi once.
PASS_BYTES = {"FIRST": 24, "D2": 32, "LF": 32, "XF": 32, "LAST2": 24, "line_step": 16,
              # the semi-implicit step works on psi in place: every pass reads and writes it once
              "D1": 16, "D1x2": 16, "SI": 16, "line_si": 16}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_gpe3d_256.json")
LINE_COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters_line_kernels.json")
TRAFFIC_FILE_SI = os.path.join(ROOT, "profiles", "traffic_gpe3d_256_semi_implicit.json")


def kernel_source_hash() -> str:
    from paper_1204_4255_amd.build import source_hash

    return source_hash()


def measured_counters(kernel: str, path: str = TRAFFIC_FILE):
    """Counter record of `kernel` from the committed rocprofv3 summary, or None when it is
    missing or the kernels changed since the counters were taken."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t.get("kernels", {}).get(kernel)


def measured_traffic(kernel: str, path: str = TRAFFIC_FILE):
    """HBM bytes per launch of `kernel` (scaled FETCH_SIZE + WRITE_SIZE), or None."""
    rec = measured_counters(kernel, path)
    return rec.get("bytes_per_launch") if rec else None

def line_kernel_counters(kernel: str):
    """Counter record of a whole-line kernel (short name, e.g. k_line_kstep<1024, 1, true, 8,
    false>) from the committed rocprofv3 summary of the forms, or None when it is missing or
    the kernels changed since."""
    try:
        with open(LINE_COUNTERS_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t.get("kernels", {}).get(kernel)


def _timed(torch, fn, reps: int = 1) -> float:
    """Seconds per call of fn (events on the current stream, after one untimed call)."""
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / 1e3 / reps


def _single(w, gi: int, b: int, rk4ip, workloads):
    """Workload of instance b of group gi alone (same instance id, so the same noise)."""
    import numpy as np
    from dataclasses import replace

    g = w.groups[gi]
    gg = replace(g, batch=1, id_base=g.id_base + b,
                 Vgrid=None if g.Vgrid is None else np.asarray(g.Vgrid)[b:b + 1])
    return workloads.Workload(w.name + "_one", [gg], w.h, w.nsteps, [np.asarray(w.psi0[gi])[b:b + 1]])


def form_batched_paths(torch, rk4ip, workloads, steps: int = 200, sample_paths: int = 8):
    """Many stochastic paths per launch vs the plain path (one path per plan, one at a time)."""
    w = workloads.sgpe1d(nsteps=steps)
    g = w.groups[0]
    probs, _k = rk4ip.problems_from_workload(w)
    psi0 = rk4ip.field_to_device(w)
    out = {"workload": f"sgpe1d {g.batch} paths x {g.n[0]} (Philox noise), {steps} steps"}
    results = {}
    tune = rk4ip.RK4IP_FLAG_AUTOTUNE
    for name, flags in (("one_launch_per_step", rk4ip.RK4IP_FLAG_GRAPH | tune),
                        ("fused_steps", rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_FUSE_1D | tune)):
        plan = rk4ip.Plan(probs, flags=flags)
        psi = psi0.clone()
        t = _timed(torch, lambda: (psi.copy_(psi0), plan.run(psi, steps)))
        out[name + "_pt_steps_per_s"] = g.batch * g.M * steps / t
        out[name + "_schedule"] = plan.schedule(0, 0)
        results[name] = psi
        plan.destroy()
    # the plain path: one path per plan, paths run one after another
    plain_ms = 0.0
    same = True
    worst = 0.0
    for b in range(sample_paths):
        w1 = _single(w, 0, b, rk4ip, workloads)
        p1, _k1 = rk4ip.problems_from_workload(w1)
        plan = rk4ip.Plan(p1, flags=rk4ip.RK4IP_FLAG_GRAPH | tune)
        f0 = rk4ip.field_to_device(w1)
        psi = f0.clone()
        plain_ms += _timed(torch, lambda: (psi.copy_(f0), plan.run(psi, steps))) * 1e3
        ref = results["fused_steps"][b * g.M:(b + 1) * g.M]
        same = same and bool(torch.equal(psi, ref))
        worst = max(worst, float(torch.linalg.vector_norm(psi - ref) / torch.linalg.vector_norm(ref)))
        plan.destroy()
    out["plain_pt_steps_per_s"] = sample_paths * g.M * steps / (plain_ms / 1e3)
    out["plain_sample"] = f"{sample_paths} paths, one plan each, run one after another"
    out["speedup_vs_plain"] = out["fused_steps_pt_steps_per_s"] / out["plain_pt_steps_per_s"]
    out["speedup_fused_vs_one_launch_per_step"] = out["fused_steps_pt_steps_per_s"] / out[
        "one_launch_per_step_pt_steps_per_s"]
    out["bitwise_equal_to_plain"] = same  # when both picked the same line kernel
    out["max_rel_diff_to_plain"] = worst
    # VALU issue of the fused kernel from the committed counter run (k-space line step)
    rr = out["fused_steps_schedule"].split(":r")[-1]
    kname = f"k_line_kstep<{g.n[0]}, 1, true, {rr}, false>"
    rec = line_kernel_counters(kname) or {}
    out["kernel"] = kname
    # the issue of its longest launch (many steps over the whole batch, as in the fused
    # form), and the duration-weighted average over every launch of the forms
    out["valu_issue_frac_profiled"] = rec.get("valu_issue_longest_dispatch")
    out["valu_issue_frac_profiled_all_launches"] = rec.get("valu_issue_frac")
    return out


def form_uneven_batch(torch, rk4ip, workloads, steps: int = 100, sample: int = 2):
    """Uneven 2D instances (32 x 128^2 + 32 x 256^2) in one plan vs one plan per instance."""
    w = workloads.adjoint2d(nsteps=steps)
    probs, _k = rk4ip.problems_from_workload(w)
    pts = sum(g.batch * g.M for g in w.groups)
    plan = rk4ip.Plan(probs, flags=rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_AUTOTUNE)
    psi0 = rk4ip.field_to_device(w)
    psi = psi0.clone()
    t = _timed(torch, lambda: (psi.copy_(psi0), plan.run(psi, steps)))
    batched = pts * steps / t
    plan.destroy()
    # one launch per pass kind over both groups (work list), against the per-group launches
    mplan = rk4ip.Plan(probs, flags=rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_MERGE_GROUPS)
    mpsi = psi0.clone()
    tm = _timed(torch, lambda: (mpsi.copy_(psi0), mplan.run(mpsi, steps)))
    merged_rel = float(torch.linalg.vector_norm(mpsi - psi) / torch.linalg.vector_norm(psi))
    mplan.destroy()
    # plain path: `sample` instances of each size, one plan each, one after another
    tot_pts, tot_s = 0, 0.0
    same = True
    off = 0
    for gi, g in enumerate(w.groups):
        for b in range(sample):
            w1 = _single(w, gi, b, rk4ip, workloads)
            p1, _k1 = rk4ip.problems_from_workload(w1)
            pl = rk4ip.Plan(p1, flags=rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_AUTOTUNE)
            f0 = rk4ip.field_to_device(w1)
            x = f0.clone()
            tot_s += _timed(torch, lambda: (x.copy_(f0), pl.run(x, steps)))
            tot_pts += g.M * steps
            ref = psi[off + b * g.M: off + (b + 1) * g.M]
            same = same and float(torch.linalg.vector_norm(x - ref) / torch.linalg.vector_norm(ref)) < 1e-5
            pl.destroy()
        off += g.batch * g.M
    # per-size throughputs weighted by the batch's point counts
    plain = tot_pts / tot_s
    return {"workload": f"adjoint2d shapes (32 x 128^2 + 32 x 256^2), forward, {steps} steps",
            "batched_pt_steps_per_s": batched, "batched_launches_per_step": 2 * len(w.groups),
            "batched_us_per_step": t / steps * 1e6,
            "merged_pt_steps_per_s": pts * steps / tm, "merged_launches_per_step": 2,
            "merged_us_per_step": tm / steps * 1e6, "merged_vs_batched": t / tm,
            "merged_rel_diff_to_batched": merged_rel,
            "plain_pt_steps_per_s": plain,
            "plain_sample": f"{sample} instances of each size, one plan each, one after another",
            "speedup_vs_plain": batched / plain, "merged_speedup_vs_plain": pts * steps / tm / plain,
            "matches_plain_within_1e-5": same}


def _torch_rk4ip(torch, w, psi0_list, V_list, steps):
    """The same midpoint-origin RK4IP step written with torch.fft, for autograd timing only."""
    import math

    outs = []
    for g, psi, V in zip(w.groups, psi0_list, V_list):
        n = g.n
        ks = []
        for a in range(2):
            m = torch.arange(n[a], dtype=torch.float64, device=psi.device)
            ks.append(2 * math.pi / (g.hi[a] - g.lo[a]) * torch.where(m < n[a] // 2, m, m - n[a]))
        k2 = ks[1][:, None] ** 2 + ks[0][None, :] ** 2
        E = torch.exp((-1j * g.alpha * k2 - g.gamma) * (w.h / 2)).to(torch.complex64)
        X, Y = [torch.tensor(c, device=psi.device) for c in g.mesh()]
        Vt = (0.5 * (g.trap[0] * X ** 2 + g.trap[1] * Y ** 2)).to(torch.float32)[None] + V.reshape(psi.shape)
        h = w.h

        def D(f):
            return torch.fft.ifft2(E * torch.fft.fft2(f))

        def hG(f):
            return (-1j * h) * (Vt + g.gnl * (f.real ** 2 + f.imag ** 2)) * f

        for _ in range(steps):
            a = D(psi)
            k1 = D(hG(psi))
            k2 = hG(a + 0.5 * k1)
            k3 = hG(a + 0.5 * k2)
            k4 = hG(D(a + k3))
            psi = D(a + k1 / 6 + k2 / 3 + k3 / 3) + k4 / 6
        outs.append(psi)
    return outs


def form_adjoint(torch, rk4ip, workloads, steps: int = 50, ckpt: int = 10):
    """Gradient of 1 - |<phi|psi(T)>|^2 w.r.t. psi0 and V on the uneven 2D batch: the
    hand-written adjoint (checkpoint every `ckpt` steps) vs the forward run alone and vs
    torch.autograd through the same step written with torch.fft."""
    import numpy as np
    from paper_1204_4255_amd.autograd import RK4IPSolver

    w = workloads.adjoint2d(nsteps=steps, ckpt_every=ckpt)
    probs, _k = rk4ip.problems_from_workload(w)
    # graph-replayed forward run and adjoint segments; the eager solver beside it
    solver = RK4IPSolver(probs, steps, ckpt, flags=rk4ip.RK4IP_FLAG_GRAPH)
    eager = RK4IPSolver(probs, steps, ckpt)
    psi0 = rk4ip.field_to_device(w)
    Vall = torch.tensor(np.concatenate([g.Vgrid.reshape(-1) for g in w.groups]).astype(np.float32), device="cuda")
    phis = [torch.tensor(p.astype(np.complex64).reshape(-1), device="cuda") for p in w.target]
    sizes = [g.batch * g.M for g in w.groups]

    def loss_flat(out):
        tot, off = 0, 0
        for g, phi, n in zip(w.groups, phis, sizes):
            c = g.dV * torch.sum(torch.conj(phi)[None] * out[off:off + n].reshape(g.batch, -1), dim=1)
            tot = tot + torch.sum(1 - torch.abs(c) ** 2)
            off += n
        return tot

    state = {}

    def ours():
        p = psi0.clone().requires_grad_(True)
        V = Vall.clone().requires_grad_(True)
        loss_flat(solver(p, V)).backward()
        state["ours"] = (p.grad, V.grad)

    def fwd_only():
        with torch.no_grad():
            solver(psi0, Vall)

    def ours_eager():
        p = psi0.clone().requires_grad_(True)
        V = Vall.clone().requires_grad_(True)
        loss_flat(eager(p, V)).backward()

    def fwd_eager():
        with torch.no_grad():
            eager(psi0, Vall)

    t_ours = _timed(torch, ours)
    t_fwd = _timed(torch, fwd_only)
    t_ours_eager = _timed(torch, ours_eager)
    t_fwd_eager = _timed(torch, fwd_eager)

    def plain_autograd():
        p = psi0.clone().requires_grad_(True)
        V = Vall.clone().requires_grad_(True)
        ps, vs, off = [], [], 0
        for g, n in zip(w.groups, sizes):
            ps.append(p[off:off + n].reshape(g.shape))
            vs.append(V[off:off + n].reshape(g.shape))
            off += n
        outs = _torch_rk4ip(torch, w, ps, vs, steps)
        loss_flat(torch.cat([o.reshape(-1) for o in outs])).backward()
        state["torch"] = (p.grad, V.grad)

    t_torch = _timed(torch, plain_autograd)
    gp, gv = state["ours"]
    tp, tv = state["torch"]
    rel = lambda a, b: float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
    return {"workload": f"adjoint2d shapes (32 x 128^2 + 32 x 256^2), {steps} steps, checkpoint every {ckpt}",
            "forward_plus_adjoint_s": t_ours, "forward_only_s": t_fwd,
            "gradient_cost_in_forward_runs": t_ours / t_fwd,
            "launch": "hipGraph replays (forward run and whole adjoint segments)",
            "eager_forward_plus_adjoint_s": t_ours_eager, "eager_forward_only_s": t_fwd_eager,
            "eager_gradient_cost_in_forward_runs": t_ours_eager / t_fwd_eager,
            "torch_autograd_s": t_torch, "speedup_vs_torch_autograd": t_torch / t_ours,
            "rel_diff_vs_torch_autograd": {"grad_psi0": rel(gp, tp), "grad_V": rel(gv, tv)}}


def form_fp64_transforms(torch, rk4ip, workloads, steps: int = 100):
    """Throughput of the FP64-transform precision form next to the complex64 form on the
    3D 256^3 and the batched 1D workloads (accuracy of both forms: the GPU parity tests)."""
    out = {}
    for name, w, base in (("gpe3d_256^3", workloads.gpe3d(nsteps=steps), rk4ip.RK4IP_FLAG_AUTOTUNE),
                          ("sgpe1d_2048x1024", workloads.sgpe1d(nsteps=steps),
                           rk4ip.RK4IP_FLAG_FUSE_1D | rk4ip.RK4IP_FLAG_AUTOTUNE)):
        probs, _k = rk4ip.problems_from_workload(w)
        pts = sum(g.batch * g.M for g in w.groups)
        psi0 = rk4ip.field_to_device(w)
        rates = {}
        for form, extra in (("c64", 0), ("fp64_transforms", rk4ip.RK4IP_FLAG_FP64_TRANSFORMS)):
            plan = rk4ip.Plan(probs, flags=rk4ip.RK4IP_FLAG_GRAPH | base | extra)
            psi = psi0.clone()
            plan.run(psi, 40)  # records the replay graph
            t = _timed(torch, lambda: (psi.copy_(psi0), plan.run(psi, steps)))
            rates[form] = pts * steps / t
            plan.destroy()
        out[name] = {"c64_pt_steps_per_s": rates["c64"], "fp64_transforms_pt_steps_per_s": rates["fp64_transforms"],
                     "fp64_cost": rates["c64"] / rates["fp64_transforms"]}
    return out


def form_semi_implicit(torch, rk4ip, workloads, steps: int = 100):
    """The semi-implicit integrator (RK4IP_FLAG_SEMI_IMPLICIT) next to RK4IP: throughput on
    the 3D 256^3 and the batched 1D workloads, the semi-implicit 3D passes' rates (event
    timed, eager), and its strong convergence measured on the GPU: 2048 paths of a damped
    stochastic GPE (64 points on [-8, 8)) to T = 0.64 at h = 2^l h_f with 2^l noise
    substeps, error of each level against the h_f run (one Wiener path per path)."""
    import numpy as np

    SI = rk4ip.RK4IP_FLAG_SEMI_IMPLICIT
    out = {}
    for name, w, base in (("gpe3d_256^3", workloads.gpe3d(nsteps=steps), rk4ip.RK4IP_FLAG_AUTOTUNE),
                          ("sgpe1d_2048x1024", workloads.sgpe1d(nsteps=steps),
                           rk4ip.RK4IP_FLAG_FUSE_1D | rk4ip.RK4IP_FLAG_AUTOTUNE)):
        probs, _k = rk4ip.problems_from_workload(w)
        pts = sum(g.batch * g.M for g in w.groups)
        psi0 = rk4ip.field_to_device(w)
        rates = {}
        for form, extra in (("rk4ip", 0), ("semi_implicit", SI)):
            plan = rk4ip.Plan(probs, flags=rk4ip.RK4IP_FLAG_GRAPH | base | extra)
            psi = psi0.clone()
            plan.run(psi, 40)  # records the replay graph
            t = _timed(torch, lambda: (psi.copy_(psi0), plan.run(psi, steps)))
            rates[form] = pts * steps / t
            plan.destroy()
        rec = {"rk4ip_pt_steps_per_s": rates["rk4ip"], "semi_implicit_pt_steps_per_s": rates["semi_implicit"],
               "semi_implicit_ms_per_step": pts / rates["semi_implicit"] * 1e3,
               "speed_ratio": rates["semi_implicit"] / rates["rk4ip"]}
        if w.groups[0].ndim == 3:
            plan = rk4ip.Plan(probs, flags=base | SI)
            work = psi0.clone()
            plan.run(work, 3)
            plan.profile(True)
            plan.run(work, 20, step0=3)
            rec["passes"] = []
            for i in range(plan.num_passes(0)):
                n, mean = plan.profile_read(0, i)
                nm = plan.schedule(0, i)
                gbs = PASS_BYTES[nm.split(":")[0]] * pts / (mean / 1e3) / 1e9 if n else None
                rec["passes"].append({"pass": nm, "launches": n, "mean_ms": mean, "achieved_GBps": gbs,
                                      "hbm_frac": gbs / HBM_PEAK_GBS if gbs else None})
            plan.destroy()
        out[name] = rec

    g = workloads.Group(n=(64,), lo=(-8.0,), hi=(8.0,), batch=2048, gnl=10.0, gamma=0.05, sigma=0.1,
                        trap=(1.0, 0.0, 0.0), seed=21)
    x = g.axis(0)
    psi0 = np.broadcast_to(np.pi ** -0.25 * np.exp(-x ** 2 / 2), g.shape)
    hf, T = 2.5e-4, 0.64
    nf = int(round(T / hf))

    def run(S):
        w = workloads.Workload("sc", [g], hf * S, nf // S, [psi0])
        probs, _k = rk4ip.problems_from_workload(w, noise_substeps=S)
        plan = rk4ip.Plan(probs, flags=SI | rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_FUSE_1D
                          | rk4ip.RK4IP_FLAG_FP64_TRANSFORMS)
        d = rk4ip.field_to_device(w)
        plan.run(d, nf // S)
        torch.cuda.synchronize()
        plan.destroy()
        return d.cpu().numpy().astype(np.complex128).reshape(g.shape)

    fine = run(1)
    levels = []
    for S in (32, 16, 8, 4, 2):
        e = np.linalg.norm(run(S) - fine, axis=1) / np.linalg.norm(fine, axis=1)
        levels.append({"h": hf * S, "noise_substeps": S, "mean_strong_error": float(np.mean(e)),
                       "stderr": float(np.std(e, ddof=1) / np.sqrt(len(e)))})
    orders = [float(np.log2(levels[i]["mean_strong_error"] / levels[i + 1]["mean_strong_error"]))
              for i in range(len(levels) - 1)]
    out["strong_convergence"] = {"workload": "2048 paths x 64 points, g = 10, gamma = 0.05, sigma = 0.1, T = 0.64, "
                                             "reference h_f = 2.5e-4 (FP64 transforms)",
                                 "levels": levels, "orders": orders}
    return out


def form_ark45(torch, rk4ip, workloads):
    """The adaptive Cash-Karp RK4(5) in the interaction picture (rk4ip_ark45, 1D): 2048
    lines of a trapped 1D GPE (1024 points) over t = 0.5 at tol 1e-6, each line adapting
    its own step; the cost of an accepted step
    next to a fixed RK4IP step on the same lattice; and the accepted steps of one soliton
    (tol 1e-7, t = 2) at resolutions 256 ... 4096, which the interaction picture keeps
    constant (the paper's step-count figure)."""
    import numpy as np

    out = {}
    # 2048 trapped lines on [-8, 8) (h max V stays inside the explicit pair's stability
    # interval), each displaced differently so that every line takes its own steps
    g = workloads.Group(n=(1024,), lo=(-8.0,), hi=(8.0,), gnl=1.0, trap=(1.0, 0.0, 0.0), batch=2048)
    x = g.axis(0)
    shift = np.linspace(0.0, 2.0, g.batch)[:, None]
    f0 = np.pi ** -0.25 * np.exp(-(x[None] - shift) ** 2 / 2)
    w = workloads.Workload("ark45_2048x1024", [g], 1e-3, 100, [f0])
    probs = [rk4ip.make_problem(g.n, g.lo, g.hi, w.h, batch=g.batch, alpha=g.alpha, gamma=g.gamma, g_nl=g.gnl,
                                trap=g.trap)]
    plan = rk4ip.Plan(probs)
    psi0 = rk4ip.field_to_device(w)
    psi = psi0.clone()
    h = torch.full((g.batch,), 1e-3, dtype=torch.float64, device="cuda")
    T, tol = 0.5, 1e-6
    plan.ark45(psi, T, tol, h)  # warm-up
    psi.copy_(psi0)
    h.fill_(1e-3)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    stats, _ = plan.ark45(psi, T, tol, h)
    b.record()
    torch.cuda.synchronize()
    t = a.elapsed_time(b) / 1e3
    st = stats.cpu().numpy()
    accepted = int(st[:, 0].sum())
    plan.destroy()
    fixed = rk4ip.Plan(probs, flags=rk4ip.RK4IP_FLAG_FUSE_1D | rk4ip.RK4IP_FLAG_AUTOTUNE | rk4ip.RK4IP_FLAG_GRAPH)
    psi.copy_(psi0)
    tf = _timed(torch, lambda: fixed.run(psi, 100))
    fixed.destroy()
    out["batched"] = {"workload": "2048 x 1024 trapped 1D GPE on [-8, 8) (g = 1, no noise, displaced "
                                  "Gaussians), t = 0.5, tol = 1e-6",
                      "seconds": t, "accepted_steps_mean": accepted / g.batch,
                      "rejected_steps_total": int(st[:, 1].sum()), "all_reached_end": bool(np.all(st[:, 2] == 1)),
                      "accepted_pt_steps_per_s": accepted * g.M / t,
                      "us_per_accepted_step": t / (accepted / g.batch) * 1e6,
                      "rk4ip_fixed_us_per_step": tf / 100 * 1e6,
                      "accepted_step_cost_in_rk4ip_steps": (t / (accepted / g.batch)) / (tf / 100)}
    counts, ex_counts = {}, {}
    for n in (256, 512, 1024, 2048, 4096):
        gs = workloads.Group(n=(n,), lo=(-20.0,), hi=(20.0,), gnl=-1.0)
        x = gs.axis(0)
        f0 = (1 / np.cosh(x) * np.exp(0.5j * x)).astype(np.complex64)
        pl = rk4ip.Plan([rk4ip.make_problem(gs.n, gs.lo, gs.hi, 1e-3, g_nl=-1.0)])
        for explicit, dst in ((False, counts), (True, ex_counts)):
            if explicit and n > 1024:
                continue  # the explicit method needs ~N^2 steps
            d = torch.tensor(f0, device="cuda")
            hh = torch.full((1,), 1e-3, dtype=torch.float64, device="cuda")
            s1, _ = pl.ark45(d, 2.0, 1e-7, hh, explicit=explicit)
            dst[str(n)] = int(s1[0, 0])
        pl.destroy()
    out["steps_vs_resolution"] = {"workload": "NLSE soliton on [-20, 20), t = 2, tol = 1e-7",
                                  "accepted_steps": counts, "accepted_steps_explicit_method": ex_counts}
    return out


def form_potential_terms(torch, rk4ip, workloads, steps: int = 100):
    """The batched 1D workload (2048 x 1024, RK4IP, graph-replayed fused launches) with the
    potential's extra terms: the real Wiener noise in the potential (sigma_V = 0.01), the
    non-local potential (a softened Coulomb kernel, strength 0.1), and both, next to the
    plain step."""
    import numpy as np

    w = workloads.sgpe1d(nsteps=steps)
    g = w.groups[0]
    n, L = g.n[0], g.hi[0] - g.lo[0]
    d = np.arange(n)
    d = np.where(d < n // 2, d, d - n) * (L / n)
    K = 0.1 / np.sqrt(d ** 2 + 1.0)
    psi0 = rk4ip.field_to_device(w)
    pts = g.batch * g.M
    out = {"workload": "2048 x 1024 damped stochastic 1D GPE, RK4IP, 100 steps per timed run"}
    for name, sv, ck in (("plain", 0.0, None), ("noisy_potential", 0.01, None), ("non_local", 0.0, K),
                         ("both", 0.01, K)):
        p = rk4ip.make_problem(g.n, g.lo, g.hi, w.h, batch=g.batch, alpha=g.alpha, gamma=g.gamma, g_nl=g.gnl,
                               trap=g.trap, sigma=g.sigma, seed=g.seed, id_base=g.id_base, sigma_V=sv, conv_K=ck)
        plan = rk4ip.Plan([p], flags=rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_FUSE_1D | rk4ip.RK4IP_FLAG_AUTOTUNE)
        psi = psi0.clone()
        plan.run(psi, 40)
        t = _timed(torch, lambda: (psi.copy_(psi0), plan.run(psi, steps)))
        out[name] = {"pt_steps_per_s": pts * steps / t, "us_per_step": t / steps * 1e6}
        plan.destroy()
    for k in ("noisy_potential", "non_local", "both"):
        out[k]["cost_vs_plain"] = out["plain"]["pt_steps_per_s"] / out[k]["pt_steps_per_s"]
    return out


def form_bases(torch, rk4ip, workloads, steps: int = 100):
    """The cosine basis on a half domain next to the Fourier basis on the full one (the
    half-interval example of Sec. 4, batched): 2048 lines of the trapped 1D GPE, 512
    cosine points on (0, 8) against 1024 Fourier points on (-8, 8), graph-replayed with
    several steps per launch."""
    import numpy as np

    out = {"workload": "2048 lines, trapped 1D GPE (g = 1), 512 cosine points on (0, 8) vs 1024 Fourier points "
                       "on (-8, 8), 100 steps"}
    B, n, L, h = 2048, 512, 8.0, 1e-3
    dx = L / n
    x = (np.arange(n) + 0.5) * dx
    f_half = np.broadcast_to(np.pi ** -0.25 * np.exp(-x ** 2 / 2), (B, n)).astype(np.complex64)
    f_full = np.concatenate([f_half[:, ::-1], f_half], axis=1)
    for name, prob, f in (
            ("cosine_half", rk4ip.make_problem((n,), (0.0,), (L,), h, batch=B, g_nl=1.0, trap=(1.0, 0, 0), basis=1),
             f_half),
            ("fourier_full", rk4ip.make_problem((2 * n,), (-L + dx / 2,), (L + dx / 2,), h, batch=B, g_nl=1.0,
                                                trap=(1.0, 0, 0)), f_full)):
        plan = rk4ip.Plan([prob], flags=rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_AUTOTUNE | rk4ip.RK4IP_FLAG_FUSE_1D)
        psi0 = torch.tensor(f.reshape(-1), device="cuda")
        psi = psi0.clone()
        plan.run(psi, 40)
        t = _timed(torch, lambda: (psi.copy_(psi0), plan.run(psi, steps)))
        out[name] = {"us_per_step": t / steps * 1e6, "stored_points": int(psi0.numel())}
        plan.destroy()
    out["time_ratio_half_to_full"] = out["cosine_half"]["us_per_step"] / out["fourier_full"]["us_per_step"]
    return out


def _pass_times(rk4ip, plan, psi0, steps: int = 20):
    """Per-pass (schedule, launches, mean ms) of an eager run, with HIP events on the
    plan's stream."""
    work = psi0.clone()
    plan.run(work, 3)
    plan.profile(True)
    plan.run(work, steps, step0=3)
    out = []
    for i in range(plan.num_passes(0)):
        n, mean = plan.profile_read(0, i)
        out.append({"pass": plan.schedule(0, i), "launches": n, "mean_us": mean * 1e3})
    plan.profile(False)
    return out


def other_workloads(torch, rk4ip, workloads):
    """Throughput of the 1D NLSE (256 points, 1000 steps) and the 2D GPE (512^2, 2000 steps)
    at their full run lengths, graph-replayed with tuned schedules. The 2D GPE's form of
    record is the FP64-transform form (the complex64 form sits at the 1e-5 limit over the
    run); both are timed, with their per-pass launch times."""
    out = {}
    A, FP64 = rk4ip.RK4IP_FLAG_AUTOTUNE, rk4ip.RK4IP_FLAG_FP64_TRANSFORMS
    for name, w, flags in (("nlse1d_256", workloads.nlse1d(), rk4ip.RK4IP_FLAG_FUSE_1D | A),
                           ("gpe2d_512^2", workloads.gpe2d(), A | FP64),
                           ("gpe2d_512^2_complex64", workloads.gpe2d(), A)):
        probs, _k = rk4ip.problems_from_workload(w)
        pts = sum(g.batch * g.M for g in w.groups)
        plan = rk4ip.Plan(probs, flags=rk4ip.RK4IP_FLAG_GRAPH | flags)
        psi0 = rk4ip.field_to_device(w)
        psi = psi0.clone()
        t = _timed(torch, lambda: (psi.copy_(psi0), plan.run(psi, w.nsteps)))
        out[name] = {"steps": w.nsteps, "seconds": t, "pt_steps_per_s": pts * w.nsteps / t,
                     "us_per_step": t / w.nsteps * 1e6}
        plan.destroy()
        if w.groups[0].ndim == 2:
            eager = rk4ip.Plan(probs, flags=flags)
            out[name]["passes_eager"] = _pass_times(rk4ip, eager, psi0)
            eager.destroy()
    out["gpe2d_512^2"]["form"] = "FP64 transforms (the form that holds 1e-5 over the run)"
    out["gpe2d_512^2_complex64"]["form"] = "complex64 (not claimed: at the 1e-5 limit over the run)"
    return out


def progress(msg: str) -> None:
    """One line on stderr as each stage ends (the JSON result alone goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


FORMS = (("other_workloads", other_workloads), ("batched_paths", form_batched_paths),
         ("uneven_batch", form_uneven_batch), ("adjoint", form_adjoint),
         ("fp64_transforms", form_fp64_transforms), ("semi_implicit", form_semi_implicit),
         ("ark45", form_ark45), ("potential_terms", form_potential_terms), ("bases", form_bases))


def measure_forms(torch, rk4ip, workloads, only=None):
    out = {}
    for name, fn in FORMS:
        if only is not None and name not in only:
            continue
        t0 = time.perf_counter()
        out[name] = fn(torch, rk4ip, workloads)
        progress(f"form {name} done ({time.perf_counter() - t0:.1f} s)")
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--no-graph", action="store_true", help="launch passes eagerly instead of replaying a hipGraph")
    ap.add_argument("--no-autotune", action="store_true", help="use the default tile schedules")
    ap.add_argument("--semi-implicit", action="store_true",
                    help="time the semi-implicit step instead of RK4IP (not the headline line; for profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched and adjoint forms (each timed against the plain path)")
    ap.add_argument("--forms-only", action="store_true", help="measure only the batched and adjoint forms")
    ap.add_argument("--forms", default=None,
                    help="comma-separated subset of the forms to measure (default: all of them)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one elementwise copy kernel of 256 MiB in + 256 MiB out (a reference for "
                         "rocprofv3 FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()
    only = None
    if args.forms is not None:
        only = [f.strip() for f in args.forms.split(",") if f.strip()]
        unknown = sorted(set(only) - {name for name, _ in FORMS})
        if unknown:
            ap.error(f"unknown forms {unknown}; known: {[name for name, _ in FORMS]}")
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the multi-GPU path is a design "
                          "(slab decomposition with RCCL all-to-all), not implemented", "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    from paper_1204_4255_amd import rk4ip, workloads

    torch.cuda.set_device(0)
    if args.forms_only:
        print(json.dumps({"forms": measure_forms(torch, rk4ip, workloads, only)}))
        return 0
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    w = workloads.gpe3d(nsteps=args.steps)
    g = w.groups[0]
    pts = g.M * g.batch
    probs, _keep = rk4ip.problems_from_workload(w)
    tune = 0 if args.no_autotune else rk4ip.RK4IP_FLAG_AUTOTUNE
    tune |= rk4ip.RK4IP_FLAG_SEMI_IMPLICIT if args.semi_implicit else 0
    flags = (0 if args.no_graph else rk4ip.RK4IP_FLAG_GRAPH) | tune
    traffic_file = TRAFFIC_FILE_SI if args.semi_implicit else TRAFFIC_FILE
    plan = rk4ip.Plan(probs, flags=flags)
    psi0 = rk4ip.field_to_device(w)
    psi = psi0.clone()

    # record the replay graph (it holds up to 32 steady-state steps) on a throwaway run,
    # restore the field, then warmup and exactly --steps timed steps bracketed by
    # synchronisation
    plan.run(psi, 40, step0=0)
    psi.copy_(psi0)
    plan.run(psi, args.warmup, step0=0)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    plan.run(psi, args.steps, step0=args.warmup)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    ms_per_step = ms / args.steps
    value = pts * args.steps / (ms / 1e3)
    progress(f"timed {args.steps} steps: {ms_per_step:.4f} ms per step")

    # per-pass launch times with HIP events on the plan's stream (eager launches)
    prof_plan = rk4ip.Plan(probs, flags=tune)
    work = psi0.clone()
    prof_plan.run(work, 3)
    prof_plan.profile(True)
    prof_plan.run(work, args.profile_steps, step0=3)
    passes = []
    for i in range(prof_plan.num_passes(0)):
        n, mean = prof_plan.profile_read(0, i)
        passes.append({"pass": prof_plan.schedule(0, i), "launches": n, "mean_ms": mean})
    prof_plan.profile(False)
    # group by kernel (same kind and axis kind share one kernel)
    kernels = {}
    for p in passes:
        kind, axis, n_, layout = p["pass"].split(":")[:4]
        key = f"{kind}:{layout}"
        k = kernels.setdefault(key, {"launches": 0, "total_ms": 0.0, "kind": kind})
        k["launches"] += p["launches"]
        k["total_ms"] += p["launches"] * p["mean_ms"]
    dom_name, dom = max(kernels.items(), key=lambda kv: kv[1]["total_ms"])
    dom_mean_ms = dom["total_ms"] / dom["launches"]
    bytes_per_launch = PASS_BYTES[dom["kind"]] * pts
    achieved = bytes_per_launch / (dom_mean_ms / 1e3) / 1e9
    traffic = measured_traffic(dom_name, traffic_file)
    counters = measured_counters(dom_name, traffic_file) or {}
    per_kernel = []
    for name, k in sorted(kernels.items(), key=lambda kv: -kv[1]["total_ms"]):
        mean = k["total_ms"] / k["launches"]
        gbs = PASS_BYTES[k["kind"]] * pts / (mean / 1e3) / 1e9
        c = measured_counters(name, traffic_file) or {}
        per_kernel.append({"kernel": name, "mean_ms": mean, "launches": k["launches"], "achieved_GBps": gbs,
                           "hbm_frac": gbs / HBM_PEAK_GBS, "valu_issue_frac_profiled": c.get("valu_issue_frac"),
                           "traffic_ratio_profiled": c.get("ratio")})
    # bytes per step averaged over the profiled run (each pass weighted by its launches)
    step_bytes = sum(PASS_BYTES[p["pass"].split(":")[0]] * p["launches"] for p in passes) * pts / args.profile_steps

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic: seeded 3D GPE initial field (trap ground state x N(0,0.05^2) phase noise)",
        "config": {"workload": "gpe3d_256^3", "lattice": [256, 256, 256], "domain": [-10, 10], "dt": w.h,
                   "g": 2000.0, "trap": [1.0, 1.5, 2.0], "instances": 1,
                   "launch": "hipGraph of 32 steps" if not args.no_graph else "eager passes",
                   "autotune": not args.no_autotune,
                   "integrator": "semi-implicit" if args.semi_implicit else "rk4ip"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": dom_name, "kernel_mean_ms": dom_mean_ms,
                     "bytes_per_launch": bytes_per_launch,
                     "valu_issue_frac_profiled": counters.get("valu_issue_frac")},
        "kernels": per_kernel,
        "step_roofline": {"bytes_per_step": step_bytes, "achieved_GBps": step_bytes / (ms_per_step / 1e3) / 1e9,
                          "frac": step_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS},
        "passes": passes,
        "wall_s": wall,
    }

    if not args.no_cpu_baseline:
        import oracle

        # bounded sample: the first CPU_STEPS steps of the same 256^3 workload from the
        # same initial field (about 10 s of FP64 work on a 16-core host)
        cpu_steps = 8
        f0 = np.asarray(w.psi0[0], dtype=np.complex64).astype(np.complex128)
        op = oracle.Problem(n=g.n, lo=g.lo, hi=g.hi, h=w.h, batch=1, alpha=g.alpha, gamma=g.gamma, gnl=g.gnl,
                            trap=g.trap)
        t0 = time.perf_counter()
        ref, _, _ = oracle.run(op, f0, cpu_steps)
        cpu_s = time.perf_counter() - t0
        one = psi0.clone()
        plan.run(one, cpu_steps)
        got = one.cpu().numpy().astype(np.complex128).reshape(ref.shape)
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        result["cpu_baseline"] = {"value": pts * cpu_steps / cpu_s, "unit": "grid-point-steps/s",
                                  "cores": oracle.threads(), "kind": "oracle",
                                  "sample": f"the first {cpu_steps} steps of the 256^3 workload (FP64, radix-2 FFT)",
                                  "seconds": cpu_s}
        result[f"parity_{cpu_steps}step_rel_l2"] = err
        progress(f"cpu baseline done ({cpu_s:.1f} s)")
    if not args.no_forms:
        result["forms"] = measure_forms(torch, rk4ip, workloads, only)
    print(json.dumps(result))
    plan.destroy()
    prof_plan.destroy()
    return 0


if __name__ == "__main__":
    sys.exit(main())
