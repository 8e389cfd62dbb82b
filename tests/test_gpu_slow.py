"""Slow GPU parity run, skipped unless RK4IP_SLOW_TESTS=1: the 3D GPE on 256^3 for its
full 500 steps, RK4IP and the semi-implicit step, the whole field of both precision forms
against the FP64 oracle every 50 steps. The oracle needs about ten (RK4IP) or seven
(semi-implicit) minutes of 16 host cores for this, so it prints its progress every 25
steps."""
import os
import time

import numpy as np
import pytest

import oracle
from gpu_helpers import log, oprob, quantised, rel
from paper_1204_4255_amd import rk4ip
from paper_1204_4255_amd import workloads as W

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("RK4IP_SLOW_TESTS") != "1", reason="set RK4IP_SLOW_TESTS=1")]


@pytest.mark.parametrize("integrator", [0, 1], ids=["rk4ip", "semi_implicit"])
def test_gpe3d_256_full_run_vs_oracle(integrator):
    import torch

    w = W.gpe3d()
    g = w.groups[0]
    p = oprob(g, w.h, integrator=integrator)
    f = quantised(w.psi0[0])
    probs, _k = rk4ip.problems_from_workload(w)
    base = rk4ip.RK4IP_FLAG_GRAPH | rk4ip.RK4IP_FLAG_AUTOTUNE | (rk4ip.RK4IP_FLAG_SEMI_IMPLICIT if integrator else 0)
    forms = {"c64": base, "fp64": base | rk4ip.RK4IP_FLAG_FP64_TRANSFORMS}
    plans = {k: rk4ip.Plan(probs, flags=fl) for k, fl in forms.items()}
    fields = {k: torch.tensor(f.astype(np.complex64).reshape(-1), device="cuda") for k in forms}
    ref = f.copy()
    errs = {k: [] for k in forms}
    t0 = time.time()
    for s in range(0, w.nsteps, w.sample_every):
        for k in forms:
            plans[k].run(fields[k], w.sample_every, step0=s)
        for h in range(0, w.sample_every, 25):
            ref, _, _ = oracle.run(p, ref, 25, step0=s + h)
            log(f"  oracle at step {s + h + 25} ({time.time() - t0:.0f} s)")
        for k in forms:
            errs[k].append(rel(fields[k].cpu().numpy().astype(np.complex128).reshape(g.shape), ref))
        log(f"  step {s + w.sample_every}: " + ", ".join(f"{k} {errs[k][-1]:.3e}" for k in forms))
    for k in forms:
        log(f"  {k}: max rel L2 over the run {max(errs[k]):.3e}")
        assert max(errs[k]) < 1e-5
