"""Shared helpers of the GPU parity tests (inputs from the workloads module, reference
values from the FP64 oracle, results from the HIP library through the C ABI)."""
import sys

import numpy as np

import oracle
from paper_1204_4255_amd import rk4ip, workloads as W


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oprob(g: W.Group, h: float, integrator: int = 0, noise_substeps: int = 1) -> oracle.Problem:
    return oracle.Problem(n=g.n, lo=g.lo, hi=g.hi, h=h, batch=g.batch, alpha=g.alpha, gamma=g.gamma, gnl=g.gnl,
                          trap=g.trap, sigma=g.sigma, seed=g.seed, id_base=g.id_base,
                          Vgrid=None if g.Vgrid is None else np.asarray(g.Vgrid, np.float32).astype(np.float64),
                          integrator=integrator, noise_substeps=noise_substeps)


def rel(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_per_instance(a, b, batch):
    a = np.asarray(a).reshape(batch, -1)
    b = np.asarray(b).reshape(batch, -1)
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def plan_for(w: W.Workload, flags: int = 0, noise_substeps: int = 1):
    probs, keep = rk4ip.problems_from_workload(w, noise_substeps=noise_substeps)
    plan = rk4ip.Plan(probs, flags=flags)
    plan._keep_V = keep
    return plan


def random_field(g: W.Group, seed: int, envelope: bool = True):
    r = np.random.Generator(np.random.PCG64(seed))
    f = r.standard_normal(g.shape) + 1j * r.standard_normal(g.shape)
    if envelope:
        grids = g.mesh()
        env = np.exp(-sum((X / (0.3 * (g.hi[a] - g.lo[a]))) ** 2 for a, X in enumerate(grids)))
        f = f * env[None] + 0.3 * env[None]
    return f.astype(np.complex128)


def quantised(f):
    """The complex64 value both sides start from."""
    return np.asarray(f, dtype=np.complex64).astype(np.complex128)


def assert_same_runs(torch, groups, whole, other, split, kspace_lines=True):
    """Runs of one workload: `whole` and `other` are one run call each (through different
    launch structures: eager, graph-replayed, several 1D steps per launch) and are bitwise
    equal; `split` is the same run as two calls. A 1D Fourier line run in FP32 keeps its
    state in k-space for the whole of a run call and transforms it back at the end, so
    where a run is split its lines agree to rounding (relative 1e-6) instead; every other
    group is bitwise equal there too."""
    off = 0
    for g in groups:
        n = g.batch * g.M
        ref = whole[off:off + n]
        assert torch.equal(other[off:off + n], ref), g.n
        x = split[off:off + n]
        if kspace_lines and len(g.n) == 1:
            assert float(torch.linalg.vector_norm(x - ref) / torch.linalg.vector_norm(ref)) < 1e-6, g.n
        else:
            assert torch.equal(x, ref), g.n
        off += n
