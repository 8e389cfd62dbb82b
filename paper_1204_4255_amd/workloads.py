"""Seeded synthetic workloads for the RK4IP step (inputs only).

This module builds the problem parameters and initial fields of the five workloads the
library is measured and checked on. It holds none of the method's arithmetic: no
transform, no propagator, no right-hand side. Both the HIP path and the CPU oracle take
their inputs from here, so they start from bit-identical complex128/float64 arrays.

The equations are the dimensionless nonlinear Schroedinger / Gross-Pitaevskii family
of Dennis, Hope & Johnsson (arXiv:1204.4255) Sec. 3.6 eq. (7) and Sec. 4.1 eq. (9):

    i dpsi/dt = -alpha lap psi + V psi + g |psi|^2 psi   (+ damping, + additive noise)

with alpha = 1/2. Lattices are periodic Fourier lattices (Sec. 3.1) with axis 0 (x)
contiguous in memory. The initial condition of Sec. 4.1 eq. (10) (the trap ground
state) is used where the workload calls for a Gaussian. Random inputs (phase noise,
potential grids) come from numpy's PCG64 generator seeded per workload.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence

import numpy as np


@dataclass
class Group:
    """One group of same-shape instances (paths or problem instances)."""

    n: Sequence[int]            # points per axis, axis 0 = x (contiguous)
    lo: Sequence[float]
    hi: Sequence[float]
    batch: int = 1
    alpha: float = 0.5
    gamma: float = 0.0
    gnl: float = 0.0
    trap: Sequence[float] = (0.0, 0.0, 0.0)
    sigma: float = 0.0
    seed: int = 0
    id_base: int = 0
    Vgrid: Optional[np.ndarray] = None   # [batch][M] float64 extra potential

    @property
    def ndim(self) -> int:
        return len(self.n)

    @property
    def M(self) -> int:
        return int(np.prod(self.n))

    @property
    def shape(self):
        return (self.batch,) + tuple(int(v) for v in reversed(self.n))

    def axis(self, a: int) -> np.ndarray:
        """Lattice coordinates x_{a,j} = lo + j (hi - lo)/n, half-open domain."""
        n = int(self.n[a])
        return self.lo[a] + np.arange(n) * ((self.hi[a] - self.lo[a]) / n)

    def mesh(self):
        """Coordinate arrays broadcast to the field shape without the batch axis."""
        axes = [self.axis(a) for a in range(self.ndim)]
        grids = np.meshgrid(*reversed(axes), indexing="ij")  # slowest axis first
        return list(reversed(grids))  # grids[a] is coordinate a

    @property
    def dV(self) -> float:
        return float(np.prod([(self.hi[a] - self.lo[a]) / self.n[a] for a in range(self.ndim)]))


@dataclass
class Workload:
    name: str
    groups: List[Group]
    h: float
    nsteps: int
    psi0: List[np.ndarray]                 # per group, complex128 [batch, ...]
    sample_every: int = 0
    ckpt_every: int = 0
    target: Optional[List[np.ndarray]] = None   # per group overlap target (no batch axis)
    description: str = ""

    @property
    def points(self) -> int:
        return sum(g.M * g.batch for g in self.groups)

    @property
    def ndim(self) -> int:
        return self.groups[0].ndim


def _renormalise(psi: np.ndarray, dV: float, N: float = 1.0) -> np.ndarray:
    s = np.sum(np.abs(psi) ** 2) * dV
    return psi * np.sqrt(N / s)


def nlse1d(n: int = 256, nsteps: int = 1000, h: float = 1e-3) -> Workload:
    """Focusing NLSE i psi_t = -1/2 psi_xx - |psi|^2 psi on [-20,20), psi0 = sech(x) e^{0.5 i x}."""
    g = Group(n=(n,), lo=(-20.0,), hi=(20.0,), gnl=-1.0)
    x = g.axis(0)
    psi0 = (1.0 / np.cosh(x) * np.exp(0.5j * x)).astype(np.complex128)[None, :]
    return Workload("nlse1d_n%d" % n, [g], h, nsteps, [psi0], sample_every=50,
                    description="1D focusing NLSE soliton, periodic x in [-20,20)")


def gpe2d(n: int = 512, nsteps: int = 2000, h: float = 5e-4, seed: int = 2) -> Workload:
    """2D GPE with trap 1/2 r^2, g = 500, Thomas-Fermi start with N(0, 0.1^2) phase noise."""
    gnl = 500.0
    g = Group(n=(n, n), lo=(-12.0, -12.0), hi=(12.0, 12.0), gnl=gnl, trap=(1.0, 1.0, 0.0), seed=seed)
    X, Y = g.mesh()
    mu = np.sqrt(gnl * 1.0 / np.pi)          # 2D Thomas-Fermi chemical potential for N = 1
    dens = np.maximum(mu - 0.5 * (X ** 2 + Y ** 2), 0.0) / gnl
    rng = np.random.Generator(np.random.PCG64(seed))
    phase = rng.normal(0.0, 0.1, size=dens.shape)
    psi = np.sqrt(dens) * np.exp(1j * phase)
    psi = _renormalise(psi, g.dV)[None].astype(np.complex128)
    return Workload("gpe2d_%dx%d" % (n, n), [g], h, nsteps, [psi], sample_every=100,
                    description="2D GPE, Thomas-Fermi x seeded phase noise on [-12,12)^2")


def sgpe1d(paths: int = 2048, n: int = 1024, nsteps: int = 5000, h: float = 1e-3, seed: int = 3,
           gamma: float = 0.01, sigma: float = 1e-3, gnl: float = 1.0, L: float = 16.0) -> Workload:
    """Damped stochastic 1D GPE, trap 1/2 x^2, additive complex Wiener noise, many paths."""
    g = Group(n=(n,), lo=(-L,), hi=(L,), batch=paths, gnl=gnl, gamma=gamma, sigma=sigma,
              trap=(1.0, 0.0, 0.0), seed=seed)
    x = g.axis(0)
    psi = (np.pi ** -0.25 * np.exp(-x ** 2 / 2)).astype(np.complex128)
    psi0 = np.broadcast_to(psi, (paths, n)).copy()
    return Workload("sgpe1d_%dx%d" % (paths, n), [g], h, nsteps, [psi0], sample_every=500,
                    description="stochastic damped 1D GPE, independent Philox paths")


def gpe3d(n: int = 256, nsteps: int = 500, h: float = 2e-4, seed: int = 4) -> Workload:
    """3D GPE on [-10,10)^3, trap 1/2(x^2 + 1.5 y^2 + 2 z^2), g = 2000, Gaussian x phase noise."""
    trap = (1.0, 1.5, 2.0)
    g = Group(n=(n, n, n), lo=(-10.0,) * 3, hi=(10.0,) * 3, gnl=2000.0, trap=trap, seed=seed)
    X, Y, Z = g.mesh()
    w = np.sqrt(np.array(trap))
    psi = np.ones(X.shape, dtype=np.complex128)
    for wa, Xa in zip(w, (X, Y, Z)):
        psi = psi * (wa / np.pi) ** 0.25 * np.exp(-wa * Xa ** 2 / 2)
    rng = np.random.Generator(np.random.PCG64(seed))
    psi = psi * np.exp(1j * rng.normal(0.0, 0.05, size=psi.shape))
    psi = _renormalise(psi, g.dV)[None].astype(np.complex128)
    return Workload("gpe3d_%d^3" % n, [g], h, nsteps, [psi], sample_every=50,
                    description="3D GPE, trap ground-state Gaussian x seeded phase noise")


def adjoint2d(n_small: int = 128, n_large: int = 256, b_small: int = 32, b_large: int = 32,
              nsteps: int = 1000, h: float = 1e-3, seed: int = 5, ckpt_every: int = 50,
              L: float = 8.0) -> Workload:
    """Uneven batch of 2D GPE instances with learnable potential grids (seeded N(0, 0.01^2))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    groups, psi0, target = [], [], []
    base = 0
    for n, b in ((n_small, b_small), (n_large, b_large)):
        if b == 0:
            continue
        g = Group(n=(n, n), lo=(-L, -L), hi=(L, L), batch=b, gnl=100.0, trap=(1.0, 1.0, 0.0),
                  seed=seed, id_base=base)
        g.Vgrid = rng.normal(0.0, 0.01, size=(b, n * n)).astype(np.float64)
        X, Y = g.mesh()
        psi = (np.pi ** -0.5 * np.exp(-(X ** 2 + Y ** 2) / 2)).astype(np.complex128)
        psi0.append(np.broadcast_to(psi, (b, n, n)).copy())
        target.append((np.pi ** -0.5 * np.exp(-((X - 0.5) ** 2 + Y ** 2) / 2)).astype(np.complex128))
        groups.append(g)
        base += b
    return Workload("adjoint2d_%dx%d^2+%dx%d^2" % (b_small, n_small, b_large, n_large), groups, h, nsteps,
                    psi0, ckpt_every=ckpt_every, target=target,
                    description="uneven 2D GPE batch, loss 1-|<phi|psi(T)>|^2, gradients wrt psi0 and V")


WORKLOADS = {
    "nlse1d": nlse1d,
    "gpe2d": gpe2d,
    "sgpe1d": sgpe1d,
    "gpe3d": gpe3d,
    "adjoint2d": adjoint2d,
}


def with_steps(w: Workload, nsteps: int) -> Workload:
    return replace(w, nsteps=nsteps)
