"""Double-precision CPU oracle for the RK4 interaction-picture (RK4IP) step.

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package. It shares no code with the HIP
library in ``paper_1204_4255_amd``; the two meet only through the seeded inputs of
``paper_1204_4255_amd.workloads`` (which hold none of the method's arithmetic).

The arithmetic lives in ``rk4ip_oracle.c`` (plain C99, FP64, own radix-2 FFT and
brute-force DFT, own Philox4x32-10). This module compiles it with gcc and wraps it with
ctypes over numpy arrays. Every function states which part of Dennis, Hope & Johnsson,
arXiv:1204.4255 it follows; the readings where the paper is silent are listed at the
top of ``rk4ip_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rk4ip_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP) into ``oracle/liboracle.so``."""
    cmd = [
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fcx-limited-range",
        "-Wall", "-Wno-unknown-pragmas", "-o", _LIB + ".tmp", _SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("integrator", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
        ("batch", ctypes.c_int64), ("h", ctypes.c_double), ("alpha", ctypes.c_double),
        ("gamma", ctypes.c_double), ("gnl", ctypes.c_double), ("trap", ctypes.c_double * 3),
        ("sigma", ctypes.c_double), ("seed", ctypes.c_uint64), ("id_base", ctypes.c_uint32),
        ("noise_substeps", ctypes.c_uint32), ("Vgrid", ctypes.c_void_p),
        ("sigma_V", ctypes.c_double), ("convK", ctypes.c_void_p),
        ("basis", ctypes.c_int32), ("pad0", ctypes.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Problem)
        vp = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.ora_dft.argtypes = [vp, vp, i64, ctypes.c_int]
        lib.ora_fft.argtypes = [vp, i64, ctypes.c_int]
        lib.ora_philox4x32_10.argtypes = [vp, vp, vp]
        lib.ora_philox_batch.argtypes = [vp, i64, ctypes.c_uint64, vp]
        lib.ora_noise.argtypes = [P, i64, vp]
        lib.ora_step.argtypes = [P, vp, i64]
        lib.ora_step.restype = ctypes.c_int
        lib.ora_step_dense.argtypes = [P, vp, i64]
        lib.ora_step_dense.restype = ctypes.c_int
        lib.ora_run.argtypes = [P, vp, i64, i64, i64, vp, vp, i64]
        lib.ora_run.restype = ctypes.c_int
        lib.ora_diag.argtypes = [P, vp, vp]
        lib.ora_overlap.argtypes = [P, vp, vp, vp]
        lib.ora_moments.argtypes = [P, vp, vp, vp]
        lib.ora_tangent.argtypes = [P, vp, vp, vp, i64, i64]
        lib.ora_tangent.restype = ctypes.c_int
        lib.ora_adjoint.argtypes = [P, vp, i64, i64, i64, vp, vp, vp]
        lib.ora_adjoint.restype = ctypes.c_int
        lib.ora_apply_D.argtypes = [P, vp, ctypes.c_int, ctypes.c_int]
        lib.ora_apply_D.restype = ctypes.c_int
        lib.ora_fft_nd.argtypes = [P, vp, ctypes.c_int]
        lib.ora_fft_nd.restype = ctypes.c_int
        lib.ora_threads.restype = ctypes.c_int
        lib.ora_vnoise.argtypes = [P, i64, vp]
        lib.ora_conv_potential.argtypes = [P, vp, vp]
        lib.ora_conv_potential.restype = ctypes.c_int
        lib.ora_ck_tableau.argtypes = [vp]
        lib.ora_ck_step.argtypes = [P, vp, ctypes.c_double, vp, vp, ctypes.c_int]
        lib.ora_ck_step.restype = ctypes.c_int
        lib.ora_ark45.argtypes = [P, vp, ctypes.c_double, ctypes.c_double, i64, vp, vp, vp, i64, ctypes.c_int]
        lib.ora_ark45.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Problem:
    """Parameters of one group of same-shape instances (all FP64).

    ``n`` lists points per axis with axis 0 (x) contiguous in memory; the PDE is
    d psi/dt = L psi + G(psi) with L(k) = -i alpha |k|^2 - gamma and
    G = -i (V + gnl |psi|^2) psi + sigma xi (Sec. 3.6 eqs. (5)-(8); Sec. 3.5 noise).
    """

    n: Sequence[int]
    lo: Sequence[float]
    hi: Sequence[float]
    h: float
    batch: int = 1
    alpha: float = 0.5
    gamma: float = 0.0
    gnl: float = 0.0
    trap: Sequence[float] = (0.0, 0.0, 0.0)
    sigma: float = 0.0
    seed: int = 0
    id_base: int = 0
    Vgrid: Optional[np.ndarray] = None  # [batch][M] float64
    integrator: int = 0        # 0: RK4IP; 1: semi-implicit in the interaction picture
    noise_substeps: int = 1    # noise of a step = normalised sum of this many finer draws
    sigma_V: float = 0.0       # real Wiener noise in the potential (reading R10)
    convK: Optional[np.ndarray] = None  # [n] kernel of the non-local potential (R11), 1D
    basis: int = 0             # 0 Fourier; 1 cosine, 2 sine on a half domain (R12), 1D
    _keep: list = field(default_factory=list, repr=False)

    @property
    def ndim(self) -> int:
        return len(self.n)

    @property
    def M(self) -> int:
        return int(np.prod(self.n))

    @property
    def shape(self):
        """numpy shape of the field: (batch, [nz], [ny], nx)."""
        return (self.batch,) + tuple(int(v) for v in reversed(self.n))

    def _c(self) -> _Problem:
        p = _Problem()
        p.ndim = self.ndim
        for a in range(3):
            p.n[a] = int(self.n[a]) if a < self.ndim else 1
            p.lo[a] = float(self.lo[a]) if a < self.ndim else 0.0
            p.hi[a] = float(self.hi[a]) if a < self.ndim else 1.0
            p.trap[a] = float(self.trap[a]) if a < len(self.trap) else 0.0
        p.batch = int(self.batch)
        p.h, p.alpha, p.gamma, p.gnl = float(self.h), float(self.alpha), float(self.gamma), float(self.gnl)
        p.sigma = float(self.sigma)
        p.seed = int(self.seed) & 0xFFFFFFFFFFFFFFFF
        p.id_base = int(self.id_base) & 0xFFFFFFFF
        p.integrator = int(self.integrator)
        p.noise_substeps = int(self.noise_substeps)
        self._keep = []
        if self.Vgrid is not None:
            vg = np.ascontiguousarray(self.Vgrid, dtype=np.float64).reshape(self.batch, self.M)
            self._keep.append(vg)
            p.Vgrid = vg.ctypes.data
        else:
            p.Vgrid = None
        p.sigma_V = float(self.sigma_V)
        p.basis = int(self.basis)
        if self.convK is not None:
            ck = np.ascontiguousarray(self.convK, dtype=np.float64).reshape(-1)
            if ck.size != int(self.n[0]):
                raise ValueError("convK needs one value per lattice offset")
            self._keep.append(ck)
            p.convK = ck.ctypes.data
        else:
            p.convK = None
        return p


def _cfield(p: Problem, psi) -> np.ndarray:
    a = np.ascontiguousarray(psi, dtype=np.complex128)
    if a.size != p.batch * p.M:
        raise ValueError(f"field has {a.size} values, expected {p.batch * p.M}")
    return a.reshape(p.shape).copy()


def threads() -> int:
    """OpenMP threads the oracle runs with."""
    return int(_load().ora_threads())


def dft(x, sign: int = -1) -> np.ndarray:
    """Brute-force DFT, unnormalised (Sec. 3.2 transform written as a sum)."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.empty_like(x)
    _load().ora_dft(x.ctypes.data, out.ctypes.data, x.size, sign)
    return out


def fft(x, sign: int = -1) -> np.ndarray:
    """Oracle radix-2 FFT of a power-of-two vector, unnormalised."""
    x = np.ascontiguousarray(x, dtype=np.complex128).copy()
    _load().ora_fft(x.ctypes.data, x.size, sign)
    return x


def fft_nd(p: Problem, psi, sign: int = -1) -> np.ndarray:
    """Unnormalised multi-dimensional transform of every instance."""
    f = _cfield(p, psi)
    pc = p._c()
    if _load().ora_fft_nd(ctypes.byref(pc), f.ctypes.data, sign):
        raise ValueError("invalid problem")
    return f


def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block function (Salmon et al. SC'11) on one counter/key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    _load().ora_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def philox_batch(ctr, seed: int) -> np.ndarray:
    """Philox words for a [count][4] array of counters under key (seed lo, seed hi)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(c)
    _load().ora_philox_batch(c.ctypes.data, c.shape[0], int(seed) & 0xFFFFFFFFFFFFFFFF, out.ctypes.data)
    return out


def noise(p: Problem, step: int) -> np.ndarray:
    """The noise field xi of every instance at a step (E|xi|^2 = 1/(h dV))."""
    out = np.empty(p.shape, dtype=np.complex128)
    pc = p._c()
    _load().ora_noise(ctypes.byref(pc), int(step), out.ctypes.data)
    return out


def vnoise(p: Problem, step: int) -> np.ndarray:
    """The real noise eta of the potential at a step, [batch][M] (E eta^2 = 1/(h dV))."""
    out = np.empty((p.batch, p.M), dtype=np.float64)
    pc = p._c()
    _load().ora_vnoise(ctypes.byref(pc), int(step), out.ctypes.data)
    return out


def conv_potential(p: Problem, psi) -> np.ndarray:
    """The non-local potential V_c of every instance (reading R11), [batch][n]."""
    f = _cfield(p, psi)
    out = np.empty((p.batch, p.M), dtype=np.float64)
    pc = p._c()
    if _load().ora_conv_potential(ctypes.byref(pc), f.ctypes.data, out.ctypes.data):
        raise ValueError("invalid problem")
    return out


def step(p: Problem, psi, step_index: int = 0, dense: bool = False) -> np.ndarray:
    """One RK4IP step of every instance; returns the new field."""
    f = _cfield(p, psi)
    pc = p._c()
    fn = _load().ora_step_dense if dense else _load().ora_step
    if fn(ctypes.byref(pc), f.ctypes.data, int(step_index)):
        raise ValueError("invalid problem")
    return f


def run(p: Problem, psi, nsteps: int, step0: int = 0, sample_every: int = 0, ckpt_every: int = 0):
    """Advance nsteps steps. Returns (psi, diag or None, ckpt or None).

    diag[s][b] = (N, E_kin, E_pot, E_int) at relative steps 0, s, 2s, ... <= nsteps;
    ckpt[c] = state at relative steps 0, M, 2M, ... < nsteps.
    """
    f = _cfield(p, psi)
    pc = p._c()
    diag = None
    if sample_every > 0:
        diag = np.zeros((nsteps // sample_every + 1, p.batch, 4), dtype=np.float64)
    ckpt = None
    if ckpt_every > 0:
        ckpt = np.zeros(((nsteps + ckpt_every - 1) // ckpt_every,) + p.shape, dtype=np.complex128)
    rc = _load().ora_run(
        ctypes.byref(pc), f.ctypes.data, int(step0), int(nsteps), int(sample_every),
        diag.ctypes.data if diag is not None else None, int(0) if ckpt is None else ckpt.ctypes.data,
        int(ckpt_every),
    )
    if rc:
        raise ValueError("invalid problem")
    return f, diag, ckpt


def ck_tableau():
    """The Cash-Karp pair the adaptive integrator uses: (c[6], a[6][5], b[6], b*[6])."""
    out = np.empty(48, dtype=np.float64)
    _load().ora_ck_tableau(out.ctypes.data)
    return out[:6], out[6:36].reshape(6, 5), out[36:42], out[42:48]


def ck_step(p: Problem, psi, h: float, ip: bool = True):
    """One Cash-Karp step of size h of every instance (Sec. 3.5's adaptive RK45 in the
    interaction picture, reading R8; ip=False: the explicit comparison method of Sec. 3.6).
    Returns (fifth-order result, error estimate[batch])."""
    f = _cfield(p, psi)
    out = np.empty_like(f)
    err = np.empty(p.batch, dtype=np.float64)
    pc = p._c()
    if _load().ora_ck_step(ctypes.byref(pc), f.ctypes.data, float(h), out.ctypes.data, err.ctypes.data, int(bool(ip))):
        raise ValueError("invalid problem")
    return out, err


def ark45(p: Problem, psi, t_span: float, tol: float, h0, max_attempts: int = 1 << 20, log_cap: int = 0,
          ip: bool = True):
    """Adaptive Cash-Karp integration of every instance over [0, t_span] (readings R8, R9),
    each instance with its own step. h0: first trial step (scalar or [batch]).
    Returns (psi, h_next[batch], stats[batch][2] = (accepted, rejected), h_log or None,
    done) with h_log[b][i] the i-th accepted step of instance b (log_cap entries)."""
    f = _cfield(p, psi)
    h = np.ascontiguousarray(np.broadcast_to(np.asarray(h0, dtype=np.float64), (p.batch,))).copy()
    stats = np.zeros((p.batch, 2), dtype=np.int64)
    log = np.full((p.batch, log_cap), np.nan) if log_cap > 0 else None
    pc = p._c()
    rc = _load().ora_ark45(ctypes.byref(pc), f.ctypes.data, float(t_span), float(tol), int(max_attempts),
                           h.ctypes.data, stats.ctypes.data, None if log is None else log.ctypes.data,
                           int(log_cap), int(bool(ip)))
    if rc < 0:
        raise ValueError("invalid problem")
    return f, h, stats, log, rc == 0


def diag(p: Problem, psi) -> np.ndarray:
    """[batch][4] = (N, E_kin, E_pot, E_int) in FP64 (Sec. 3.4 quadrature)."""
    f = _cfield(p, psi)
    out = np.zeros((p.batch, 4), dtype=np.float64)
    pc = p._c()
    _load().ora_diag(ctypes.byref(pc), f.ctypes.data, out.ctypes.data)
    return out


def overlap(p: Problem, phi, psi) -> np.ndarray:
    """c_b = dV sum conj(phi) psi_b for one target phi shared by all instances."""
    f = _cfield(p, psi)
    t = np.ascontiguousarray(phi, dtype=np.complex128).reshape(-1)
    if t.size != p.M:
        raise ValueError("target has the wrong size")
    out = np.zeros(p.batch, dtype=np.complex128)
    pc = p._c()
    _load().ora_overlap(ctypes.byref(pc), t.ctypes.data, f.ctypes.data, out.ctypes.data)
    return out


def moments(p: Problem, psi):
    """Per-point mean of |psi|^2 over instances and its (P-1) sample variance."""
    f = _cfield(p, psi)
    mean = np.zeros(p.M, dtype=np.float64)
    var = np.zeros(p.M, dtype=np.float64)
    pc = p._c()
    _load().ora_moments(ctypes.byref(pc), f.ctypes.data, mean.ctypes.data, var.ctypes.data)
    return mean.reshape(p.shape[1:]), var.reshape(p.shape[1:])


def apply_D(p: Problem, psi, dense: bool = False, adjoint: bool = False) -> np.ndarray:
    """D = e^{L h/2} (or its transpose D^T = e^{conj(L) h/2}) applied to every instance."""
    f = _cfield(p, psi)
    pc = p._c()
    if _load().ora_apply_D(ctypes.byref(pc), f.ctypes.data, int(dense), int(adjoint)):
        raise ValueError("invalid problem")
    return f


def tangent(p: Problem, psi, dpsi, dV=None, nsteps: int = 1, step0: int = 0):
    """Tangent-linear model: returns (psi_S, dpsi_S) for a perturbation (dpsi, dV)."""
    f = _cfield(p, psi)
    d = _cfield(p, dpsi)
    dv = None
    if dV is not None:
        dv = np.ascontiguousarray(dV, dtype=np.float64).reshape(p.batch, p.M).copy()
    pc = p._c()
    if _load().ora_tangent(ctypes.byref(pc), f.ctypes.data, d.ctypes.data,
                           None if dv is None else dv.ctypes.data, int(step0), int(nsteps)):
        raise ValueError("invalid problem")
    return f, d


def adjoint(p: Problem, psi0, lamT, nsteps: int, ckpt_every: int, step0: int = 0, want_V: bool = True):
    """Discrete adjoint: gradients (d/dRe + i d/dIm) w.r.t. psi0 and the potential grid
    of a loss whose adjoint at the final state is lamT."""
    f = _cfield(p, psi0)
    lam = _cfield(p, lamT)
    g = np.zeros(p.shape, dtype=np.complex128)
    gV = np.zeros(p.shape, dtype=np.float64) if want_V else None
    pc = p._c()
    rc = _load().ora_adjoint(ctypes.byref(pc), f.ctypes.data, int(step0), int(nsteps), int(ckpt_every),
                             lam.ctypes.data, g.ctypes.data, None if gV is None else gV.ctypes.data)
    if rc:
        raise ValueError("invalid problem")
    return g, gV
