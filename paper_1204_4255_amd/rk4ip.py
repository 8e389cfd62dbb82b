"""ctypes binding of the HIP library ``librk4ip.so`` (C ABI in ``include/rk4ip.h``).

Argument marshalling only: every step of the RK4IP path runs in the library's gfx950
kernels. PyTorch supplies device memory (workspaces, fields) and the current stream.
Importing this module does not need a GPU; loading the library does need the built
``librk4ip.so`` and raises if it is missing (there is no CPU fallback).

Function names mirror the C entry points (``rk4ip_plan``, ``rk4ip_step``, ``rk4ip_run``,
``rk4ip_adjoint`` ...). ``Plan`` bundles a plan with the torch-owned workspace it uses.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librk4ip.so")

RK4IP_OK = 0
RK4IP_ERR_INVALID_ARG = -1
RK4IP_ERR_UNSUPPORTED_SHAPE = -2
RK4IP_ERR_WORKSPACE_TOO_SMALL = -3
RK4IP_ERR_HIP = -4
RK4IP_ERR_NONFINITE = -5
RK4IP_ERR_NOT_CAPTURABLE = -6
RK4IP_ERR_NO_DEVICE = -7

RK4IP_FLAG_GRAPH = 0x1
RK4IP_FLAG_AUTOTUNE = 0x2
RK4IP_FLAG_FUSE_1D = 0x4
RK4IP_FLAG_FP64_TRANSFORMS = 0x8
RK4IP_FLAG_SEMI_IMPLICIT = 0x10
RK4IP_FLAG_MERGE_GROUPS = 0x20
BASIS_FOURIER, BASIS_COSINE, BASIS_SINE = 0, 1, 2

# every symbol include/rk4ip.h declares
EXPORTS = [
    "rk4ip_workspace_bytes", "rk4ip_plan", "rk4ip_set_stream", "rk4ip_step", "rk4ip_run",
    "rk4ip_diagnostics", "rk4ip_overlap", "rk4ip_moments", "rk4ip_adjoint_workspace_bytes",
    "rk4ip_adjoint", "rk4ip_ark45", "rk4ip_status", "rk4ip_destroy", "rk4ip_strerror", "rk4ip_last_error",
    "rk4ip_schedule", "rk4ip_num_passes", "rk4ip_profile", "rk4ip_profile_read", "rk4ip_debug_philox", "rk4ip_debug_noise", "rk4ip_debug_fft",
    "rk4ip_debug_apply_D", "rk4ip_step_noalloc",
]


class Rk4ipError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class rk4ip_problem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("basis", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
        ("batch", ctypes.c_int64), ("dt", ctypes.c_double), ("alpha", ctypes.c_double),
        ("gamma", ctypes.c_double), ("g_nl", ctypes.c_double), ("trap", ctypes.c_double * 3),
        ("V_grid", ctypes.c_void_p), ("sigma", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("id_base", ctypes.c_uint32), ("noise_substeps", ctypes.c_uint32),
        ("sigma_V", ctypes.c_double), ("conv_K", ctypes.c_void_p),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Load librk4ip.so and declare the ABI. Raises if the library is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    vp, i64, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64
    P = ctypes.POINTER(rk4ip_problem)
    sig = {
        "rk4ip_workspace_bytes": (ctypes.c_size_t, [P, i32, u32]),
        "rk4ip_plan": (i32, [P, i32, vp, ctypes.c_size_t, vp, u32, ctypes.POINTER(vp)]),
        "rk4ip_set_stream": (i32, [vp, vp]),
        "rk4ip_step": (i32, [vp, vp, i64]),
        "rk4ip_run": (i32, [vp, vp, i64, i64, i64, vp, vp, i64]),
        "rk4ip_diagnostics": (i32, [vp, vp, vp]),
        "rk4ip_overlap": (i32, [vp, i32, vp, vp, vp]),
        "rk4ip_moments": (i32, [vp, i32, vp, vp, vp]),
        "rk4ip_adjoint_workspace_bytes": (ctypes.c_size_t, [vp, i64]),
        "rk4ip_adjoint": (i32, [vp, vp, i64, i64, i64, vp, vp, vp, vp, ctypes.c_size_t]),
        "rk4ip_ark45": (i32, [vp, vp, ctypes.c_double, ctypes.c_double, i64, vp, vp, vp, i64, i32]),
        "rk4ip_status": (i32, [vp]),
        "rk4ip_destroy": (i32, [vp]),
        "rk4ip_strerror": (ctypes.c_char_p, [i32]),
        "rk4ip_last_error": (ctypes.c_char_p, [vp]),
        "rk4ip_schedule": (ctypes.c_char_p, [vp, i32, i32]),
        "rk4ip_num_passes": (i32, [vp, i32]),
        "rk4ip_profile": (i32, [vp, i32]),
        "rk4ip_profile_read": (i32, [vp, i32, i32, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]),
        "rk4ip_debug_philox": (i32, [u64, vp, i64, vp, vp]),
        "rk4ip_debug_noise": (i32, [vp, i32, i64, vp]),
        "rk4ip_debug_fft": (i32, [vp, i32, i32, vp, vp, i64, i32]),
        "rk4ip_debug_apply_D": (i32, [vp, vp, i32]),
        "rk4ip_step_noalloc": (i32, [P, i32, vp, i64, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _buf(t, numel: int, dtype, what: str, optional: bool = False) -> Optional[int]:
    """Device pointer of a contiguous tensor of exactly `numel` elements of `dtype`. The C
    ABI sees only the pointer, so a buffer of the wrong size or type is refused here
    before any kernel could read or write past its end."""
    if t is None:
        if optional:
            return None
        raise Rk4ipError(RK4IP_ERR_INVALID_ARG, f"{what}: missing")
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise Rk4ipError(RK4IP_ERR_INVALID_ARG,
                         f"{what}: need a contiguous device {dtype} tensor of {numel} elements, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device}{'' if t.is_contiguous() else ' (strided)'}")
    return int(t.data_ptr())


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(status: int, plan_handle=None, what: str = "rk4ip call"):
    if status != RK4IP_OK:
        lib = load()
        msg = lib.rk4ip_strerror(status).decode()
        if plan_handle:
            extra = lib.rk4ip_last_error(plan_handle).decode()
            if extra:
                msg += ": " + extra
        raise Rk4ipError(status, f"{what}: {msg}")


def make_problem(n: Sequence[int], lo: Sequence[float], hi: Sequence[float], dt: float, batch: int = 1,
                 alpha: float = 0.5, gamma: float = 0.0, g_nl: float = 0.0, trap: Sequence[float] = (0, 0, 0),
                 V_grid=None, sigma: float = 0.0, seed: int = 0, id_base: int = 0,
                 noise_substeps: int = 1, sigma_V: float = 0.0, conv_K=None, basis: int = 0) -> rk4ip_problem:
    """Fill an rk4ip_problem; V_grid is a device float32 tensor [batch][M] or None; conv_K
    a host float64 array [n] (kept alive on the returned struct until the plan is made)."""
    p = rk4ip_problem()
    nd = len(n)
    p.ndim = nd
    for a in range(3):
        p.n[a] = int(n[a]) if a < nd else 1
        p.lo[a] = float(lo[a]) if a < nd else 0.0
        p.hi[a] = float(hi[a]) if a < nd else 1.0
        p.trap[a] = float(trap[a]) if a < len(trap) else 0.0
    p.batch = int(batch)
    p.dt, p.alpha, p.gamma, p.g_nl = float(dt), float(alpha), float(gamma), float(g_nl)
    if V_grid is not None:
        import torch

        M = int(np.prod([p.n[a] for a in range(3)]))
        p.V_grid = _buf(V_grid, p.batch * M, torch.float32, "V_grid")
        p._V_grid = V_grid  # the struct holds the tensor alive with its pointer
    else:
        p.V_grid = None
    p.sigma = float(sigma)
    p.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    p.id_base = int(id_base) & 0xFFFFFFFF
    p.noise_substeps = int(noise_substeps)
    p.sigma_V = float(sigma_V)
    p.basis = int(basis)
    if conv_K is not None:
        ck = np.ascontiguousarray(conv_K, dtype=np.float64).reshape(-1)
        if ck.size != p.n[0]:
            raise Rk4ipError(RK4IP_ERR_INVALID_ARG, f"conv_K: need {p.n[0]} values, got {ck.size}")
        p._conv_K = ck
        p.conv_K = ck.ctypes.data
    else:
        p.conv_K = None
    return p


def problems_array(probs: List[rk4ip_problem]):
    arr = (rk4ip_problem * len(probs))(*probs)
    return arr


def rk4ip_workspace_bytes(probs: List[rk4ip_problem], flags: int = 0) -> int:
    arr = problems_array(probs)
    return int(load().rk4ip_workspace_bytes(arr, len(probs), flags))


def rk4ip_strerror(status: int) -> str:
    return load().rk4ip_strerror(status).decode()


def rk4ip_debug_philox(seed: int, ctr, out) -> None:
    """Philox4x32-10 of device uint32 counters [n][4] (torch int32 storage) into out."""
    import torch

    n = ctr.numel() // 4
    if ctr.numel() != 4 * n:
        raise Rk4ipError(RK4IP_ERR_INVALID_ARG, "ctr: need [n][4] words")
    cp = _buf(ctr, 4 * n, torch.int32, "ctr")
    op = _buf(out, 4 * n, torch.int32, "out")
    _check(load().rk4ip_debug_philox(int(seed) & 0xFFFFFFFFFFFFFFFF, cp, n, op, _stream()),
           what="rk4ip_debug_philox")


def step_noalloc(probs: List[rk4ip_problem], psi, step_index: int = 0):
    """rk4ip_step_noalloc: one step of every instance of `probs` in place on psi (device
    complex64, all points of all groups), without a plan or a workspace (the library's
    static device buffer holds the tables and work fields)."""
    import torch

    arr = problems_array(list(probs))
    points = sum(int(p.batch * p.n[0] * p.n[1] * p.n[2]) for p in probs)
    _check(load().rk4ip_step_noalloc(arr, len(probs), _buf(psi, points, torch.complex64, "psi"), int(step_index),
                                     _stream()), None, "rk4ip_step_noalloc")


class Plan:
    """A plan plus the torch-allocated workspace it lives in."""

    def __init__(self, probs: List[rk4ip_problem], flags: int = 0, device: str = "cuda"):
        import torch

        lib = load()
        self.probs = list(probs)
        self._arr = problems_array(self.probs)
        self.flags = flags
        nbytes = int(lib.rk4ip_workspace_bytes(self._arr, len(self.probs), flags))
        if nbytes == 0:
            raise Rk4ipError(RK4IP_ERR_INVALID_ARG, "rk4ip_workspace_bytes: invalid problem description")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._ws_ptr = aligned
        self.ws_bytes = nbytes
        h = ctypes.c_void_p()
        _check(lib.rk4ip_plan(self._arr, len(self.probs), ctypes.c_void_p(aligned), nbytes, _stream(), flags,
                              ctypes.byref(h)), what="rk4ip_plan")
        self.handle = h
        self.points = sum(int(p.batch) * int(np.prod([p.n[a] for a in range(3)])) for p in self.probs)
        self.ninst = sum(int(p.batch) for p in self.probs)

    # -- life cycle
    def destroy(self):
        if getattr(self, "handle", None):
            load().rk4ip_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def _group_points(self, group: int) -> int:
        if not 0 <= int(group) < len(self.probs):
            raise Rk4ipError(RK4IP_ERR_INVALID_ARG, f"group {group} out of range")
        p = self.probs[group]
        return int(p.n[0] * p.n[1] * p.n[2])

    def _psi(self, psi, what: str = "psi") -> int:
        import torch

        return _buf(psi, self.points, torch.complex64, what)

    def _sync_stream(self):
        load().rk4ip_set_stream(self.handle, _stream())

    # -- calls
    def step(self, psi, step_index: int = 0):
        self._sync_stream()
        _check(load().rk4ip_step(self.handle, self._psi(psi), int(step_index)), self.handle, "rk4ip_step")

    def run(self, psi, nsteps: int, step0: int = 0, sample_every: int = 0, ckpt_every: int = 0):
        """Returns (diag or None, ckpt or None) as device tensors."""
        import torch

        self._sync_stream()
        diag = None
        if sample_every > 0:
            diag = torch.zeros((nsteps // sample_every + 1, self.ninst, 4), dtype=torch.float64, device=psi.device)
        ckpt = None
        if ckpt_every > 0:
            nck = (nsteps + ckpt_every - 1) // ckpt_every
            ckpt = torch.empty((max(nck, 1), self.points), dtype=torch.complex64, device=psi.device)
        _check(load().rk4ip_run(self.handle, self._psi(psi), int(step0), int(nsteps), int(sample_every), _ptr(diag),
                                _ptr(ckpt), int(ckpt_every)), self.handle, "rk4ip_run")
        return diag, ckpt

    def diagnostics(self, psi):
        import torch

        self._sync_stream()
        out = torch.zeros((self.ninst, 4), dtype=torch.float64, device=psi.device)
        _check(load().rk4ip_diagnostics(self.handle, self._psi(psi), _ptr(out)), self.handle, "rk4ip_diagnostics")
        return out

    def overlap(self, group: int, phi, psi):
        import torch

        self._sync_stream()
        out = torch.zeros((int(self.probs[group].batch), 2), dtype=torch.float64, device=psi.device)
        _check(load().rk4ip_overlap(self.handle, group, _buf(phi, self._group_points(group), torch.complex64, "phi"),
                                    self._psi(psi), _ptr(out)), self.handle, "rk4ip_overlap")
        return out

    def moments(self, group: int, psi):
        import torch

        self._sync_stream()
        p = self.probs[group]
        M = int(p.n[0] * p.n[1] * p.n[2])
        mean = torch.zeros(M, dtype=torch.float64, device=psi.device)
        var = torch.zeros(M, dtype=torch.float64, device=psi.device)
        _check(load().rk4ip_moments(self.handle, group, self._psi(psi), _ptr(mean), _ptr(var)), self.handle,
               "rk4ip_moments")
        return mean, var

    def adjoint_workspace_bytes(self, ckpt_every: int) -> int:
        return int(load().rk4ip_adjoint_workspace_bytes(self.handle, int(ckpt_every)))

    def adjoint(self, ckpt, nsteps: int, ckpt_every: int, lambda_T, step0: int = 0, want_V: bool = True):
        """Returns (grad_psi0, grad_V or None) as device tensors."""
        import torch

        self._sync_stream()
        nb = self.adjoint_workspace_bytes(ckpt_every)
        # kept between calls (stream-ordered reuse), so that the segment graphs recorded on
        # it are replayed by later calls
        ws = getattr(self, "_keep_adj_ws", None)
        if ws is None or ws.numel() < nb + 256 or ws.device != lambda_T.device:
            ws = torch.empty(nb + 256, dtype=torch.uint8, device=lambda_T.device)
        aligned = (ws.data_ptr() + 255) // 256 * 256
        g = torch.empty_like(lambda_T)
        gV = torch.zeros(self.points, dtype=torch.float32, device=lambda_T.device) if want_V else None
        nck = max((int(nsteps) + int(ckpt_every) - 1) // max(int(ckpt_every), 1), 1)
        _check(load().rk4ip_adjoint(self.handle, _buf(ckpt, nck * self.points, torch.complex64, "ckpt"), int(step0),
                                    int(nsteps), int(ckpt_every), self._psi(lambda_T, "lambda_T"), _ptr(g), _ptr(gV),
                                    ctypes.c_void_p(aligned), nb),
               self.handle, "rk4ip_adjoint")
        self._keep_adj_ws = ws
        return g, gV

    def ark45(self, psi, t_span: float, tol: float, h, max_attempts: int = 1 << 20, log_cap: int = 0,
              explicit: bool = False):
        """Adaptive Cash-Karp integration over [0, t_span] (1D noise-free groups), in place on
        psi. h: device float64 [ninst], the first trial steps, updated to the next ones.
        Returns (stats [ninst][3] = accepted, rejected, reached; h_log [ninst][log_cap] or
        None) as device tensors."""
        import torch

        self._sync_stream()
        stats = torch.zeros((self.ninst, 3), dtype=torch.int64, device=psi.device)
        log = None
        if log_cap > 0:
            log = torch.full((self.ninst, log_cap), float("nan"), dtype=torch.float64, device=psi.device)
        _check(load().rk4ip_ark45(self.handle, self._psi(psi), float(t_span), float(tol), int(max_attempts),
                                  _buf(h, self.ninst, torch.float64, "h"),
                                  _ptr(stats), _ptr(log), int(log_cap), int(bool(explicit))), self.handle,
               "rk4ip_ark45")
        return stats, log

    def status(self) -> int:
        return int(load().rk4ip_status(self.handle))

    def schedule(self, group: int, pass_index: int) -> str:
        r = load().rk4ip_schedule(self.handle, group, pass_index)
        return r.decode() if r else ""

    def num_passes(self, group: int) -> int:
        return int(load().rk4ip_num_passes(self.handle, group))

    def profile(self, enable: bool):
        _check(load().rk4ip_profile(self.handle, int(bool(enable))), self.handle, "rk4ip_profile")

    def profile_read(self, group: int, pass_index: int):
        """(launch count, mean ms) of one pass since profiling was enabled."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(load().rk4ip_profile_read(self.handle, group, pass_index, ctypes.byref(n), ctypes.byref(ms)),
               self.handle, "rk4ip_profile_read")
        return int(n.value), float(ms.value)

    def noise(self, group: int, step: int):
        import torch

        self._sync_stream()
        p = self.probs[group]
        M = int(p.n[0] * p.n[1] * p.n[2])
        xi = torch.empty((int(p.batch), M), dtype=torch.complex64, device="cuda")
        _check(load().rk4ip_debug_noise(self.handle, group, int(step), _ptr(xi)), self.handle, "rk4ip_debug_noise")
        return xi

    def fft(self, group: int, axis: int, x, sign: int = -1):
        import torch

        self._sync_stream()
        self._group_points(group)
        n = int(self.probs[group].n[axis]) if 0 <= int(axis) < 3 else 0
        if n <= 0 or x.numel() % n:
            raise Rk4ipError(RK4IP_ERR_INVALID_ARG, f"fft: {x.numel()} elements are not whole lines of {n}")
        xp = _buf(x, x.numel(), torch.complex64, "x")
        out = torch.empty_like(x)
        _check(load().rk4ip_debug_fft(self.handle, group, axis, xp, _ptr(out), x.numel() // n, sign),
               self.handle, "rk4ip_debug_fft")
        return out

    def apply_D(self, psi, adjoint: bool = False):
        self._sync_stream()
        _check(load().rk4ip_debug_apply_D(self.handle, self._psi(psi), int(bool(adjoint))), self.handle,
               "rk4ip_debug_apply_D")


def problems_from_workload(w, device: str = "cuda", noise_substeps: int = 1):
    """rk4ip_problem list (and the device V grids it points to) for a workloads.Workload."""
    import torch

    probs, keep = [], []
    for g in w.groups:
        V = None
        if g.Vgrid is not None:
            V = torch.tensor(np.asarray(g.Vgrid, dtype=np.float32), device=device).contiguous()
            keep.append(V)
        probs.append(make_problem(g.n, g.lo, g.hi, w.h, batch=g.batch, alpha=g.alpha, gamma=g.gamma, g_nl=g.gnl,
                                  trap=g.trap, V_grid=V, sigma=g.sigma, seed=g.seed, id_base=g.id_base,
                                  noise_substeps=noise_substeps))
    return probs, keep


def field_to_device(w, device: str = "cuda"):
    """Concatenate the workload's initial fields into one complex64 device vector."""
    import torch

    flat = np.concatenate([np.asarray(p, dtype=np.complex64).reshape(-1) for p in w.psi0])
    return torch.tensor(flat, device=device)
