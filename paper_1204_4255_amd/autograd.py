"""torch.autograd wrapper of the RK4IP run and its hand-written discrete adjoint.

``RK4IPSolver`` owns a plan whose groups read their potential grids from a solver-owned
device buffer. ``solver(psi0, V)`` copies V into that buffer, runs ``nsteps`` steps on the
GPU keeping a checkpoint every ``ckpt_every`` steps, and returns psi(T). Its backward
calls ``rk4ip_adjoint``: each checkpoint segment is recomputed and walked backwards, so
memory is O(nsteps/ckpt_every + ckpt_every) fields. Gradients follow PyTorch's complex
convention (d/dRe + i d/dIm) for psi0 and are real for V.
"""
from __future__ import annotations

from typing import List, Sequence

import torch

from . import rk4ip


class _RK4IPFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi0, V, solver):
        solver._load_V(V)
        psi = psi0.detach().contiguous().clone()
        _, ckpt = solver.plan.run(psi, solver.nsteps, step0=solver.step0, ckpt_every=solver.ckpt_every)
        ctx.solver = solver
        ctx.ckpt = ckpt
        # the plan reads V from the solver's one buffer, which a later call overwrites:
        # keep this call's potential for the backward recompute
        ctx.V = solver.V.clone()
        return psi

    @staticmethod
    def backward(ctx, grad_out):
        s = ctx.solver
        # the recompute and the adjoint must see the potential of the forward call this
        # backward belongs to (copy and adjoint run in order on the current stream)
        with torch.no_grad():
            s.V.copy_(ctx.V)
        g, gV = s.plan.adjoint(ctx.ckpt, s.nsteps, s.ckpt_every, grad_out.contiguous().to(torch.complex64),
                               step0=s.step0, want_V=True)
        return g, gV, None


class RK4IPSolver:
    """Differentiable RK4IP run over one or more groups with learnable potential grids.

    probs: rk4ip_problem list (their V_grid pointers are replaced by the solver's buffer);
    the potential V passed at call time is a float32 tensor of all instances concatenated
    ([total points]).
    """

    def __init__(self, probs: Sequence[rk4ip.rk4ip_problem], nsteps: int, ckpt_every: int, step0: int = 0,
                 device: str = "cuda", flags: int = 0):
        import numpy as np

        self.nsteps = int(nsteps)
        self.ckpt_every = int(ckpt_every)
        self.step0 = int(step0)
        total = sum(int(p.batch) * int(np.prod([p.n[a] for a in range(3)])) for p in probs)
        self.V = torch.zeros(total, dtype=torch.float32, device=device)
        own: List[rk4ip.rk4ip_problem] = []
        off = 0
        for p in probs:
            q = rk4ip.rk4ip_problem()
            ctypes_copy(q, p)
            M = int(p.batch) * int(np.prod([p.n[a] for a in range(3)]))
            q.V_grid = self.V.data_ptr() + 4 * off
            off += M
            own.append(q)
        self.plan = rk4ip.Plan(own, flags=flags, device=device)

    def _load_V(self, V):
        with torch.no_grad():
            self.V.copy_(V.detach().reshape(-1).to(torch.float32))

    def __call__(self, psi0, V):
        return _RK4IPFunction.apply(psi0, V, self)


def ctypes_copy(dst, src):
    import ctypes

    ctypes.memmove(ctypes.addressof(dst), ctypes.addressof(src), ctypes.sizeof(src))
