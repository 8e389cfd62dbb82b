"""GPU parity of the hand-written adjoint (rk4ip_adjoint / RK4IPSolver) against the
oracle's discrete adjoint, plus a loose central-difference check of the GPU gradients."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, oprob, quantised, random_field, rel
from paper_1204_4255_amd import rk4ip
from paper_1204_4255_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available()
    rk4ip.load()
    return t


def _groups(shapes, seed=3, sigma=0.01, gamma=0.05):
    rng = np.random.Generator(np.random.PCG64(seed))
    gs, base = [], 0
    for n, b in shapes:
        nd = len(n)
        g = W.Group(n=n, lo=(-5.0,) * nd, hi=(5.0,) * nd, batch=b, gnl=4.0, trap=(1.0, 0.8, 1.2), gamma=gamma,
                    sigma=sigma, seed=seed, id_base=base)
        g.Vgrid = (0.05 * rng.standard_normal((b, g.M))).astype(np.float32)
        gs.append(g)
        base += b
    return gs


def _run_case(torch, shapes, nsteps, M, step0=5):
    from paper_1204_4255_amd.autograd import RK4IPSolver

    gs = _groups(shapes)
    h = 2e-3
    fields = [quantised(random_field(g, 7 + i)) for i, g in enumerate(gs)]
    w = W.Workload("adj", gs, h, nsteps, fields)
    probs, _ = rk4ip.problems_from_workload(w)
    solver = RK4IPSolver(probs, nsteps, M, step0=step0)
    psi0 = rk4ip.field_to_device(w).requires_grad_(True)
    V = torch.tensor(np.concatenate([g.Vgrid.reshape(-1) for g in gs]), device="cuda", requires_grad=True)
    rng = np.random.Generator(np.random.PCG64(11))
    tot = psi0.numel()
    lamT_np = (rng.standard_normal(tot) + 1j * rng.standard_normal(tot)).astype(np.complex64)
    lamT = torch.tensor(lamT_np, device="cuda")
    out = solver(psi0, V)
    # loss whose adjoint at psi_T is lamT: Re <lamT, psi_T>
    loss = torch.sum((torch.conj(lamT) * out).real)
    loss.backward()
    g_psi = psi0.grad.cpu().numpy().astype(np.complex128)
    g_V = V.grad.cpu().numpy().astype(np.float64)
    off = 0
    for gr, f in zip(gs, fields):
        n = gr.batch * gr.M
        ref_g, ref_V = oracle.adjoint(oprob(gr, h), f, lamT_np[off:off + n].astype(np.complex128).reshape(gr.shape),
                                      nsteps=nsteps, ckpt_every=M, step0=step0)
        e1 = rel(g_psi[off:off + n], ref_g)
        e2 = rel(g_V[off:off + n], ref_V)
        log(f"  group n={gr.n} x{gr.batch}: grad_psi0 rel {e1:.2e}, grad_V rel {e2:.2e}")
        assert e1 < 1e-5 and e2 < 1e-5, (e1, e2)
        off += n
    return solver


@pytest.mark.parametrize("shapes,nsteps,M", [
    ([((64,), 3), ((256,), 2)], 7, 3),
    ([((16, 16), 3), ((32, 32), 2)], 7, 3),
    ([((16, 8, 8), 2)], 5, 2),
    ([((64, 32), 1)], 6, 6),
])
def test_adjoint_matches_oracle(torch, shapes, nsteps, M):
    log(f"adjoint shapes={shapes} steps={nsteps} ckpt={M}")
    _run_case(torch, shapes, nsteps, M)


def test_adjoint2d_workload_shapes(torch):
    """The uneven 32 x 128^2 + 32 x 256^2 batch at full shape, 20 steps, checkpoint 5."""
    from paper_1204_4255_amd.autograd import RK4IPSolver

    nsteps, M = 20, 5
    log(f"adjoint2d full shapes, {nsteps} steps, ckpt {M}")
    w = W.adjoint2d(nsteps=nsteps, ckpt_every=M)
    probs, _ = rk4ip.problems_from_workload(w)
    solver = RK4IPSolver(probs, nsteps, M)
    psi0 = rk4ip.field_to_device(w).requires_grad_(True)
    V = torch.tensor(np.concatenate([g.Vgrid.reshape(-1) for g in w.groups]).astype(np.float32), device="cuda",
                     requires_grad=True)
    out = solver(psi0, V)
    # loss = sum_b 1 - |<phi|psi_b(T)>|^2 evaluated with torch ops on the device
    loss = 0
    off = 0
    targets = []
    for g, phi in zip(w.groups, w.target):
        n = g.batch * g.M
        t = torch.tensor(phi.astype(np.complex64).reshape(-1), device="cuda")
        targets.append(t)
        c = g.dV * torch.sum(torch.conj(t)[None] * out[off:off + n].reshape(g.batch, -1), dim=1)
        loss = loss + torch.sum(1 - torch.abs(c) ** 2)
        off += n
    loss.backward()
    g_psi = psi0.grad.cpu().numpy().astype(np.complex128)
    g_V = V.grad.cpu().numpy().astype(np.float64)
    outs = out.detach().cpu().numpy().astype(np.complex128)
    off = 0
    for g, phi, f in zip(w.groups, w.target, w.psi0):
        n = g.batch * g.M
        f = quantised(f)
        ref_T, _, _ = oracle.run(oprob(g, w.h), f, nsteps)
        c = oracle.overlap(oprob(g, w.h), phi, ref_T)
        lamT = -2 * g.dV * c[:, None, None] * phi[None]
        ref_g, ref_V = oracle.adjoint(oprob(g, w.h), f, lamT, nsteps=nsteps, ckpt_every=M)
        e0 = rel(outs[off:off + n], ref_T)
        e1 = rel(g_psi[off:off + n], ref_g)
        e2 = rel(g_V[off:off + n], ref_V)
        log(f"  n={g.n} x{g.batch}: psi_T rel {e0:.2e}, grad_psi0 rel {e1:.2e}, grad_V rel {e2:.2e}")
        assert e0 < 1e-5 and e1 < 1e-5 and e2 < 1e-5
        off += n


def test_gpu_gradient_central_difference(torch):
    """Central differences of the GPU forward run (FP32 loss) along a random direction."""
    from paper_1204_4255_amd.autograd import RK4IPSolver

    gs = _groups([((32, 32), 2)], sigma=0.0, gamma=0.0)
    nsteps, M, h = 10, 4, 2e-3
    fields = [quantised(random_field(g, 3)) for g in gs]
    w = W.Workload("fd", gs, h, nsteps, fields)
    probs, _ = rk4ip.problems_from_workload(w)
    solver = RK4IPSolver(probs, nsteps, M)
    g0 = gs[0]
    X, Y = g0.mesh()
    phi = torch.tensor((np.pi ** -0.5 * np.exp(-((X - 0.5) ** 2 + Y ** 2) / 2)).astype(np.complex64).reshape(-1),
                       device="cuda")

    def loss_of(psi0, V):
        out = solver(psi0, V).reshape(g0.batch, -1)
        c = g0.dV * torch.sum(torch.conj(phi)[None] * out.to(torch.complex128), dim=1)
        return torch.sum(1 - torch.abs(c) ** 2)

    psi0 = rk4ip.field_to_device(w).requires_grad_(True)
    V = torch.tensor(g0.Vgrid.reshape(-1), device="cuda", requires_grad=True)
    loss_of(psi0, V).backward()
    rng = np.random.Generator(np.random.PCG64(5))
    d = torch.tensor((rng.standard_normal(psi0.numel()) + 1j * rng.standard_normal(psi0.numel())).astype(np.complex64),
                     device="cuda")
    d = d * (torch.linalg.vector_norm(psi0.detach()) / torch.linalg.vector_norm(d))   # same size as psi0
    # the loss moves little with V over T = 0.02, so take a direction large enough that
    # the difference stands well above the FP32 rounding of the forward runs (~1e-6 of
    # the loss)
    dv = torch.tensor(25.0 * rng.standard_normal(V.numel()).astype(np.float32), device="cuda")
    eps = 1e-2  # FP32 forward: larger steps keep the difference above rounding
    with torch.no_grad():
        lp = loss_of(psi0 + eps * d, V).item()
        lm = loss_of(psi0 - eps * d, V).item()
        fd = (lp - lm) / (2 * eps)
        an = float(torch.sum((torch.conj(psi0.grad) * d).real))
        lpv = loss_of(psi0, V + eps * dv).item()
        lmv = loss_of(psi0, V - eps * dv).item()
        fdv = (lpv - lmv) / (2 * eps)
        anv = float(torch.sum(V.grad * dv))
    log(f"  FD psi0: {fd:.6e} vs adjoint {an:.6e}; FD V: {fdv:.6e} vs adjoint {anv:.6e}")
    assert abs(fd - an) <= 2e-3 * abs(an) + 1e-6
    assert abs(fdv - anv) <= 2e-3 * abs(anv) + 1e-6


def test_solver_called_twice_before_backward(torch):
    """The plan reads V from the solver's one buffer. Two calls with different V before one
    backward: the gradient through the first call must equal that of the first call alone
    (each call keeps its own potential for the backward recompute)."""
    from paper_1204_4255_amd.autograd import RK4IPSolver

    gs = _groups([((32, 16), 2)], sigma=0.01, gamma=0.02)
    nsteps, M, h = 8, 3, 2e-3
    fields = [quantised(random_field(g, 5)) for g in gs]
    w = W.Workload("reent", gs, h, nsteps, fields)
    probs, _ = rk4ip.problems_from_workload(w)
    solver = RK4IPSolver(probs, nsteps, M)
    base = rk4ip.field_to_device(w)
    V1 = torch.tensor(gs[0].Vgrid.reshape(-1), device="cuda")
    V2 = V1 * 3.0 + 0.5
    rng = np.random.Generator(np.random.PCG64(2))
    lam = torch.tensor((rng.standard_normal(base.numel()) + 1j * rng.standard_normal(base.numel()))
                       .astype(np.complex64), device="cuda")

    def grads(second):
        p = base.clone().requires_grad_(True)
        V = V1.clone().requires_grad_(True)
        out1 = solver(p, V)
        if second:
            p2 = base.clone().requires_grad_(True)
            out2 = solver(p2, V2.clone().requires_grad_(True))
            del out2
        torch.sum((torch.conj(lam) * out1).real).backward()
        return p.grad.clone(), V.grad.clone()

    g_alone, gv_alone = grads(False)
    g_both, gv_both = grads(True)
    log(f"  grad_psi0 diff {float((g_both - g_alone).abs().max()):.3e}, grad_V diff "
        f"{float((gv_both - gv_alone).abs().max()):.3e}")
    assert torch.equal(g_both, g_alone) and torch.equal(gv_both, gv_alone)


def test_adjoint_graph_segments_equal_eager(torch):
    """With RK4IP_FLAG_GRAPH the forward run and each whole checkpoint segment of the adjoint
    (recompute into the segment's slots, backward walk) replay hipGraphs: the gradients equal
    the eager ones bitwise, on two calls in a row (the second replays the graphs recorded on
    the solver's kept workspace), with a last partial segment run eagerly."""
    from paper_1204_4255_amd.autograd import RK4IPSolver

    gs = _groups([((64,), 3), ((16, 16), 2), ((16, 8, 8), 1)])
    nsteps, M, h = 11, 4, 2e-3
    fields = [quantised(random_field(g, 17 + i)) for i, g in enumerate(gs)]
    w = W.Workload("adjg", gs, h, nsteps, fields)
    probs, _ = rk4ip.problems_from_workload(w)
    V0 = torch.tensor(np.concatenate([g.Vgrid.reshape(-1) for g in gs]), device="cuda")
    rng = np.random.Generator(np.random.PCG64(3))
    base = rk4ip.field_to_device(w)
    lam = torch.tensor((rng.standard_normal(base.numel()) + 1j * rng.standard_normal(base.numel()))
                       .astype(np.complex64), device="cuda")

    def grads(solver, scale):
        p = (base * scale).requires_grad_(True)
        V = V0.clone().requires_grad_(True)
        torch.sum((torch.conj(lam) * solver(p, V)).real).backward()
        return p.grad.clone(), V.grad.clone()

    eager = RK4IPSolver(probs, nsteps, M, step0=3)
    graph = RK4IPSolver(probs, nsteps, M, step0=3, flags=rk4ip.RK4IP_FLAG_GRAPH)
    for scale in (1.0, 0.8):
        ge, gve = grads(eager, scale)
        gg, gvg = grads(graph, scale)
        log(f"  scale {scale}: grad_psi0 max diff {float((gg - ge).abs().max()):.3e}, "
            f"grad_V max diff {float((gvg - gve).abs().max()):.3e}")
        assert torch.equal(gg, ge) and torch.equal(gvg, gve)
