"""Properties of the GPU step that need no oracle: every instance of a batch evolves
exactly as it would alone (same noise id, bitwise), for RK4IP, the semi-implicit step and
the cosine basis, one or several steps per launch; and a global phase commutes with the
noise-free step to single precision."""
import numpy as np
import pytest

from gpu_helpers import log, quantised, rel
from paper_1204_4255_amd import rk4ip

pytestmark = pytest.mark.gpu

SI = rk4ip.RK4IP_FLAG_SEMI_IMPLICIT
FUSE = rk4ip.RK4IP_FLAG_FUSE_1D | rk4ip.RK4IP_FLAG_GRAPH


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    rk4ip.load()
    return t


def _dev(torch, a):
    return torch.tensor(np.asarray(a, dtype=np.complex64).reshape(-1), device="cuda")


@pytest.mark.parametrize("flags", [0, SI, FUSE, SI | FUSE])
@pytest.mark.parametrize("basis", [0, 1])
def test_each_instance_evolves_as_it_would_alone(torch, flags, basis):
    n, B, S = 256, 6, 40
    x = (np.arange(n) + (0.5 if basis else 0.0)) * 16.0 / n + (0.0 if basis else -8.0)
    shifts = np.linspace(-1.0, 1.0, B)[:, None] * (0 if basis else 1)
    f0 = quantised(np.pi ** -0.25 * np.exp(-(x[None] - shifts) ** 2 / 2) * np.exp(0.2j * x[None] * np.arange(1, B + 1)[:, None] / B))
    lo, hi = ((0.0,), (16.0,)) if basis else ((-8.0,), (8.0,))
    kw = dict(g_nl=2.0, trap=(1.0, 0, 0), gamma=0.05, sigma=0.01, seed=77, basis=basis)
    batch = rk4ip.Plan([rk4ip.make_problem((n,), lo, hi, 1e-3, batch=B, id_base=10, **kw)], flags=flags)
    d = _dev(torch, f0)
    batch.run(d, S, step0=5)
    got = d.cpu().numpy().reshape(B, n)
    for b in range(B):
        one = rk4ip.Plan([rk4ip.make_problem((n,), lo, hi, 1e-3, batch=1, id_base=10 + b, **kw)], flags=flags)
        e = _dev(torch, f0[b])
        one.run(e, S, step0=5)
        assert np.array_equal(e.cpu().numpy(), got[b]), b


@pytest.mark.parametrize("n,flags", [((256,), 0), ((64, 32), 0), ((32, 16, 8), 0), ((64, 32), SI), ((256,), SI)])
def test_a_global_phase_commutes_with_the_step(torch, n, flags):
    nd = len(n)
    p = rk4ip.make_problem(n, (-4.0,) * nd, (4.0,) * nd, 1e-3, batch=2, g_nl=3.0, trap=(1.0, 1.0, 1.0), gamma=0.05)
    plan = rk4ip.Plan([p], flags=flags)
    rng = np.random.Generator(np.random.PCG64(3))
    shape = (2,) + tuple(reversed(n))
    f = quantised(rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
    c = np.exp(0.7j)
    a = _dev(torch, f)
    b = _dev(torch, c * f)
    plan.run(a, 20)
    plan.run(b, 20)
    ha = a.cpu().numpy().astype(np.complex128)
    hb = b.cpu().numpy().astype(np.complex128)
    err = rel(hb, c * ha)
    log(f"  n={n} flags={flags}: phase covariance {err:.2e}")
    assert err < 2e-6
