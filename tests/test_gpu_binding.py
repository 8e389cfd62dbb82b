"""The Python binding's buffer checks on a GPU: every entry point refuses a field, V grid,
checkpoint set or step-size vector of the wrong size, dtype, layout or device before the
C ABI (which sees bare pointers) is called, and the plan keeps working afterwards."""
import numpy as np
import pytest

from gpu_helpers import log
from paper_1204_4255_amd import rk4ip

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available(), "GPU tests need a GPU"
    rk4ip.load()
    return t


def test_mismatched_buffers_are_refused_before_any_call(torch):
    n, batch = 64, 2
    p = rk4ip.make_problem((n,), (-4.0,), (4.0,), 1e-3, batch=batch, g_nl=1.0, trap=(1.0, 0, 0))
    plan = rk4ip.Plan([p])
    x = np.linspace(-4, 4, n, endpoint=False)
    f0 = np.broadcast_to(np.exp(-x ** 2 / 2), (batch, n)).astype(np.complex64).reshape(-1)
    good = torch.tensor(f0, device="cuda")
    c64 = dict(dtype=torch.complex64, device="cuda")
    bad = {
        "short": torch.zeros(batch * n - 1, **c64),
        "long": torch.zeros(batch * n + 1, **c64),
        "strided": torch.zeros(2 * batch * n, **c64)[::2],
        "complex128": torch.zeros(batch * n, dtype=torch.complex128, device="cuda"),
        "host": torch.zeros(batch * n, dtype=torch.complex64),
    }
    h = torch.full((batch,), 1e-3, dtype=torch.float64, device="cuda")
    for name, b in bad.items():
        log(f"binding: psi {name}")
        calls = [lambda: plan.step(b), lambda: plan.run(b, 2), lambda: plan.diagnostics(b),
                 lambda: plan.moments(0, b), lambda: plan.overlap(0, good[:n], b), lambda: plan.apply_D(b),
                 lambda: plan.ark45(b, 0.01, 1e-6, h)]
        for call in calls:
            with pytest.raises(rk4ip.Rk4ipError) as e:
                call()
            assert e.value.status == rk4ip.RK4IP_ERR_INVALID_ARG
    with pytest.raises(rk4ip.Rk4ipError):
        plan.overlap(0, good, good)  # phi is one instance, not the whole field
    with pytest.raises(rk4ip.Rk4ipError):
        plan.ark45(good.clone(), 0.01, 1e-6, h[:1])  # one trial step per instance
    with pytest.raises(rk4ip.Rk4ipError):
        rk4ip.make_problem((n,), (-4.0,), (4.0,), 1e-3, batch=batch,
                           V_grid=torch.zeros(n, dtype=torch.float32, device="cuda"))  # [batch][n] needed
    _, ck = plan.run(good.clone(), 4, ckpt_every=2)
    with pytest.raises(rk4ip.Rk4ipError):
        plan.adjoint(ck[:1], 4, 2, torch.ones_like(good))  # two checkpoints needed
    # nothing was launched by the refused calls: the plan still matches a fresh one
    a = good.clone()
    plan.run(a, 10)
    fresh = rk4ip.Plan([p])
    b = good.clone()
    fresh.run(b, 10)
    torch.cuda.synchronize()
    assert plan.status() == rk4ip.RK4IP_OK
    assert torch.equal(a, b)
