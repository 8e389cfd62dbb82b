"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
symbol the header declares, sizes workspaces and rejects bad arguments with the
documented status codes before it touches a device."""
import ctypes
import os
import re

import numpy as np

import pytest

from paper_1204_4255_amd import rk4ip

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rk4ip.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rk4ip_[a-zA-Z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(rk4ip.LIB_PATH):
        pytest.skip("librk4ip.so not built")
    return rk4ip.load()


def test_header_declares_binding_exports():
    assert _declared() == sorted(rk4ip.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_strerror_strings(lib):
    for code in range(-7, 1):
        assert rk4ip.rk4ip_strerror(code)
    assert rk4ip.rk4ip_strerror(-99) == "unknown status"


def _p(**kw):
    base = dict(n=(64, 32), lo=(-4, -4), hi=(4, 4), dt=1e-3, batch=3)
    base.update(kw)
    return rk4ip.make_problem(**base)


def test_workspace_bytes_counts_fields_tables_partials(lib):
    nb = rk4ip.rk4ip_workspace_bytes([_p()])
    pts = 64 * 32 * 3
    assert nb >= 2 * 8 * pts + 2 * 8 * (64 + 32) + 8 * 4 * (3 * 32 + 3 * 64)
    assert nb % 256 == 0
    two = rk4ip.rk4ip_workspace_bytes([_p(), _p(n=(16, 16, 16), lo=(0, 0, 0), hi=(1, 1, 1), batch=1)])
    assert two > nb


@pytest.mark.parametrize("kw", [
    dict(dt=0.0), dict(dt=-1.0), dict(batch=0), dict(gamma=-0.1), dict(sigma=-1.0),
    dict(hi=(-4, 4)), dict(dt=float("nan")),
])
def test_invalid_descriptions_give_zero_workspace(lib, kw):
    assert rk4ip.rk4ip_workspace_bytes([_p(**kw)]) == 0


@pytest.mark.parametrize("n", [(48, 32), (64, 4), (2048, 8), (6,), (8192,)])
def test_unsupported_shapes(lib, n):
    p = rk4ip.make_problem(n=n, lo=(0,) * len(n), hi=(1,) * len(n), dt=0.1)
    assert rk4ip.rk4ip_workspace_bytes([p]) == 0
    arr = rk4ip.problems_array([p])
    h = ctypes.c_void_p()
    rc = lib.rk4ip_plan(arr, 1, ctypes.c_void_p(256), 1 << 30, None, 0, ctypes.byref(h))
    assert rc == rk4ip.RK4IP_ERR_UNSUPPORTED_SHAPE and not h.value


def test_plan_argument_checks_without_device(lib):
    arr = rk4ip.problems_array([_p()])
    h = ctypes.c_void_p()
    nb = rk4ip.rk4ip_workspace_bytes([_p()])
    assert lib.rk4ip_plan(arr, 1, ctypes.c_void_p(256), nb, None, 0, None) == rk4ip.RK4IP_ERR_INVALID_ARG
    assert lib.rk4ip_plan(None, 1, ctypes.c_void_p(256), nb, None, 0, ctypes.byref(h)) == rk4ip.RK4IP_ERR_INVALID_ARG
    assert lib.rk4ip_plan(arr, 0, ctypes.c_void_p(256), nb, None, 0, ctypes.byref(h)) == rk4ip.RK4IP_ERR_INVALID_ARG
    assert lib.rk4ip_plan(arr, 1, None, nb, None, 0, ctypes.byref(h)) == rk4ip.RK4IP_ERR_INVALID_ARG
    assert lib.rk4ip_plan(arr, 1, ctypes.c_void_p(300), nb, None, 0, ctypes.byref(h)) == rk4ip.RK4IP_ERR_INVALID_ARG
    assert lib.rk4ip_plan(arr, 1, ctypes.c_void_p(256), nb, None, 0x100, ctypes.byref(h)) == rk4ip.RK4IP_ERR_INVALID_ARG
    assert (lib.rk4ip_plan(arr, 1, ctypes.c_void_p(256), nb - 256, None, 0, ctypes.byref(h))
            == rk4ip.RK4IP_ERR_WORKSPACE_TOO_SMALL)
    mixed = rk4ip.problems_array([_p(), _p(dt=2e-3)])
    assert lib.rk4ip_plan(mixed, 2, ctypes.c_void_p(256), 1 << 30, None, 0, ctypes.byref(h)) == rk4ip.RK4IP_ERR_INVALID_ARG
    bad = _p()
    bad.basis = 3
    assert rk4ip.rk4ip_workspace_bytes([bad]) == 0
    ids = _p(batch=10)
    ids.id_base = 0xFFFFFFFF - 3
    assert rk4ip.rk4ip_workspace_bytes([ids]) == 0


def test_null_plan_calls_are_rejected(lib):
    assert lib.rk4ip_step(None, ctypes.c_void_p(256), 0) == rk4ip.RK4IP_ERR_INVALID_ARG
    assert lib.rk4ip_run(None, ctypes.c_void_p(256), 0, 1, 0, None, None, 0) == rk4ip.RK4IP_ERR_INVALID_ARG
    assert lib.rk4ip_status(None) == rk4ip.RK4IP_ERR_INVALID_ARG
    assert lib.rk4ip_destroy(None) == rk4ip.RK4IP_ERR_INVALID_ARG
    assert lib.rk4ip_last_error(None) == b""
    assert lib.rk4ip_debug_philox(0, None, 1, None, None) == rk4ip.RK4IP_ERR_INVALID_ARG
    assert lib.rk4ip_ark45(None, ctypes.c_void_p(256), 1.0, 1e-6, 10, ctypes.c_void_p(256), ctypes.c_void_p(256),
                           None, 0, 0) == rk4ip.RK4IP_ERR_INVALID_ARG


def test_valid_plan_without_gpu_reports_no_device(lib):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    arr = rk4ip.problems_array([_p()])
    h = ctypes.c_void_p()
    nb = rk4ip.rk4ip_workspace_bytes([_p()])
    rc = lib.rk4ip_plan(arr, 1, ctypes.c_void_p(256), nb, None, 0, ctypes.byref(h))
    assert rc == rk4ip.RK4IP_ERR_NO_DEVICE and not h.value


def test_fp64_transform_flag_sizes_and_limits(lib):
    """The FP64-transform form adds FP64 copies of the tables to the workspace and limits
    1D lines to 2048 points (its tables and exchange buffers live in LDS)."""
    f64 = rk4ip.RK4IP_FLAG_FP64_TRANSFORMS
    p = _p()
    n32 = rk4ip.rk4ip_workspace_bytes([p])
    n64 = rk4ip.rk4ip_workspace_bytes([p], f64)
    assert n64 > n32 > 0
    for n, ok in (((2048,), True), ((4096,), False)):
        q = rk4ip.make_problem(n=n, lo=(0,), hi=(1,), dt=0.1)
        assert (rk4ip.rk4ip_workspace_bytes([q], f64) > 0) == ok
        assert rk4ip.rk4ip_workspace_bytes([q]) > 0
    assert rk4ip.rk4ip_workspace_bytes([p], 0x100) == 0  # unknown flag bits


def test_semi_implicit_flag_and_noise_substeps(lib):
    """The semi-implicit form uses the RK4 form's tables (the half-step propagator, twice
    where two steps meet) and workspace; noise_substeps is 0, 1 or a power of two up to
    1024."""
    si = rk4ip.RK4IP_FLAG_SEMI_IMPLICIT
    p = _p()
    assert rk4ip.rk4ip_workspace_bytes([p], si) == rk4ip.rk4ip_workspace_bytes([p]) > 0
    line = rk4ip.make_problem(n=(256,), lo=(0,), hi=(1,), dt=0.1)
    assert rk4ip.rk4ip_workspace_bytes([line], si) == rk4ip.rk4ip_workspace_bytes([line]) > 0
    for S, ok in ((0, True), (1, True), (2, True), (64, True), (1024, True), (3, False), (12, False),
                  (2048, False)):
        assert (rk4ip.rk4ip_workspace_bytes([_p(noise_substeps=S)], si) > 0) == ok, S
        assert (rk4ip.rk4ip_workspace_bytes([_p(noise_substeps=S)]) > 0) == ok, S
    assert rk4ip.rk4ip_workspace_bytes([p], si | rk4ip.RK4IP_FLAG_FP64_TRANSFORMS) > rk4ip.rk4ip_workspace_bytes([p], si)


def test_potential_terms_sizes_and_limits(lib):
    """The non-local kernel's transform adds n complex64 entries to the workspace and is
    taken on 1D groups only, with finite values; the noise in the potential needs sigma_V >= 0.
    A plain Fourier line also keeps the table (e^{L h} - 1)/n (n entries) and its k-space
    state (batch x n complex64), which the lines with the potential's extra terms (run in
    x-space) do not."""
    line = dict(n=(256,), lo=(0,), hi=(1,), dt=0.1)
    plain = rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(**line)])
    base = rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(**line, sigma_V=0.3)])
    assert plain == base + 2 * 256 * 8
    K = np.ones(256)
    assert rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(**line, conv_K=K)]) == base + 256 * 8
    assert rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(**line, batch=4)]) == (
        rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(**line, batch=4, sigma_V=0.3)]) + 5 * 256 * 8)
    assert rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(**line, sigma_V=-0.3)]) == 0
    bad = K.copy()
    bad[3] = np.nan
    assert rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(**line, conv_K=bad)]) == 0
    assert rk4ip.rk4ip_workspace_bytes([_p(sigma_V=0.1)]) == rk4ip.rk4ip_workspace_bytes([_p()])
    assert rk4ip.rk4ip_workspace_bytes([_p(conv_K=np.ones(64))]) == 0


def test_cosine_and_sine_bases_sizes_and_limits(lib):
    """A cosine / sine group runs through the n-point transform of its reordered line: its
    two mode-pairing tables of n FP64 entries besides the two tables every line keeps (a
    Fourier line run in x-space, one with noise in its potential, keeps those two only),
    and lines up to 4096 points. In the FP64-transform form, or with noise in its potential, it
    runs on the even / odd extension (twice the stored points; its tables doubled)."""
    line = dict(lo=(0,), hi=(7,), dt=0.1)
    f = rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(n=(256,), sigma_V=0.1, **line)])
    f64 = rk4ip.RK4IP_FLAG_FP64_TRANSFORMS
    for basis in (1, 2):
        c = rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(n=(256,), basis=basis, **line)])
        assert c == f + 2 * 256 * 16
        ext = rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(n=(256,), basis=basis, sigma_V=0.1, **line)])
        assert ext == f + 2 * 256 * 8  # the two tables doubled
        assert rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(n=(4096,), basis=basis, **line)]) > 0
        assert rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(n=(4096,), basis=basis, sigma_V=0.1, **line)]) == 0
        assert rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(n=(1024,), basis=basis, **line)], f64) > 0
        assert rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(n=(2048,), basis=basis, **line)], f64) == 0
        assert rk4ip.rk4ip_workspace_bytes([_p(basis=basis)]) == 0
        assert rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(n=(64,), basis=basis, conv_K=np.ones(64),
                                                               **line)]) == 0


def test_binding_refuses_buffers_that_do_not_fit(lib):
    """The C ABI takes bare pointers, so the binding checks every tensor it hands over:
    host tensors, wrong dtypes, strided views and wrong sizes are refused before a call."""
    import torch

    with pytest.raises(rk4ip.Rk4ipError):
        rk4ip._buf(torch.zeros(8, dtype=torch.complex64), 8, torch.complex64, "psi")  # host memory
    with pytest.raises(rk4ip.Rk4ipError):
        rk4ip._buf(None, 8, torch.complex64, "psi")
    assert rk4ip._buf(None, 8, torch.complex64, "psi", optional=True) is None
    with pytest.raises(rk4ip.Rk4ipError):
        rk4ip.make_problem((64,), (0,), (1,), 1e-3, conv_K=np.ones(63))
    with pytest.raises(rk4ip.Rk4ipError):
        rk4ip.make_problem((64,), (0,), (1,), 1e-3, batch=2, V_grid=torch.zeros(128))  # host memory


def test_instances_beyond_32bit_tile_offsets_are_refused(lib):
    """The pass kernels address a tile with 32-bit byte offsets from the instance origin, so
    one instance holds at most 2^29 complex64 points: 1024^3 is refused, 1024 x 1024 x 512
    (exactly 4 GiB) is taken, and so is 512^3 with a large batch."""
    big = dict(lo=(0, 0, 0), hi=(1, 1, 1), dt=1e-3)
    assert rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(n=(1024, 1024, 1024), **big)]) == 0
    assert rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(n=(1024, 1024, 512), **big)]) > 0
    assert rk4ip.rk4ip_workspace_bytes([rk4ip.make_problem(n=(512, 512, 512), batch=8, **big)]) > 0
    h = ctypes.c_void_p()
    arr = (rk4ip.rk4ip_problem * 1)(rk4ip.make_problem(n=(1024, 1024, 1024), **big))
    rc = lib.rk4ip_plan(arr, 1, ctypes.c_void_p(256), 1 << 40, None, 0, ctypes.byref(h))
    assert rc == rk4ip.RK4IP_ERR_UNSUPPORTED_SHAPE and not h.value


def test_noalloc_step_refuses_before_touching_a_device(lib):
    """rk4ip_step_noalloc checks its arguments before it looks for a device: more than 16
    groups, a non-local kernel or a problem beyond its static buffer are refused with the
    documented codes; a valid call on a host without a gfx950 says so."""
    fake = ctypes.c_void_p(256)
    small = rk4ip.make_problem((64,), (0,), (1,), 1e-3)
    many = rk4ip.problems_array([small] * 17)
    assert lib.rk4ip_step_noalloc(many, 17, fake, 0, None) == rk4ip.RK4IP_ERR_INVALID_ARG
    conv = rk4ip.problems_array([rk4ip.make_problem((64,), (0,), (1,), 1e-3, conv_K=np.ones(64))])
    assert lib.rk4ip_step_noalloc(conv, 1, fake, 0, None) == rk4ip.RK4IP_ERR_INVALID_ARG
    big = rk4ip.problems_array([rk4ip.make_problem((256, 256, 128), (0, 0, 0), (1, 1, 1), 1e-3)])
    assert lib.rk4ip_step_noalloc(big, 1, fake, 0, None) == rk4ip.RK4IP_ERR_WORKSPACE_TOO_SMALL
    one = rk4ip.problems_array([small])
    assert lib.rk4ip_step_noalloc(one, 1, None, 0, None) == rk4ip.RK4IP_ERR_INVALID_ARG
    assert lib.rk4ip_step_noalloc(one, 1, fake, -1, None) == rk4ip.RK4IP_ERR_INVALID_ARG
    import torch

    if not torch.cuda.is_available():
        assert lib.rk4ip_step_noalloc(one, 1, fake, 0, None) == rk4ip.RK4IP_ERR_NO_DEVICE


def test_merge_groups_flag_limits(lib):
    """RK4IP_FLAG_MERGE_GROUPS takes RK4IP with FP32 transforms on lattices whose axes have
    128 or 256 points (and enough x columns for the strided tiles); it adds the groups'
    kernel parameters to the workspace."""
    M = rk4ip.RK4IP_FLAG_MERGE_GROUPS
    ok = [rk4ip.make_problem((128, 128), (0, 0), (1, 1), 1e-3, batch=3),
          rk4ip.make_problem((256, 256), (0, 0), (1, 1), 1e-3, batch=2),
          rk4ip.make_problem((64,), (0,), (1,), 1e-3)]
    assert rk4ip.rk4ip_workspace_bytes(ok, M) > rk4ip.rk4ip_workspace_bytes(ok, 0) > 0
    for bad in ([rk4ip.make_problem((64, 64), (0, 0), (1, 1), 1e-3)],
                [rk4ip.make_problem((512, 128), (0, 0), (1, 1), 1e-3)]):
        assert rk4ip.rk4ip_workspace_bytes(bad, M) == 0
        assert rk4ip.rk4ip_workspace_bytes(bad, 0) > 0
    assert rk4ip.rk4ip_workspace_bytes(ok, M | rk4ip.RK4IP_FLAG_SEMI_IMPLICIT) == 0
    assert rk4ip.rk4ip_workspace_bytes(ok, M | rk4ip.RK4IP_FLAG_FP64_TRANSFORMS) == 0
