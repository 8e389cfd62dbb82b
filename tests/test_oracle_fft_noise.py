"""Pins of the oracle's transforms and noise generator against values fixed outside it.

Transforms (Sec. 3.2: FFT per dimension of the tensor-product lattice): brute-force DFT
sums, the exact delta spectrum of a lattice exponential, the inverse relation and
Parseval. numpy's FFT appears only as an extra cross-check at large sizes.
Noise (Sec. 3.5, Wiener noise): the published Philox4x32-10 known-answer vectors and the
distributional properties the reading of the noise fixes (E xi = 0, E|xi|^2 = 1/(h dV),
E xi^2 = 0, no lag correlation, Gaussian marginals).
"""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand(n, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    return r.standard_normal(n) + 1j * r.standard_normal(n)


@pytest.mark.parametrize("n", [2, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft_matches_bruteforce_dft(n, sign):
    x = _rand(n, n)
    ref = np.array([sum(x[j] * np.exp(sign * 2j * np.pi * j * m / n) for j in range(n)) for m in range(n)])
    assert np.max(np.abs(oracle.fft(x, sign) - ref)) <= 1e-13 * n
    assert np.max(np.abs(oracle.dft(x, sign) - ref)) <= 1e-13 * n


@pytest.mark.parametrize("n", [8, 256, 4096])
def test_fft_of_lattice_exponential_is_delta(n):
    m0 = 3 % n
    j = np.arange(n)
    x = np.exp(2j * np.pi * m0 * j / n)
    X = oracle.fft(x, -1)
    ref = np.zeros(n, complex)
    ref[m0] = n
    assert np.max(np.abs(X - ref)) <= 1e-12 * n


@pytest.mark.parametrize("n", [16, 1024])
def test_fft_inverse_and_parseval(n):
    x = _rand(n, 7)
    X = oracle.fft(x, -1)
    back = oracle.fft(X, +1) / n
    assert np.max(np.abs(back - x)) <= 1e-13 * np.sqrt(n)
    assert abs(np.sum(np.abs(X) ** 2) / n - np.sum(np.abs(x) ** 2)) <= 1e-12 * np.sum(np.abs(x) ** 2)


@pytest.mark.parametrize("n", [512, 4096])
def test_fft_cross_check_numpy(n):
    x = _rand(n, 11)
    assert np.max(np.abs(oracle.fft(x, -1) - np.fft.fft(x))) <= 1e-12 * np.sqrt(n)


def test_fft_nd_is_tensor_product_of_1d_dfts():
    # 3D lattice 8 x 4 x 2 (x contiguous): the transform must equal the full triple sum.
    p = oracle.Problem(n=(8, 4, 2), lo=(0, 0, 0), hi=(1, 1, 1), h=0.1)
    f = _rand(p.M, 3).reshape(p.shape)
    F = oracle.fft_nd(p, f, -1)[0]
    nz, ny, nx = 2, 4, 8
    ref = np.zeros((nz, ny, nx), complex)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nx):
                ph = np.exp(-2j * np.pi * (kx * x / nx + ky * y / ny + kz * z / nz))
                ref[kz, ky, kx] = np.sum(f[0] * ph)
    assert np.max(np.abs(F - ref)) <= 1e-12


# ---------------------------------------------------------------------------- noise


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert oracle.philox4x32_10(ctr, key).tolist() == out


def test_philox_batch_matches_single_calls():
    r = np.random.Generator(np.random.PCG64(5))
    ctr = r.integers(0, 2 ** 32, size=(64, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0x123456789ABCDEF0
    out = oracle.philox_batch(ctr, seed)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for i in range(64):
        assert out[i].tolist() == oracle.philox4x32_10(ctr[i], key).tolist()


def _noise_problem(n=4096, batch=16, h=1e-3, L=16.0):
    return oracle.Problem(n=(n,), lo=(-L,), hi=(L,), h=h, batch=batch, sigma=1.0, seed=99, id_base=7)


def test_noise_moments():
    p = _noise_problem()
    xi = oracle.noise(p, step=12).reshape(-1)
    dV = 32.0 / 4096
    s2 = 1.0 / (p.h * dV)                # E|xi|^2 fixed by the reading of Wiener noise
    K = xi.size
    z = xi / np.sqrt(s2)                 # unit complex normal: E|z|^2 = 1
    assert abs(np.mean(z.real)) < 4 / np.sqrt(2 * K) * 1.0 + 0  # sd of mean is 1/sqrt(2K)
    assert abs(np.mean(z.imag)) < 4 / np.sqrt(2 * K)
    assert abs(np.mean(np.abs(z) ** 2) - 1.0) < 4 * 1.0 / np.sqrt(K)     # Var|z|^2 = 1
    assert abs(np.mean(z * z)) < 4 / np.sqrt(K)                          # E z^2 = 0
    lag = np.mean(z[1:] * np.conj(z[:-1]))
    assert abs(lag) < 4 / np.sqrt(K)


def test_noise_gaussian_marginals():
    from scipy import stats

    p = _noise_problem()
    xi = oracle.noise(p, step=3).reshape(-1)
    z = xi * np.sqrt(2 * p.h * (32.0 / 4096))   # standard normal real and imaginary parts
    for comp in (z.real, z.imag):
        assert stats.kstest(comp, "norm").pvalue > 1e-4
    # modulus^2 / 2 of a circular complex normal is Exp(1)
    assert stats.kstest(np.abs(z) ** 2 / 2, "expon").pvalue > 1e-4


def test_noise_independent_across_steps_and_instances():
    p = _noise_problem(n=2048, batch=4)
    a = oracle.noise(p, step=0)
    b = oracle.noise(p, step=1)
    K = a.size
    c = np.mean(a * np.conj(b)) / np.mean(np.abs(a) ** 2)
    assert abs(c) < 4 / np.sqrt(K)
    c2 = np.mean(a[0] * np.conj(a[1])) / np.mean(np.abs(a[0]) ** 2)
    assert abs(c2) < 4 / np.sqrt(a.shape[1])
    # deterministic: same step, same counters, same values
    assert np.array_equal(oracle.noise(p, step=1), b)
