"""Closed forms shared by the oracle pins and the GPU tests: the amplitude recursion of a
plane wave under a density-dependent potential, and the non-local test case."""
import numpy as np


def plane_wave_amplitude(A, S, h, E, kappa, si):
    """S steps of the RK4IP (si False) or semi-implicit (three midpoint iterations) step
    on the scalar equation dA/dt = lambda A - i kappa |A|^2 A, E = e^{lambda h/2}."""

    def G(y):
        return -1j * kappa * abs(y) ** 2 * y

    for _ in range(S):
        a = E * A
        if si:
            m = a
            for _ in range(3):
                m = a + 0.5 * h * G(m)
            A = E * (2 * m - a)
        else:
            k1 = E * h * G(A)
            k2 = h * G(a + k1 / 2)
            k3 = h * G(a + k2 / 2)
            k4 = h * G(E * (a + k3))
            A = E * (a + k1 / 6 + k2 / 3 + k3 / 3) + k4 / 6
    return A


def non_local_case():
    n, L, gnl = 256, 16.0, 0.5
    dx = L / n
    dd = np.arange(n)
    dd = np.where(dd < n // 2, dd, dd - n) * dx
    K = 1.0 / np.sqrt(dd ** 2 + 1.0)  # softened Coulomb kernel at the lattice offsets
    qs, amps = [2, -7, 30], [1.0, 0.7, 1.3]
    x = np.arange(n) * dx - L / 2
    psi0 = np.stack([a * np.exp(2j * np.pi * q * (x + L / 2) / L) for q, a in zip(qs, amps)])
    return n, L, gnl, dx, K, qs, amps, psi0
