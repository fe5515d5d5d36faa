"""Pins of the oracle's body force (an acceleration field entering the forcing moments in the
manner of a Guo forcing: F += rho a, S += rho (u a + a u), the corrected velocity carrying half of
rho a; the paper drives its Poiseuille and Couette flows with such a force, Sec. III A and C).

- Momentum: the single-rate update changes a site's momentum by exactly its forcing moment F; the
  gradient part sums to zero over a periodic lattice, so the total momentum grows by exactly
  M a per step under a uniform acceleration a (M the conserved mass).
- Kolmogorov flow: a_y = A sin(k x) drives the steady shear u_y = A sin(k x) / (nu k^2) with
  nu = T tau (Sec. II D), in both temperature modes.
- A zero acceleration field is the force-free step, bit for bit.
"""
import numpy as np
import pytest

import oracle
from fitting import sine_amplitude
from paper_2501_00620_amd import workloads as wl


def test_uniform_force_adds_exactly_its_momentum():
    rho, u, T = wl.fourier_fields(6, 5, 4, seed=2, u_max=0.1)
    L = oracle.OracleLattice(6, 5, 4, 0.7)
    L.init(rho, u, T)
    a = np.array([1e-4, -2e-4, 3e-5])
    L.set_body_force(a)
    e, _ = oracle.velocity_set()
    P0 = e.T.astype(float) @ L.F.reshape(19, -1).sum(axis=1)
    M = L.F.sum()
    L.step(50)
    P1 = e.T.astype(float) @ L.F.reshape(19, -1).sum(axis=1)
    np.testing.assert_allclose(P1 - P0, 50 * M * a, rtol=0, atol=1e-13)
    assert abs(L.F.sum() / M - 1) < 1e-14


def test_zero_force_is_the_force_free_step():
    rho, u, T = wl.fourier_fields(7, 6, 5, seed=9, u_max=0.2)
    out = []
    for accel in (None, np.zeros((3, 5, 6, 7))):
        L = oracle.OracleLattice(7, 6, 5, 0.65)
        L.init(rho, u, T)
        L.set_body_force(accel)
        L.step(5)
        out.append(L.F.copy())
    np.testing.assert_array_equal(out[0], out[1])


@pytest.mark.slow
@pytest.mark.parametrize("mode", ["thermal", "iso"])
@pytest.mark.parametrize("T0", [1 / 3, 0.2])
def test_kolmogorov_flow_amplitude(mode, T0):
    N, tau, A = 64, 0.6, 1e-6
    k = 2 * np.pi / N
    x = np.arange(N)
    L = oracle.OracleLattice(N, 1, 1, tau, mode=mode)
    L.init(np.ones((1, 1, N)), np.zeros((3, 1, 1, N)), np.full((1, 1, N), T0))
    accel = np.zeros((3, 1, 1, N))
    accel[1, 0, 0] = A * np.sin(k * x)
    L.set_body_force(accel)
    L.step(8000)  # ~9 viscous times 1/(nu k^2)
    amp = sine_amplitude(L.moments()[1][1, 0, 0], k, x)
    assert abs(amp / (A / (T0 * tau * k * k)) - 1) < 0.005
