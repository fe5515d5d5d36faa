"""Pins of the oracle's multiple-relaxation-time step (the non-hydrodynamic moments of Table I
relaxed at their own rate; the extension the paper names after Eq. 55 and writes generally with a
collision matrix).

- A uniform state at rest perturbed along one non-hydrodynamic row of Table I keeps its
  hydrodynamic moments (the rows are orthogonal under the weights), streams onto itself, and the
  perturbation's moment decays by exactly (1 - omega_g) per step, omega_g = 1/(tau_g + 1/2); with
  tau_g = tau it decays at the single rate.
- Mass, momentum and energy stay exactly conserved (the energy lives on rows 1 and 5-7).
- The shear viscosity stays T tau: the stress rows keep the rate omega.
"""
import numpy as np
import pytest

import oracle
from paper_2501_00620_amd import workloads as wl
from fitting import mode_amplitude, sine_amplitude


def ghost_row_state(a, eps=1e-3, shape=(3, 4, 5)):
    M = oracle.table_m()
    _, w = oracle.velocity_set()
    Na = 1.0 / np.sum(w * M[a] ** 2)
    f0 = oracle.feq(1.0, 0.0, 0.0, 0.0)
    df = eps * w * M[a] * Na  # the populations whose only Table I moment is eps on row a
    F = np.broadcast_to((f0 + df)[:, None, None, None], (19,) + shape).copy()
    b = np.broadcast_to(oracle.beq(0.0, 0.0, 0.0, 1 / 3)[:, None, None, None], (6,) + shape).copy()
    return M, F, b


@pytest.mark.parametrize("a", range(10, 19))
@pytest.mark.parametrize("tau_g", [0.5, 0.8, None])
def test_ghost_moment_decays_at_its_own_rate(a, tau_g):
    tau = 0.7
    M, F, b = ghost_row_state(a)
    nz, ny, nx = F.shape[1:]
    L = oracle.OracleLattice(nx, ny, nz, tau, tau_ghost=tau_g)
    L.set_state(F, b)
    m0 = M @ F[:, 0, 0, 0]
    L.step(1)
    m1 = M @ L.F[:, 0, 0, 0]
    omega_g = 1 / ((tau if tau_g is None else tau_g) + 0.5)
    assert abs(m1[a] / m0[a] - (1 - omega_g)) < 1e-10
    others = [c for c in range(19) if c != a]
    np.testing.assert_allclose(m1[others], m0[others], rtol=0, atol=1e-15)
    # uniform: every site alike
    assert np.ptp(L.F.reshape(19, -1), axis=1).max() < 1e-16


def test_mrt_conserves_mass_momentum_energy():
    dims = (9, 8, 7)
    rho, u, T = wl.fourier_fields(*dims, seed=31, u_max=0.2)
    L = oracle.OracleLattice(*dims, 0.7, tau_ghost=0.5)
    L.init(rho, u, T)
    i0 = L.invariants()
    L.step(100)
    i1 = L.invariants()
    scale = np.array([i0[0]] * 4 + [i0[4]])
    assert np.abs((i1 - i0) / scale).max() < 1e-13


def test_mrt_changes_the_state():
    # the ghost rate acts on a non-uniform flow (the pins above are not vacuous)
    dims = (9, 8, 7)
    rho, u, T = wl.fourier_fields(*dims, seed=31, u_max=0.2)
    out = []
    for tau_g in (None, 0.5):
        L = oracle.OracleLattice(*dims, 0.7, tau_ghost=tau_g)
        L.init(rho, u, T)
        L.step(20)
        out.append(L.F.copy())
    assert np.abs(out[0] - out[1]).max() > 1e-8


@pytest.mark.slow
def test_mrt_shear_viscosity_is_rho_T_tau():
    N, tau, T0 = 64, 0.6, 0.2
    k = 2 * np.pi / N
    x = np.arange(N)
    L = oracle.OracleLattice(N, 1, 1, tau, tau_ghost=0.5)
    u = np.zeros((3, 1, 1, N))
    u[1] = 1e-3 * np.sin(k * x)
    L.init(np.ones((1, 1, N)), u, np.full((1, 1, N), T0))
    ts, amp = [], []
    for t in range(0, 2001, 50):
        if t:
            L.step(50)
        uy = L.moments()[1][1, 0, 0]
        ts.append(t)
        amp.append(np.hypot(sine_amplitude(uy, k, x), mode_amplitude(uy, k, x)))
    nu = -np.polyfit(np.array(ts[4:], float), np.log(amp[4:]), 1)[0] / k ** 2
    assert abs(nu / (T0 * tau) - 1) < 0.01
