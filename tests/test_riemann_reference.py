"""Pins of the exact Riemann solver that the Sod-tube pin of the oracle uses as its reference.

The solver (tests/riemann.py) is checked against what fixes it from outside:
- the textbook star state of Sod's shock tube at gamma = 1.4 (rho, u, p = 1, 0, 1 | 0.125, 0, 0.1):
  p* = 0.30313, u* = 0.92745, rho*_L = 0.42632, rho*_R = 0.26557 (five significant digits);
- the closed form of the star pressure when both waves are rarefactions;
- the Rankine-Hugoniot conditions (mass, momentum, energy fluxes) across every shock it returns;
- the trivial problem (equal states), whose solution is the state itself.
"""
import math

import numpy as np
import pytest

from riemann import RiemannSolution


def test_sod_star_state_gamma_1_4():
    s = RiemannSolution(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4)
    for got, want in ((s.p_star, 0.30313), (s.u_star, 0.92745), (s.rho_starL, 0.42632), (s.rho_starR, 0.26557)):
        assert abs(got - want) <= 0.6e-5 * max(1.0, abs(want)) + 5e-6, (got, want)
    w = s.wave_speeds()
    assert "left_head" in w and "right_shock" in w


def _two_rarefaction_p_star(rL, uL, pL, rR, uR, pR, g):
    # both waves rarefactions: the Riemann invariants give p* in closed form
    z = (g - 1.0) / (2.0 * g)
    aL, aR = math.sqrt(g * pL / rL), math.sqrt(g * pR / rR)
    num = aL + aR - 0.5 * (g - 1.0) * (uR - uL)
    den = aL / pL ** z + aR / pR ** z
    return (num / den) ** (1.0 / z)


@pytest.mark.parametrize("g", [1.4, 5.0 / 3.0])
@pytest.mark.parametrize("case", [(1.0, -0.5, 1.0, 0.8, 0.6, 0.7), (1.0, -1.0, 0.4, 1.0, 1.0, 0.4),
                                  (0.3, -0.4, 0.2, 1.0, 0.5, 0.5)])
def test_two_rarefactions_closed_form(case, g):
    s = RiemannSolution(*case, g)
    assert s.p_star < min(case[2], case[5])
    assert abs(s.p_star - _two_rarefaction_p_star(*case, g)) <= 1e-12 * case[2]


def _euler_flux(rho, u, p, g):
    E = p / (g - 1.0) + 0.5 * rho * u * u
    return np.array([rho * u, rho * u * u + p, u * (E + p)]), np.array([rho, rho * u, E])


@pytest.mark.parametrize("g", [1.4, 5.0 / 3.0])
@pytest.mark.parametrize("case", [(1.0, 0.0, 1.0, 0.125, 0.0, 0.1), (1.0, 0.0, 1000.0, 1.0, 0.0, 0.01),
                                  (0.5, 0.3, 0.2, 1.0, -0.4, 1.5), (1.0, 0.0, 1.0 / 3.0, 0.125, 0.0, 0.0333)])
def test_shocks_satisfy_rankine_hugoniot(case, g):
    s = RiemannSolution(*case, g)
    w = s.wave_speeds()
    sides = (("left_shock", case[:3], (s.rho_starL, s.u_star, s.p_star)),
             ("right_shock", case[3:], (s.rho_starR, s.u_star, s.p_star)))
    n = 0
    for key, outer, star in sides:
        if key not in w:
            continue
        S = w[key]
        fo, qo = _euler_flux(*outer, g)
        fs, qs = _euler_flux(*star, g)
        # F(star) - F(outer) = S (U(star) - U(outer))
        np.testing.assert_allclose(fs - fo, S * (qs - qo), rtol=1e-10, atol=1e-10 * max(1.0, abs(fo).max()))
        n += 1
    assert n >= 1


def test_equal_states_are_the_solution():
    s = RiemannSolution(0.7, 0.2, 0.4, 0.7, 0.2, 0.4, 1.4)
    assert abs(s.p_star - 0.4) <= 1e-12 and abs(s.u_star - 0.2) <= 1e-12
    for xi in (-2.0, 0.0, 0.19, 0.21, 3.0):
        np.testing.assert_allclose(s.sample(xi), (0.7, 0.2, 0.4), rtol=1e-12)
