"""Exact solution of the Riemann problem of the 1-D Euler equations for an ideal gas.

The textbook two-rarefaction/two-shock construction: the star pressure solves
f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the shock (Rankine-Hugoniot) branch for
p > p_K and the isentropic rarefaction branch otherwise; the solution is then sampled on
rays x/t.  Written for the tests from the gas-dynamics definitions, with p = rho T (T in energy
units) and sound speed a = sqrt(gamma p / rho).
"""
import math

import numpy as np


def _f(p, rho, pk, g):
    a = math.sqrt(g * pk / rho)
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        f = (p - pk) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - 0.5 * (p - pk) / (B + p))
    else:
        f = 2.0 * a / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = (1.0 / (rho * a)) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


class RiemannSolution:
    def __init__(self, rhoL, uL, pL, rhoR, uR, pR, gamma):
        self.L = (rhoL, uL, pL)
        self.R = (rhoR, uR, pR)
        self.g = g = gamma
        p = 0.5 * (pL + pR)
        for _ in range(100):
            fL, dL = _f(p, rhoL, pL, g)
            fR, dR = _f(p, rhoR, pR, g)
            dp = (fL + fR + uR - uL) / (dL + dR)
            pn = max(p - dp, 1e-14)
            if abs(pn - p) < 1e-15 * (pn + p):
                p = pn
                break
            p = pn
        self.p_star = p
        fL, _ = _f(p, rhoL, pL, g)
        fR, _ = _f(p, rhoR, pR, g)
        self.u_star = 0.5 * (uL + uR) + 0.5 * (fR - fL)
        # star densities
        self.rho_starL = self._star_rho(rhoL, pL)
        self.rho_starR = self._star_rho(rhoR, pR)

    def _star_rho(self, rho, pk):
        g, p = self.g, self.p_star
        if p > pk:
            r = p / pk
            gm = (g - 1.0) / (g + 1.0)
            return rho * (r + gm) / (gm * r + 1.0)
        return rho * (p / pk) ** (1.0 / g)

    def wave_speeds(self):
        """Dict of the left wave (head, tail or shock), contact and right wave speeds."""
        g = self.g
        rhoL, uL, pL = self.L
        rhoR, uR, pR = self.R
        aL, aR = math.sqrt(g * pL / rhoL), math.sqrt(g * pR / rhoR)
        out = {"contact": self.u_star}
        if self.p_star > pL:
            out["left_shock"] = uL - aL * math.sqrt((g + 1) / (2 * g) * self.p_star / pL + (g - 1) / (2 * g))
        else:
            out["left_head"] = uL - aL
            out["left_tail"] = self.u_star - aL * (self.p_star / pL) ** ((g - 1) / (2 * g))
        if self.p_star > pR:
            out["right_shock"] = uR + aR * math.sqrt((g + 1) / (2 * g) * self.p_star / pR + (g - 1) / (2 * g))
        else:
            out["right_head"] = uR + aR
            out["right_tail"] = self.u_star + aR * (self.p_star / pR) ** ((g - 1) / (2 * g))
        return out

    def sample(self, xi):
        """(rho, u, p) on the ray x/t = xi."""
        g = self.g
        rhoL, uL, pL = self.L
        rhoR, uR, pR = self.R
        ps, us = self.p_star, self.u_star
        if xi <= us:  # left of the contact
            a = math.sqrt(g * pL / rhoL)
            if ps > pL:
                s = uL - a * math.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
                return (rhoL, uL, pL) if xi <= s else (self.rho_starL, us, ps)
            head = uL - a
            tail = us - a * (ps / pL) ** ((g - 1) / (2 * g))
            if xi <= head:
                return rhoL, uL, pL
            if xi >= tail:
                return self.rho_starL, us, ps
            c = 2.0 / (g + 1) + (g - 1) / ((g + 1) * a) * (uL - xi)
            return (rhoL * c ** (2 / (g - 1)), 2 / (g + 1) * (a + (g - 1) / 2 * uL + xi),
                    pL * c ** (2 * g / (g - 1)))
        a = math.sqrt(g * pR / rhoR)
        if ps > pR:
            s = uR + a * math.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
            return (rhoR, uR, pR) if xi >= s else (self.rho_starR, us, ps)
        head = uR + a
        tail = us + a * (ps / pR) ** ((g - 1) / (2 * g))
        if xi >= head:
            return rhoR, uR, pR
        if xi <= tail:
            return self.rho_starR, us, ps
        c = 2.0 / (g + 1) - (g - 1) / ((g + 1) * a) * (uR - xi)
        return (rhoR * c ** (2 / (g - 1)), 2 / (g + 1) * (-a + (g - 1) / 2 * uR + xi),
                pR * c ** (2 * g / (g - 1)))

    def profile(self, x, x0, t):
        out = np.array([self.sample((xx - x0) / t) for xx in x])
        return out[:, 0], out[:, 1], out[:, 2]
