"""Exact solution of the 1D Riemann problem for an ideal gas (test utility).

Part of the test infrastructure: the oracle's scheme is checked against it on
grid-aligned shock-tube problems such as Sod's, which the paper's Riemann
problem extends to 3D (Section 3).  The solution is the classical one: the
star-region pressure p* is the root of

    f(p) = f_L(p) + f_R(p) + (u_R - u_L) = 0,

where f_K is the velocity jump across a shock (Rankine-Hugoniot, p > p_K) or
a rarefaction (isentropic, p <= p_K) connecting state K to pressure p.  Then
u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2, and the self-similar solution is
sampled at xi = (x - x0)/t.
"""
import math

import numpy as np
from scipy.optimize import brentq


def _sound(gamma, rho, p):
    return math.sqrt(gamma * p / rho)


def _f(gamma, p, rhoK, pK):
    """Velocity change across the wave connecting (rhoK, pK) to pressure p."""
    cK = _sound(gamma, rhoK, pK)
    if p > pK:  # shock
        A = 2.0 / ((gamma + 1.0) * rhoK)
        B = (gamma - 1.0) / (gamma + 1.0) * pK
        return (p - pK) * math.sqrt(A / (p + B))
    # rarefaction
    return 2.0 * cK / (gamma - 1.0) * ((p / pK) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


class RiemannSolution:
    """Exact solution for left state (rhoL, uL, pL) and right (rhoR, uR, pR)."""

    def __init__(self, left, right, gamma=1.4):
        self.g = float(gamma)
        self.rhoL, self.uL, self.pL = map(float, left)
        self.rhoR, self.uR, self.pR = map(float, right)
        g = self.g
        cL = _sound(g, self.rhoL, self.pL)
        cR = _sound(g, self.rhoR, self.pR)
        if 2.0 * (cL + cR) / (g - 1.0) <= self.uR - self.uL:
            raise ValueError("vacuum is generated; not handled")

        def fun(p):
            return (_f(g, p, self.rhoL, self.pL) + _f(g, p, self.rhoR, self.pR)
                    + (self.uR - self.uL))

        lo, hi = 1e-14, max(self.pL, self.pR)
        while fun(hi) < 0.0:
            hi *= 2.0
        self.p_star = brentq(fun, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
        ps = self.p_star
        self.u_star = 0.5 * (self.uL + self.uR) + 0.5 * (
            _f(g, ps, self.rhoR, self.pR) - _f(g, ps, self.rhoL, self.pL))
        gm = (g - 1.0) / (g + 1.0)
        # star densities
        if ps > self.pL:
            self.rho_starL = self.rhoL * (ps / self.pL + gm) / (gm * ps / self.pL + 1.0)
        else:
            self.rho_starL = self.rhoL * (ps / self.pL) ** (1.0 / g)
        if ps > self.pR:
            self.rho_starR = self.rhoR * (ps / self.pR + gm) / (gm * ps / self.pR + 1.0)
        else:
            self.rho_starR = self.rhoR * (ps / self.pR) ** (1.0 / g)
        self.cL, self.cR = cL, cR

    # wave speeds -----------------------------------------------------------
    def left_wave(self):
        """(head, tail) speeds of the left wave; equal for a shock."""
        g, ps = self.g, self.p_star
        if ps > self.pL:
            s = self.uL - self.cL * math.sqrt((g + 1) / (2 * g) * ps / self.pL + (g - 1) / (2 * g))
            return s, s
        cs = self.cL * (ps / self.pL) ** ((g - 1) / (2 * g))
        return self.uL - self.cL, self.u_star - cs

    def right_wave(self):
        """(tail, head) speeds of the right wave; equal for a shock."""
        g, ps = self.g, self.p_star
        if ps > self.pR:
            s = self.uR + self.cR * math.sqrt((g + 1) / (2 * g) * ps / self.pR + (g - 1) / (2 * g))
            return s, s
        cs = self.cR * (ps / self.pR) ** ((g - 1) / (2 * g))
        return self.u_star + cs, self.uR + self.cR

    def breakpoints(self):
        """All wave speeds where the solution has a kink or a jump."""
        return sorted(set(self.left_wave() + (self.u_star,) + self.right_wave()))

    # sampling ----------------------------------------------------------------
    def sample(self, xi):
        """(rho, u, p) at similarity coordinate xi = (x - x0)/t."""
        g = self.g
        if xi < self.u_star:
            head, tail = self.left_wave()
            if xi < head:
                return self.rhoL, self.uL, self.pL
            if xi >= tail:
                return self.rho_starL, self.u_star, self.p_star
            # inside the left rarefaction fan
            u = 2.0 / (g + 1.0) * (self.cL + 0.5 * (g - 1.0) * self.uL + xi)
            c = 2.0 / (g + 1.0) * (self.cL + 0.5 * (g - 1.0) * (self.uL - xi))
            rho = self.rhoL * (c / self.cL) ** (2.0 / (g - 1.0))
            p = self.pL * (c / self.cL) ** (2.0 * g / (g - 1.0))
            return rho, u, p
        tail, head = self.right_wave()
        if xi > head:
            return self.rhoR, self.uR, self.pR
        if xi <= tail:
            return self.rho_starR, self.u_star, self.p_star
        u = 2.0 / (g + 1.0) * (-self.cR + 0.5 * (g - 1.0) * self.uR + xi)
        c = 2.0 / (g + 1.0) * (self.cR - 0.5 * (g - 1.0) * (self.uR - xi))
        rho = self.rhoR * (c / self.cR) ** (2.0 / (g - 1.0))
        p = self.pR * (c / self.cR) ** (2.0 * g / (g - 1.0))
        return rho, u, p

    def cell_averages(self, edges, t, x0=0.5, field=0):
        """Exact averages of rho (field 0), u (1) or p (2) over cells with
        the given edges at time t > 0.  Each cell is split at the wave
        positions and integrated with 8-point Gauss-Legendre per piece, so
        constant pieces and the rarefaction fan are integrated to round-off."""
        xg, wg = np.polynomial.legendre.leggauss(8)
        waves = [x0 + s * t for s in self.breakpoints()]
        out = np.empty(len(edges) - 1)
        for c in range(len(edges) - 1):
            a, b = float(edges[c]), float(edges[c + 1])
            cuts = [a] + [w for w in waves if a < w < b] + [b]
            acc = 0.0
            for lo, hi in zip(cuts[:-1], cuts[1:]):
                mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
                for xq, wq in zip(xg, wg):
                    acc += wq * half * self.sample((mid + half * xq - x0) / t)[field]
            out[c] = acc / (b - a)
        return out
