"""Exact solution of the one-dimensional Riemann problem for an ideal gas.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper validates its scheme on the one-dimensional shock tube and compares
with the analytical solution (Sec. V, citing Sod).  That solution is the
classical one: two constant states separated by a diaphragm evolve into a
left wave (shock or rarefaction), a contact discontinuity and a right wave.
The star pressure p* solves

    f_L(p*) + f_R(p*) + (u_R - u_L) = 0,

with, for side K,
    shock (p > p_K):        (p - p_K) sqrt(A_K / (p + B_K)),
                            A_K = 2 / ((gamma+1) rho_K),
                            B_K = (gamma-1)/(gamma+1) p_K
    rarefaction (p <= p_K): 2 a_K / (gamma-1) ((p/p_K)^((gamma-1)/(2 gamma)) - 1)
and u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2.  The solution is then a
function of S = x/t only, sampled wave by wave.

Dimensionless units as in Sec. II: p = rho T, sound speed sqrt(gamma T).
"""
import math

import numpy as np


def _f_and_df(p, rho, pk, ak, gamma):
    if p > pk:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (B + p))
    ratio = p / pk  # rarefaction
    f = 2.0 * ak / (gamma - 1.0) * (ratio ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
    df = 1.0 / (rho * ak) * ratio ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


class RiemannSolution:
    """Exact solution for left/right states (rho, u, p) and ratio gamma."""

    def __init__(self, left, right, gamma, tol=1e-14, max_iter=200):
        self.rl, self.ul, self.pl = map(float, left)
        self.rr, self.ur, self.pr = map(float, right)
        self.gamma = g = float(gamma)
        if min(self.rl, self.rr, self.pl, self.pr) <= 0:
            raise ValueError("densities and pressures must be positive")
        self.al = math.sqrt(g * self.pl / self.rl)
        self.ar = math.sqrt(g * self.pr / self.rr)
        du = self.ur - self.ul
        if 2.0 * (self.al + self.ar) / (g - 1.0) <= du:
            raise ValueError("the initial states generate vacuum")
        # two-rarefaction guess, then Newton's method kept positive
        z = (g - 1.0) / (2.0 * g)
        p = ((self.al + self.ar - 0.5 * (g - 1.0) * du)
             / (self.al / self.pl ** z + self.ar / self.pr ** z)) ** (1.0 / z)
        p = max(p, 1e-12)
        for _ in range(max_iter):
            fl, dfl = _f_and_df(p, self.rl, self.pl, self.al, g)
            fr, dfr = _f_and_df(p, self.rr, self.pr, self.ar, g)
            p_new = p - (fl + fr + du) / (dfl + dfr)
            if p_new <= 0:
                p_new = 0.5 * p
            if abs(p_new - p) <= tol * 0.5 * (p_new + p):
                p = p_new
                break
            p = p_new
        else:
            raise RuntimeError("star pressure did not converge")
        fl, _ = _f_and_df(p, self.rl, self.pl, self.al, g)
        fr, _ = _f_and_df(p, self.rr, self.pr, self.ar, g)
        self.p_star = p
        self.u_star = 0.5 * (self.ul + self.ur) + 0.5 * (fr - fl)
        self.rho_star_l = self._star_density(p, self.rl, self.pl)
        self.rho_star_r = self._star_density(p, self.rr, self.pr)

    def _star_density(self, p, rk, pk):
        g = self.gamma
        if p > pk:  # shock
            q = p / pk
            gm = (g - 1.0) / (g + 1.0)
            return rk * (q + gm) / (gm * q + 1.0)
        return rk * (p / pk) ** (1.0 / g)  # isentropic

    def wave_speeds(self):
        """Dict of the characteristic speeds bounding each wave."""
        g, ps = self.gamma, self.p_star
        out = {}
        if ps > self.pl:
            out["left_shock"] = self.ul - self.al * math.sqrt(
                (g + 1.0) / (2.0 * g) * ps / self.pl + (g - 1.0) / (2.0 * g))
        else:
            a_star = self.al * (ps / self.pl) ** ((g - 1.0) / (2.0 * g))
            out["left_head"] = self.ul - self.al
            out["left_tail"] = self.u_star - a_star
        out["contact"] = self.u_star
        if ps > self.pr:
            out["right_shock"] = self.ur + self.ar * math.sqrt(
                (g + 1.0) / (2.0 * g) * ps / self.pr + (g - 1.0) / (2.0 * g))
        else:
            a_star = self.ar * (ps / self.pr) ** ((g - 1.0) / (2.0 * g))
            out["right_tail"] = self.u_star + a_star
            out["right_head"] = self.ur + self.ar
        return out

    def max_speed(self):
        return max(abs(v) for v in self.wave_speeds().values())

    def sample(self, S):
        """(rho, u, p) at similarity coordinates S = x / t (array)."""
        S = np.atleast_1d(np.asarray(S, dtype=np.float64))
        rho, u, p = np.empty_like(S), np.empty_like(S), np.empty_like(S)
        for j, s in enumerate(S):
            rho[j], u[j], p[j] = self._sample_one(float(s))
        return rho, u, p

    def _sample_one(self, s):
        g = self.gamma
        ps, us = self.p_star, self.u_star
        if s <= us:  # left of the contact
            rk, uk, pk, ak = self.rl, self.ul, self.pl, self.al
            if ps > pk:  # left shock
                sl = uk - ak * math.sqrt((g + 1.0) / (2.0 * g) * ps / pk
                                         + (g - 1.0) / (2.0 * g))
                return (rk, uk, pk) if s <= sl else (self.rho_star_l, us, ps)
            head = uk - ak
            a_star = ak * (ps / pk) ** ((g - 1.0) / (2.0 * g))
            tail = us - a_star
            if s <= head:
                return rk, uk, pk
            if s >= tail:
                return self.rho_star_l, us, ps
            c = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * ak) * (uk - s)
            return (rk * c ** (2.0 / (g - 1.0)),
                    2.0 / (g + 1.0) * (ak + 0.5 * (g - 1.0) * uk + s),
                    pk * c ** (2.0 * g / (g - 1.0)))
        rk, uk, pk, ak = self.rr, self.ur, self.pr, self.ar
        if ps > pk:  # right shock
            sr = uk + ak * math.sqrt((g + 1.0) / (2.0 * g) * ps / pk
                                     + (g - 1.0) / (2.0 * g))
            return (rk, uk, pk) if s >= sr else (self.rho_star_r, us, ps)
        head = uk + ak
        a_star = ak * (ps / pk) ** ((g - 1.0) / (2.0 * g))
        tail = us + a_star
        if s >= head:
            return rk, uk, pk
        if s <= tail:
            return self.rho_star_r, us, ps
        c = 2.0 / (g + 1.0) - (g - 1.0) / ((g + 1.0) * ak) * (uk - s)
        return (rk * c ** (2.0 / (g - 1.0)),
                2.0 / (g + 1.0) * (-ak + 0.5 * (g - 1.0) * uk + s),
                pk * c ** (2.0 * g / (g - 1.0)))


def shock_tube_profile(left, right, gamma, nx, steps, r, x_d=None):
    """Exact (rho, u, p) at the cell centres of an nx-cell tube after
    ``steps`` lattice steps.

    Cell i spans [i, i+1); the diaphragm sits at the edge x_d = nx // 2 (cells
    i < x_d start in the left state).  A lattice step moves a population with
    velocity xi = r e by e cells, so the time after n steps is n / r in units
    where a unit velocity crosses one cell per unit time.  The paper's own
    conversion t = step / (X r) is the same with lengths scaled by X.
    """
    if x_d is None:
        x_d = nx // 2
    t = steps / r
    xc = np.arange(nx) + 0.5
    sol = RiemannSolution(left, right, gamma)
    if t == 0:
        S = np.where(xc < x_d, -np.inf, np.inf)
    else:
        S = (xc - x_d) / t
    return sol.sample(S)


def l1_errors(rho, u, p, rho_ex, u_ex, p_ex):
    """Mean absolute error per field over the cells."""
    return (float(np.mean(np.abs(rho - rho_ex))),
            float(np.mean(np.abs(u - u_ex))),
            float(np.mean(np.abs(p - p_ex))))
