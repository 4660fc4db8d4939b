"""Exact solution of the 1D Riemann problem for the ideal-gas Euler equations.

TEST INFRASTRUCTURE ONLY (used to pin the oracle and to check the GPU runs on
shock tubes; the paper compares its Riemann-problem runs with exact solutions
in Sec. 4.2.1).  Written from the mathematics of the problem: the star-region
pressure p* is the root of

    f(p) = f_L(p) + f_R(p) + (u_R - u_L) = 0,

where f_K is the Rankine-Hugoniot velocity jump across a shock (p > p_K) or
the Riemann-invariant jump across a rarefaction (p <= p_K).  f is increasing
and concave in p, so a Newton iteration kept inside a bisection bracket
converges from any start.  When u_R - u_L >= 2 (c_L + c_R) / (gamma - 1) the
two rarefactions separate and a vacuum forms between them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def _sound(gamma, rho, p):
    return math.sqrt(gamma * p / rho)


def _f_and_df(gamma, p, rho_k, p_k, c_k):
    """Velocity jump across the K-wave as a function of the star pressure."""
    if p > p_k:  # shock: Rankine-Hugoniot
        a = 2.0 / ((gamma + 1.0) * rho_k)
        b = (gamma - 1.0) / (gamma + 1.0) * p_k
        root = math.sqrt(a / (p + b))
        f = (p - p_k) * root
        df = root * (1.0 - 0.5 * (p - p_k) / (p + b))
    else:  # rarefaction: isentropic, Riemann invariant
        e = (gamma - 1.0) / (2.0 * gamma)
        f = 2.0 * c_k / (gamma - 1.0) * ((p / p_k) ** e - 1.0)
        df = 1.0 / (rho_k * c_k) * (p / p_k) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


@dataclass
class RiemannSolution:
    gamma: float
    left: tuple
    right: tuple
    vacuum: bool
    p_star: float
    u_star: float
    rho_star_l: float
    rho_star_r: float
    iterations: int

    def residual(self) -> float:
        """f_L(p*) + f_R(p*) + (u_R - u_L)."""
        g = self.gamma
        rl, ul, pl = self.left
        rr, ur, pr = self.right
        fl, _ = _f_and_df(g, self.p_star, rl, pl, _sound(g, rl, pl))
        fr, _ = _f_and_df(g, self.p_star, rr, pr, _sound(g, rr, pr))
        return fl + fr + (ur - ul)

    def sample(self, xi):
        """Primitive (rho, u, p) at similarity coordinates xi = (x - x0) / t."""
        xi = np.asarray(xi, dtype=np.float64)
        rho = np.empty_like(xi)
        u = np.empty_like(xi)
        p = np.empty_like(xi)
        for i, s in np.ndenumerate(xi):
            rho[i], u[i], p[i] = self._sample1(float(s))
        return rho, u, p

    def _sample1(self, s):
        g = self.gamma
        rl, ul, pl = self.left
        rr, ur, pr = self.right
        cl, cr = _sound(g, rl, pl), _sound(g, rr, pr)
        gm, gp = g - 1.0, g + 1.0
        if self.vacuum:
            s_hl, s_vl = ul - cl, ul + 2.0 * cl / gm
            s_hr, s_vr = ur + cr, ur - 2.0 * cr / gm
            if s <= s_hl:
                return rl, ul, pl
            if s < s_vl:
                return self._fan_left(s)
            if s <= s_vr:
                return 0.0, 0.5 * (s_vl + s_vr), 0.0
            if s < s_hr:
                return self._fan_right(s)
            return rr, ur, pr
        ps, us = self.p_star, self.u_star
        if s <= us:  # left of the contact
            if ps > pl:
                s_sh = ul - cl * math.sqrt(gp / (2 * g) * ps / pl + gm / (2 * g))
                return (rl, ul, pl) if s <= s_sh else (self.rho_star_l, us, ps)
            s_head = ul - cl
            s_tail = us - cl * (ps / pl) ** (gm / (2 * g))
            if s <= s_head:
                return rl, ul, pl
            if s >= s_tail:
                return self.rho_star_l, us, ps
            return self._fan_left(s)
        if ps > pr:
            s_sh = ur + cr * math.sqrt(gp / (2 * g) * ps / pr + gm / (2 * g))
            return (rr, ur, pr) if s >= s_sh else (self.rho_star_r, us, ps)
        s_head = ur + cr
        s_tail = us + cr * (ps / pr) ** (gm / (2 * g))
        if s >= s_head:
            return rr, ur, pr
        if s <= s_tail:
            return self.rho_star_r, us, ps
        return self._fan_right(s)

    def _fan_left(self, s):
        g = self.gamma
        rl, ul, pl = self.left
        cl = _sound(g, rl, pl)
        u = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s)
        c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - s))
        return rl * (c / cl) ** (2.0 / (g - 1.0)), u, pl * (c / cl) ** (2.0 * g / (g - 1.0))

    def _fan_right(self, s):
        g = self.gamma
        rr, ur, pr = self.right
        cr = _sound(g, rr, pr)
        u = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + s)
        c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - s))
        return rr * (c / cr) ** (2.0 / (g - 1.0)), u, pr * (c / cr) ** (2.0 * g / (g - 1.0))


def solve(left, right, gamma: float = 1.4, tol: float = 1e-15, max_iter: int = 200) -> RiemannSolution:
    """Star state of the Riemann problem with primitive states (rho, u, p)."""
    rl, ul, pl = map(float, left)
    rr, ur, pr = map(float, right)
    cl, cr = _sound(gamma, rl, pl), _sound(gamma, rr, pr)
    du = ur - ul
    if du >= 2.0 * (cl + cr) / (gamma - 1.0):
        return RiemannSolution(gamma, (rl, ul, pl), (rr, ur, pr), True, 0.0, 0.5 * (ul + ur),
                               0.0, 0.0, 0)

    def F(p):
        fl, dfl = _f_and_df(gamma, p, rl, pl, cl)
        fr, dfr = _f_and_df(gamma, p, rr, pr, cr)
        return fl + fr + du, dfl + dfr

    # bracket: f(0+) < 0 (no vacuum); grow the upper end until f > 0
    lo, hi = 0.0, max(pl, pr)
    while F(hi)[0] < 0.0:
        lo, hi = hi, 2.0 * hi
    # start from the two-rarefaction estimate, clipped into the bracket
    e = (gamma - 1.0) / (2.0 * gamma)
    num = cl + cr - 0.5 * (gamma - 1.0) * du
    den = cl / pl ** e + cr / pr ** e
    p = (num / den) ** (1.0 / e) if num > 0 else 0.5 * (lo + hi)
    if not (lo < p < hi):
        p = 0.5 * (lo + hi)
    it = 0
    for it in range(1, max_iter + 1):
        f, df = F(p)
        if f < 0.0:
            lo = p
        else:
            hi = p
        p_new = p - f / df if df > 0 else 0.5 * (lo + hi)
        if not (lo < p_new < hi):
            p_new = 0.5 * (lo + hi)
        if abs(p_new - p) <= tol * max(p_new, 1e-300) or hi - lo <= tol * hi:
            p = p_new
            break
        p = p_new
    fl, _ = _f_and_df(gamma, p, rl, pl, cl)
    fr, _ = _f_and_df(gamma, p, rr, pr, cr)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    gm, gp = gamma - 1.0, gamma + 1.0
    if p > pl:
        rsl = rl * (p / pl + gm / gp) / (gm / gp * p / pl + 1.0)
    else:
        rsl = rl * (p / pl) ** (1.0 / gamma)
    if p > pr:
        rsr = rr * (p / pr + gm / gp) / (gm / gp * p / pr + 1.0)
    else:
        rsr = rr * (p / pr) ** (1.0 / gamma)
    return RiemannSolution(gamma, (rl, ul, pl), (rr, ur, pr), False, p, u, rsl, rsr, it)


def sample_cells(left, right, gamma: float, n: int, x0: float, t: float,
                 lo: float = 0.0, hi: float = 1.0):
    """Exact (rho, u, p) at the cell centres of an n-cell grid on [lo, hi] at time t."""
    sol = solve(left, right, gamma)
    x = lo + (np.arange(n) + 0.5) * (hi - lo) / n
    return sol.sample((x - x0) / t)
