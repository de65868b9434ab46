"""Carnahan-Starling thermodynamics for the oracle's tests: critical point and Maxwell coexistence.

TEST INFRASTRUCTURE ONLY (see ``oracle.py``).

p(rho) = rho R T (1 + eta + eta^2 - eta^3) / (1 - eta)^3 - a rho^2, eta = b rho / 4.
The critical point solves p' = p'' = 0; coexistence solves equal pressure and equal chemical
potential (the Maxwell equal-area construction named in Sec. 4, after eq. 19).
"""
from __future__ import annotations

import mpmath
import sympy as sp
from scipy.optimize import brentq


def p_cs(rho, T, a=1.0, b=4.0, R=1.0):
    eta = b * rho / 4.0
    return rho * R * T * (1 + eta + eta**2 - eta**3) / (1 - eta) ** 3 - a * rho**2


def critical_point(a=1.0, b=4.0, R=1.0):
    """(rho_c, T_c) from dp/drho = d2p/drho2 = 0, solved symbolically-numerically to 30 digits."""
    r, T = sp.symbols("r T", positive=True)
    eta = b * r / 4
    P = r * R * T * (1 + eta + eta**2 - eta**3) / (1 - eta) ** 3 - a * r**2
    sol = sp.nsolve([sp.diff(P, r), sp.diff(P, r, 2)], [r, T], [0.13 * 4 / b, 0.0943 * a / b * 4], prec=30)
    return float(sol[0]), float(sol[1])


def spinodal(T, a=1.0, b=4.0, R=1.0):
    """The two zeros of dp/drho bracketing the unstable branch."""
    rc, Tc = critical_point(a, b, R)
    h = 1e-7
    dp = lambda r: (p_cs(r + h, T, a, b, R) - p_cs(r - h, T, a, b, R)) / (2 * h)
    lo = brentq(dp, 1e-6, rc)
    hi = brentq(dp, rc, 0.99 * 4 / b)
    return lo, hi


def maxwell(T, a=1.0, b=4.0, R=1.0):
    """Coexisting (rho_v, rho_l): p(rho_v) = p(rho_l) = p_sat and int_{rho_v}^{rho_l} (p - p_sat) / rho^2 drho = 0
    (equal areas in the p-v plane, v = 1/rho).  Bisection on p_sat between the spinodal pressures."""
    s_lo, s_hi = spinodal(T, a, b, R)
    p = lambda r: p_cs(r, T, a, b, R)
    r_top = 0.999 * 4 / b
    while p(r_top) < p(s_lo):
        r_top = 0.5 * (r_top + 4 / b)

    def branches(ps):
        rv = brentq(lambda r: p(r) - ps, 1e-300 if ps > 0 else 1e-12, s_lo, xtol=1e-300, rtol=1e-15)
        rl = brentq(lambda r: p(r) - ps, s_hi, r_top, xtol=1e-300, rtol=1e-15)
        return rv, rl

    # closed-form antiderivative of p / rho^2 (sympy), so the area needs no quadrature; its
    # logarithms of (rho - 1) carry the same imaginary part at both ends, which cancels
    r, Ts = sp.symbols("r T", positive=True)
    eta = sp.nsimplify(b) * r / 4
    expr = (r * sp.nsimplify(R) * Ts * (1 + eta + eta**2 - eta**3) / (1 - eta) ** 3 - sp.nsimplify(a) * r**2) / r**2
    prim = sp.lambdify((r, Ts), sp.integrate(sp.apart(sp.cancel(expr), r), r), "mpmath")
    Tm = mpmath.mpf(T)

    def area(ps):
        rv, rl = branches(ps)
        return float(mpmath.re(prim(mpmath.mpf(rl), Tm) - prim(mpmath.mpf(rv), Tm))) - ps * (1.0 / rv - 1.0 / rl)

    p_hi = p(s_lo)
    p_lo = max(p(s_hi), 1e-300)
    ps = brentq(area, p_lo * (1 + 1e-12) + 1e-300, p_hi * (1 - 1e-12), xtol=1e-300, rtol=1e-15)
    rv, rl = branches(ps)
    return float(rv), float(rl)


def rho_max(T, a=1.0, b=4.0, R=1.0):
    """Largest density for which the pseudopotential is real: rho/3 - p(rho) >= 0 (G = -1)."""
    g = lambda r: r / 3.0 - p_cs(r, T, a, b, R)
    _, s_hi = spinodal(T, a, b, R)
    return brentq(g, s_hi, 0.999 * 4 / b)
