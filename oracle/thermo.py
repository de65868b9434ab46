"""Carnahan-Starling thermodynamics for the oracle's tests: critical point and Maxwell coexistence.

TEST INFRASTRUCTURE ONLY (see ``oracle.py``).

p(rho) = rho R T (1 + eta + eta^2 - eta^3) / (1 - eta)^3 - a rho^2, eta = b rho / 4.
The critical point solves p' = p'' = 0; coexistence solves equal pressure and equal chemical
potential (the Maxwell equal-area construction named in Sec. 4, after eq. 19).
"""
from __future__ import annotations

import functools
import warnings

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


# ---------------------------------------------------------------- Peng-Robinson (eq. 10)
PR_A, PR_B, PR_R, PR_OMEGA = 2.0 / 49.0, 2.0 / 21.0, 1.0, 0.344  # Sec. 2.2: a, b, R, water


@functools.lru_cache(maxsize=None)
def critical_point_pr(a=PR_A, b=PR_B, R=PR_R):
    """(rho_c, T_c) of eq. 10 with alpha = 1: dp/drho = d2p/drho2 = 0, solved to 30 digits."""
    r, T = sp.symbols("r T", positive=True)
    bb, aa, RR = sp.nsimplify(b), sp.nsimplify(a), sp.nsimplify(R)
    P = r * RR * T / (1 - bb * r) - aa * r**2 / (1 + 2 * bb * r - bb**2 * r**2)
    sol = sp.nsolve([sp.diff(P, r), sp.diff(P, r, 2)], [r, T], [0.25 / b, 0.17 * a / (b * R)], prec=30)
    return float(sol[0]), float(sol[1])


def alpha_pr(T, Tc, omega=PR_OMEGA):
    m = 0.37464 + 1.54226 * omega - 0.26992 * omega**2
    return (1.0 + m * (1.0 - (T / Tc) ** 0.5)) ** 2


def p_pr(rho, T, a=PR_A, b=PR_B, R=PR_R, omega=PR_OMEGA):
    _, Tc = critical_point_pr(a, b, R)
    aa = a * alpha_pr(T, Tc, omega)
    return rho * R * T / (1 - b * rho) - aa * rho**2 / (1 + 2 * b * rho - (b * rho) ** 2)


def maxwell_pr(T, a=PR_A, b=PR_B, R=PR_R, omega=PR_OMEGA):
    """Coexisting (rho_v, rho_l) of eq. 10 by the equal-area rule in the p-v plane, from the
    pressure alone (numerical quadrature): no chemical potential enters."""
    from scipy.integrate import quad

    rc, Tc = critical_point_pr(a, b, R)
    aa = a * alpha_pr(T, Tc, omega)
    p = lambda r: r * R * T / (1 - b * r) - aa * r**2 / (1 + 2 * b * r - (b * r) ** 2)
    h = 1e-7
    dp = lambda r: (p(r + h) - p(r - h)) / (2 * h)
    s_lo = brentq(dp, 1e-6, rc)
    s_hi = brentq(dp, rc, 0.999 / b)

    def branches(ps):
        rv = brentq(lambda r: p(r) - ps, 1e-200, s_lo, xtol=1e-300, rtol=1e-15)
        rl = brentq(lambda r: p(r) - ps, s_hi, 0.999999 / b, xtol=1e-300, rtol=1e-15)
        return rv, rl

    def area(ps):
        rv, rl = branches(ps)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")  # quad flags roundoff near the root; the root is still found
            val, _ = quad(lambda r: (p(r) - ps) / r**2, rv, rl, epsabs=1e-15, epsrel=1e-13, limit=200)
        return val

    p_hi = p(s_lo)
    p_lo = max(p(s_hi), 1e-14)
    ps = brentq(area, p_lo * (1 + 1e-12), p_hi * (1 - 1e-12), xtol=1e-300, rtol=1e-14)
    rv, rl = branches(ps)
    return float(rv), float(rl)
