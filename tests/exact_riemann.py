"""Exact Riemann solutions used to pin the oracle (test side only).

Euler: the exact solver of E. F. Toro, "Riemann Solvers and Numerical Methods for Fluid
Dynamics" (3rd ed., Springer 2009), Chapter 4: the star pressure is the root of the
pressure function f(p) = f_L(p) + f_R(p) + (u_R - u_L), with the shock branch
f_K = (p - p_K) sqrt(A_K / (p + B_K)) and the rarefaction branch
f_K = 2 c_K / (gamma - 1) ((p / p_K)^((gamma - 1) / (2 gamma)) - 1); the solution is then
sampled in x/t.

Burgers: the entropy solution of u_t + (u^2/2)_x = 0 with a jump (shock at speed
(uL + uR)/2 when uL > uR, rarefaction fan u = x/t when uL < uR).
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq


def _fK(p, rhoK, pK, cK, g):
    if p > pK:
        A = 2.0 / ((g + 1.0) * rhoK)
        B = (g - 1.0) / (g + 1.0) * pK
        return (p - pK) * np.sqrt(A / (p + B))
    return 2.0 * cK / (g - 1.0) * ((p / pK) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def euler_star(left, right, gamma=1.4):
    """Star-region pressure and velocity (p*, u*) and densities (rho*_L, rho*_R)."""
    rL, uL, pL = left
    rR, uR, pR = right
    g = gamma
    cL = np.sqrt(g * pL / rL)
    cR = np.sqrt(g * pR / rR)
    f = lambda p: _fK(p, rL, pL, cL, g) + _fK(p, rR, pR, cR, g) + (uR - uL)
    ps = brentq(f, 1e-12, 100.0 * max(pL, pR), xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (uL + uR) + 0.5 * (_fK(ps, rR, pR, cR, g) - _fK(ps, rL, pL, cL, g))
    gr = (g - 1.0) / (g + 1.0)
    if ps > pL:
        rsL = rL * (ps / pL + gr) / (gr * ps / pL + 1.0)
    else:
        rsL = rL * (ps / pL) ** (1.0 / g)
    if ps > pR:
        rsR = rR * (ps / pR + gr) / (gr * ps / pR + 1.0)
    else:
        rsR = rR * (ps / pR) ** (1.0 / g)
    return ps, us, rsL, rsR


def euler_sample(left, right, xi, gamma=1.4):
    """Exact (rho, u, p) at similarity coordinates xi = (x - x0) / t (numpy array)."""
    rL, uL, pL = left
    rR, uR, pR = right
    g = gamma
    cL = np.sqrt(g * pL / rL)
    cR = np.sqrt(g * pR / rR)
    ps, us, rsL, rsR = euler_star(left, right, gamma)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for n, s in enumerate(xi.flat):
        if s <= us:
            if ps > pL:  # left shock
                SL = uL - cL * np.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
                val = (rL, uL, pL) if s <= SL else (rsL, us, ps)
            else:  # left rarefaction
                csL = cL * (ps / pL) ** ((g - 1) / (2 * g))
                SHL, STL = uL - cL, us - csL
                if s <= SHL:
                    val = (rL, uL, pL)
                elif s >= STL:
                    val = (rsL, us, ps)
                else:
                    uu = 2 / (g + 1) * (cL + (g - 1) / 2 * uL + s)
                    cc = 2 / (g + 1) * (cL + (g - 1) / 2 * (uL - s))
                    rr = rL * (cc / cL) ** (2 / (g - 1))
                    val = (rr, uu, pL * (cc / cL) ** (2 * g / (g - 1)))
        else:
            if ps > pR:  # right shock
                SR = uR + cR * np.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
                val = (rR, uR, pR) if s >= SR else (rsR, us, ps)
            else:  # right rarefaction
                csR = cR * (ps / pR) ** ((g - 1) / (2 * g))
                SHR, STR = uR + cR, us + csR
                if s >= SHR:
                    val = (rR, uR, pR)
                elif s <= STR:
                    val = (rsR, us, ps)
                else:
                    uu = 2 / (g + 1) * (-cR + (g - 1) / 2 * uR + s)
                    cc = 2 / (g + 1) * (cR - (g - 1) / 2 * (uR - s))
                    rr = rR * (cc / cR) ** (2 / (g - 1))
                    val = (rr, uu, pR * (cc / cR) ** (2 * g / (g - 1)))
        rho.flat[n], u.flat[n], p.flat[n] = val
    return rho, u, p


def euler_wave_positions(left, right, t, x0=0.5, gamma=1.4):
    """Sod-type positions at time t: rarefaction head, tail, contact, shock."""
    rL, uL, pL = left
    rR, uR, pR = right
    g = gamma
    cL = np.sqrt(g * pL / rL)
    cR = np.sqrt(g * pR / rR)
    ps, us, rsL, rsR = euler_star(left, right, gamma)
    csL = cL * (ps / pL) ** ((g - 1) / (2 * g))
    SR = uR + cR * np.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
    return (x0 + (uL - cL) * t, x0 + (us - csL) * t, x0 + us * t, x0 + SR * t)


def burgers_sample(uL, uR, xi):
    """Entropy solution of the Burgers Riemann problem at xi = (x - x0) / t."""
    xi = np.asarray(xi, dtype=np.float64)
    if uL > uR:
        s = 0.5 * (uL + uR)
        return np.where(xi < s, uL, uR)
    return np.where(xi <= uL, uL, np.where(xi >= uR, uR, xi))


def swe_dam_break(hL, hR, xi, g=9.81):
    """Exact wet-bed dam break of the shallow-water equations (h_L > h_R > 0, both at rest) at
    xi = (x - x0) / t: a left rarefaction and a right shock around the middle state (h_m, u_m).
    The rarefaction gives u_m = 2 (c_L - c_m) (c = sqrt(g h)), the shock
    u_m = (h_m - h_R) sqrt(g (1/h_m + 1/h_R) / 2); h_m is found by bisection. Returns
    (h, u, h_m, u_m, shock speed)."""
    cL = np.sqrt(g * hL)

    def f(hm):
        return 2.0 * (cL - np.sqrt(g * hm)) - (hm - hR) * np.sqrt(0.5 * g * (1.0 / hm + 1.0 / hR))

    lo, hi = hR, hL
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    hm = 0.5 * (lo + hi)
    cm = np.sqrt(g * hm)
    um = 2.0 * (cL - cm)
    S = hm * um / (hm - hR)
    xi = np.asarray(xi, dtype=np.float64)
    c_fan = (2.0 * cL - xi) / 3.0
    h = np.where(xi < -cL, hL, np.where(xi < um - cm, c_fan * c_fan / g, np.where(xi < S, hm, hR)))
    u = np.where(xi < -cL, 0.0, np.where(xi < um - cm, 2.0 * (cL - c_fan), np.where(xi < S, um, 0.0)))
    return h, u, hm, um, S
