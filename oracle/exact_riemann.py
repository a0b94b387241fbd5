"""Exact solution of the 1D Riemann problem for the ideal-gas Euler equations.

Test infrastructure: it checks shock-tube runs (the Sod and Lax problems of
Sec. 4.2.1 and the seeded Riemann states) and is not part of the scheme.
The classical construction: the star-region pressure p* solves
f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the shock (Rankine-Hugoniot)
branch for p > p_K and the isentropic rarefaction branch otherwise; the
self-similar solution is then sampled at x/t.
"""
from __future__ import annotations

import math

import numpy as np


def _fK(p, rho, pk, gamma):
    """Velocity jump function of one side and its derivative in p."""
    c = math.sqrt(gamma * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (p + B))
    # rarefaction
    e = (gamma - 1.0) / (2.0 * gamma)
    return (2.0 * c / (gamma - 1.0)) * ((p / pk) ** e - 1.0), (1.0 / (rho * c)) * (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma))


def star_state(left, right, gamma=1.4, tol=1e-15, maxit=200):
    """(p*, u*) of the Riemann problem with primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    if 2.0 * (cl + cr) / (gamma - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated")
    # two-rarefaction guess, always positive
    e = (gamma - 1.0) / (2.0 * gamma)
    p = ((cl + cr - 0.5 * (gamma - 1.0) * (ur - ul)) / (cl / pl ** e + cr / pr ** e)) ** (1.0 / e)
    p = max(p, 1e-14)
    for _ in range(maxit):
        fl, dl = _fK(p, rl, pl, gamma)
        fr, dr = _fK(p, rr, pr, gamma)
        pn = p - (fl + fr + ur - ul) / (dl + dr)
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fK(p, rl, pl, gamma)
    fr, _ = _fK(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, xi, gamma=1.4):
    """Primitive solution (rho, u, p) at similarity coordinates xi = (x-x0)/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, gamma)
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    for j, s in enumerate(xi):
        if s <= us:  # left of the contact
            rho_k, u_k, p_k, sgn = rl, ul, pl, -1.0
        else:
            rho_k, u_k, p_k, sgn = rr, ur, pr, 1.0
        c_k = math.sqrt(gamma * p_k / rho_k)
        if ps > p_k:  # shock on this side
            rho_s = rho_k * (ps / p_k + g1) / (g1 * ps / p_k + 1.0)
            S = u_k + sgn * c_k * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / p_k + (gamma - 1.0) / (2.0 * gamma))
            outside = (s < S) if sgn < 0 else (s > S)
            if outside:
                rho[j], u[j], p[j] = rho_k, u_k, p_k
            else:
                rho[j], u[j], p[j] = rho_s, us, ps
        else:  # rarefaction on this side
            rho_s = rho_k * (ps / p_k) ** (1.0 / gamma)
            c_s = c_k * (ps / p_k) ** ((gamma - 1.0) / (2.0 * gamma))
            head = u_k + sgn * c_k
            tail = us + sgn * c_s
            if (sgn < 0 and s <= head) or (sgn > 0 and s >= head):
                rho[j], u[j], p[j] = rho_k, u_k, p_k
            elif (sgn < 0 and s >= tail) or (sgn > 0 and s <= tail):
                rho[j], u[j], p[j] = rho_s, us, ps
            else:  # inside the fan
                uf = 2.0 / (gamma + 1.0) * (-sgn * c_k + 0.5 * (gamma - 1.0) * u_k + s)
                # sound speed from the Riemann invariant carried across the fan
                cf = sgn * (uf - u_k) * (gamma - 1.0) / 2.0 + c_k
                rho[j] = rho_k * (cf / c_k) ** (2.0 / (gamma - 1.0))
                u[j] = uf
                p[j] = p_k * (cf / c_k) ** (2.0 * gamma / (gamma - 1.0))
    return rho, u, p


def wave_speeds(left, right, gamma=1.4):
    """Fastest left- and right-going signal speeds of the exact solution."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, gamma)
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    if ps > pl:
        sl = ul - cl * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pl + (gamma - 1.0) / (2.0 * gamma))
    else:
        sl = ul - cl
    if ps > pr:
        sr = ur + cr * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pr + (gamma - 1.0) / (2.0 * gamma))
    else:
        sr = ur + cr
    return sl, sr
