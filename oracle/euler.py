"""Exact solution of the Riemann problem of the 1D Euler equations of an ideal
gas (test infrastructure: only the tests use it).

The paper checks its fluid-limit Sod results (nu >> 1) against the exact
Euler solution with gamma = (d + 2)/d for a d-dimensional velocity space
(Sec. 5.1.1).  The BGK moments (n, u, theta) map to density n, velocity u
and pressure p = n theta.  This is the classical construction: the star
pressure solves f_L(p) + f_R(p) + u_R - u_L = 0, with f_K the shock
(Rankine-Hugoniot) branch for p > p_K and the rarefaction (isentropic,
Riemann-invariant) branch otherwise; the solution is then sampled along
x/t through the left wave, the contact and the right wave.
"""
from __future__ import annotations

import math

import numpy as np


def _f_and_df(p, rho, pk, gamma):
    """Velocity change across the K wave for star pressure p, and d/dp."""
    a = math.sqrt(gamma * pk / rho)
    if p > pk:                                     # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + B))
    e = (gamma - 1.0) / (2.0 * gamma)              # rarefaction
    f = 2.0 * a / (gamma - 1.0) * ((p / pk) ** e - 1.0)
    return f, (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma)) / (rho * a)


def star_state(left, right, gamma):
    """(p*, u*) of the Riemann problem; left/right = (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dl = _f_and_df(p, rl, pl, gamma)
        fr, dr = _f_and_df(p, rr, pr, gamma)
        g = fl + fr + ur - ul
        step = g / (dl + dr)
        p_new = max(1e-14, p - step)
        if abs(p_new - p) <= 1e-15 * max(p, p_new):
            p = p_new
            break
        p = p_new
    fl, _ = _f_and_df(p, rl, pl, gamma)
    fr, _ = _f_and_df(p, rr, pr, gamma)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(left, right, gamma, s):
    """(rho, u, p) at similarity coordinates s = x / t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, gamma)
    al = math.sqrt(gamma * pl / rl)
    ar = math.sqrt(gamma * pr / rr)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    s = np.asarray(s, dtype=np.float64)
    rho = np.empty_like(s)
    u = np.empty_like(s)
    p = np.empty_like(s)
    for i, x in enumerate(s.ravel()):
        if x <= us:                                   # left of the contact
            if ps > pl:                               # left shock
                rs = rl * (ps / pl + g1) / (g1 * ps / pl + 1.0)
                sl = ul - al * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pl
                                         + (gamma - 1.0) / (2.0 * gamma))
                val = (rl, ul, pl) if x <= sl else (rs, us, ps)
            else:                                     # left rarefaction
                rs = rl * (ps / pl) ** (1.0 / gamma)
                ast = al * (ps / pl) ** ((gamma - 1.0) / (2.0 * gamma))
                head, tail = ul - al, us - ast
                if x <= head:
                    val = (rl, ul, pl)
                elif x >= tail:
                    val = (rs, us, ps)
                else:
                    c = 2.0 / (gamma + 1.0) + g1 / al * (ul - x)
                    val = (rl * c ** (2.0 / (gamma - 1.0)),
                           2.0 / (gamma + 1.0) * (al + 0.5 * (gamma - 1.0) * ul + x),
                           pl * c ** (2.0 * gamma / (gamma - 1.0)))
        else:                                         # right of the contact
            if ps > pr:                               # right shock
                rs = rr * (ps / pr + g1) / (g1 * ps / pr + 1.0)
                sr = ur + ar * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pr
                                         + (gamma - 1.0) / (2.0 * gamma))
                val = (rs, us, ps) if x <= sr else (rr, ur, pr)
            else:                                     # right rarefaction
                rs = rr * (ps / pr) ** (1.0 / gamma)
                ast = ar * (ps / pr) ** ((gamma - 1.0) / (2.0 * gamma))
                head, tail = ur + ar, us + ast
                if x >= head:
                    val = (rr, ur, pr)
                elif x <= tail:
                    val = (rs, us, ps)
                else:
                    c = 2.0 / (gamma + 1.0) - g1 / ar * (ur - x)
                    val = (rr * c ** (2.0 / (gamma - 1.0)),
                           2.0 / (gamma + 1.0) * (-ar + 0.5 * (gamma - 1.0) * ur + x),
                           pr * c ** (2.0 * gamma / (gamma - 1.0)))
        rho.flat[i], u.flat[i], p.flat[i] = val
    return rho, u, p
