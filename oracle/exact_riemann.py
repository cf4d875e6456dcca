"""Exact solution of the Riemann problem of the 1D Euler equations (ideal gas),
for the error tables of the shock-tube problems (Sec. 6).

TEST INFRASTRUCTURE ONLY.  The published method of Toro ("Riemann Solvers
and Numerical Methods for Fluid Dynamics", ch. 4): the star-region pressure
is the root of f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the shock
(Rankine-Hugoniot) branch for p > p_K and the rarefaction (isentropic)
branch otherwise; Newton iteration from the two-rarefaction estimate, then
the self-similar solution is sampled at x/t.
"""

from __future__ import annotations

import numpy as np


def _f(p, rho, pK, cK, g):
    """Velocity change across the K wave and its derivative in p."""
    if p > pK:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pK
        q = np.sqrt(A / (p + B))
        return (p - pK) * q, q * (1.0 - 0.5 * (p - pK) / (p + B))
    r = p / pK
    return (2.0 * cK / (g - 1.0)) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0), \
        (1.0 / (rho * cK)) * r ** (-(g + 1.0) / (2.0 * g))


def star_state(WL, WR, gamma: float):
    """(p*, u*) of the Riemann problem with primitive states W = (rho, u, p)."""
    g = gamma
    rl, ul, pl = WL
    rr, ur, pr = WR
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        raise ValueError("the data generate vacuum")
    z = (g - 1.0) / (2.0 * g)
    p = ((cl + cr - 0.5 * (g - 1.0) * (ur - ul)) / (cl / pl ** z + cr / pr ** z)) ** (1.0 / z)
    p = max(p, 1e-14 * min(pl, pr))
    for _ in range(200):
        fl, dl = _f(p, rl, pl, cl, g)
        fr, dr = _f(p, rr, pr, cr, g)
        pn = p - (fl + fr + ur - ul) / (dl + dr)
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= 1e-15 * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, cl, g)
    fr, _ = _f(p, rr, pr, cr, g)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(WL, WR, gamma: float, s):
    """Primitive solution (rho, u, p) at the similarity variables s = x/t."""
    g = gamma
    rl, ul, pl = WL
    rr, ur, pr = WR
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    ps, us = star_state(WL, WR, gamma)
    s = np.asarray(s, dtype=np.float64)
    rho = np.empty_like(s)
    u = np.empty_like(s)
    p = np.empty_like(s)
    gm = (g - 1.0) / (g + 1.0)
    for i, x in np.ndenumerate(s):
        if x <= us:   # left of the contact
            if ps > pl:   # left shock
                SL = ul - cl * np.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
                if x <= SL:
                    W = (rl, ul, pl)
                else:
                    W = (rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps)
            else:         # left rarefaction
                csl = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
                if x <= ul - cl:
                    W = (rl, ul, pl)
                elif x >= us - csl:
                    W = (rl * (ps / pl) ** (1.0 / g), us, ps)
                else:
                    uu = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + x)
                    cc = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - x))
                    rr_ = rl * (cc / cl) ** (2.0 / (g - 1.0))
                    W = (rr_, uu, pl * (cc / cl) ** (2.0 * g / (g - 1.0)))
        else:         # right of the contact
            if ps > pr:   # right shock
                SR = ur + cr * np.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
                if x >= SR:
                    W = (rr, ur, pr)
                else:
                    W = (rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps)
            else:         # right rarefaction
                csr = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
                if x >= ur + cr:
                    W = (rr, ur, pr)
                elif x <= us + csr:
                    W = (rr * (ps / pr) ** (1.0 / g), us, ps)
                else:
                    uu = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + x)
                    cc = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - x))
                    rr_ = rr * (cc / cr) ** (2.0 / (g - 1.0))
                    W = (rr_, uu, pr * (cc / cr) ** (2.0 * g / (g - 1.0)))
        rho[i], u[i], p[i] = W
    return rho, u, p


def solution(WL, WR, gamma: float, x, t: float, x_diaphragm: float):
    """Primitive solution at positions x and time t > 0."""
    return sample(WL, WR, gamma, (np.asarray(x, dtype=np.float64) - x_diaphragm) / t)
