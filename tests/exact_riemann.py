"""Exact Riemann solver for the 1D Euler equations of an ideal gas.

Used to pin the oracle on the Sod shock tube (the paper compares its RP1 run
with the exact solution, Sec. 3.2).  Written from the textbook construction:
the star pressure is the root of f_L(p) + f_R(p) + (u_R - u_L) = 0, where
f_K is the shock (Rankine-Hugoniot) branch for p > p_K and the rarefaction
(isentropic) branch otherwise; Newton's method finds the root.  The solution
is then sampled on x/t.
"""
from __future__ import annotations

import math

import numpy as np


def _fk(p, rho, pk, g):
    a = math.sqrt(g * pk / rho)
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (p + B))
    e = (g - 1.0) / (2.0 * g)
    return 2.0 * a / (g - 1.0) * ((p / pk) ** e - 1.0), (p / pk) ** (-(g + 1.0) / (2.0 * g)) / (rho * a)


def star_state(left, right, g=1.4):
    rl, ul, pl = left
    rr, ur, pr = right
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dl = _fk(p, rl, pl, g)
        fr, dr = _fk(p, rr, pr, g)
        dp = (fl + fr + ur - ul) / (dl + dr)
        pn = max(1e-12, p - dp)
        if abs(pn - p) < 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, g)
    fr, _ = _fk(p, rr, pr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)

    def rho_star(rk, pk):
        if p > pk:
            r = (g - 1.0) / (g + 1.0)
            return rk * (p / pk + r) / (r * p / pk + 1.0)
        return rk * (p / pk) ** (1.0 / g)

    return p, u, rho_star(rl, pl), rho_star(rr, pr)


def sample(left, right, xi, g=1.4):
    """Primitive (rho, u, p) at similarity coordinates xi = (x - x_d)/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us, rsl, rsr = star_state(left, right, g)
    al, ar = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    out = np.zeros((np.size(xi), 3))
    for k, s in enumerate(np.atleast_1d(xi)):
        if s <= us:   # left of the contact
            if ps > pl:
                sl = ul - al * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                out[k] = (rl, ul, pl) if s < sl else (rsl, us, ps)
            else:
                asl = al * (ps / pl) ** ((g - 1) / (2 * g))
                if s < ul - al:
                    out[k] = (rl, ul, pl)
                elif s > us - asl:
                    out[k] = (rsl, us, ps)
                else:
                    c = 2 / (g + 1) * (al + (g - 1) / 2 * (ul - s))
                    uu = 2 / (g + 1) * (al + (g - 1) / 2 * ul + s)
                    out[k] = (rl * (c / al) ** (2 / (g - 1)), uu, pl * (c / al) ** (2 * g / (g - 1)))
        else:
            if ps > pr:
                sr = ur + ar * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                out[k] = (rr, ur, pr) if s > sr else (rsr, us, ps)
            else:
                asr = ar * (ps / pr) ** ((g - 1) / (2 * g))
                if s > ur + ar:
                    out[k] = (rr, ur, pr)
                elif s < us + asr:
                    out[k] = (rsr, us, ps)
                else:
                    c = 2 / (g + 1) * (ar - (g - 1) / 2 * (ur - s))
                    uu = 2 / (g + 1) * (-ar + (g - 1) / 2 * ur + s)
                    out[k] = (rr * (c / ar) ** (2 / (g - 1)), uu, pr * (c / ar) ** (2 * g / (g - 1)))
    return out
