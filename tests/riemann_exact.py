"""Exact solution of the 1D Riemann problem for an ideal gas (the classic
two-rarefaction/two-shock pressure iteration), used to pin the shock-tube run."""
import math

import numpy as np


def _fk(p, rho, pk, ck, g):
    if p > pk:   # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        f = (p - pk) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - (p - pk) / (2.0 * (B + p)))
    else:        # rarefaction
        f = 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * ck) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(L, R, g=1.4):
    rl, ul, pl = L
    rr, ur, pr = R
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dfl = _fk(p, rl, pl, cl, g)
        fr, dfr = _fk(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        p_new = max(1e-10, p - dp)
        if abs(p_new - p) < 1e-14 * p:
            p = p_new
            break
        p = p_new
    fl, _ = _fk(p, rl, pl, cl, g)
    fr, _ = _fk(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(L, R, s, g=1.4):
    """state (rho, u, p) at similarity coordinate s = x/t"""
    rl, ul, pl = L
    rr, ur, pr = R
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star_state(L, R, g)
    gm = (g - 1.0) / (g + 1.0)
    if s <= us:
        if ps > pl:
            rs = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
            sh = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
            return (rl, ul, pl) if s < sh else (rs, us, ps)
        rs = rl * (ps / pl) ** (1.0 / g)
        cs = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
        if s < ul - cl:
            return (rl, ul, pl)
        if s > us - cs:
            return (rs, us, ps)
        u = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * ul + s)
        c = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * (ul - s))
        rho = rl * (c / cl) ** (2.0 / (g - 1.0))
        return (rho, u, pl * (c / cl) ** (2.0 * g / (g - 1.0)))
    if ps > pr:
        rs = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
        sh = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
        return (rr, ur, pr) if s > sh else (rs, us, ps)
    rs = rr * (ps / pr) ** (1.0 / g)
    cs = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
    if s > ur + cr:
        return (rr, ur, pr)
    if s < us + cs:
        return (rs, us, ps)
    u = 2.0 / (g + 1.0) * (-cr + (g - 1.0) / 2.0 * ur + s)
    c = 2.0 / (g + 1.0) * (cr - (g - 1.0) / 2.0 * (ur - s))
    rho = rr * (c / cr) ** (2.0 / (g - 1.0))
    return (rho, u, pr * (c / cr) ** (2.0 * g / (g - 1.0)))


def density_cell_averages(L, R, x0, x1, n, xd, t, g=1.4, sub=64):
    dx = (x1 - x0) / n
    out = np.empty(n)
    for i in range(n):
        xs = x0 + (i + (np.arange(sub) + 0.5) / sub) * dx
        out[i] = np.mean([sample(L, R, (x - xd) / t, g)[0] for x in xs])
    return out
