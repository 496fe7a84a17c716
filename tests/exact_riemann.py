"""Exact solution of the Riemann problem of the 1D Euler equations for an
ideal gas (the textbook iterative solver: Newton iteration on the star-region
pressure, then sampling of the self-similar wave pattern; E. F. Toro,
"Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4).

Used only as an independent pin of the oracle in the pure-hydro limit.
"""
import math

import numpy as np


def _f(p, rho, pk, ck, g):
    if p > pk:  # shock
        a = 2.0 / ((g + 1.0) * rho)
        b = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(a / (p + b))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + b))
    # rarefaction
    pr = p / pk
    f = 2.0 * ck / (g - 1.0) * (pr ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho * ck) * pr ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, g):
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    p = max(1e-10, 0.5 * (pl + pr))
    for _ in range(200):
        fl, dfl = _f(p, rl, pl, cl, g)
        fr, dfr = _f(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(1e-12, p - dp)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, cl, g)
    fr, _ = _f(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(x, t, x0, left, right, g):
    """Density, velocity, pressure at positions x (array) and time t."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    out = np.empty((3, len(x)))
    for n, xi in enumerate(x):
        s = (xi - x0) / t
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= sl:
                    w = (rl, ul, pl)
                else:
                    r = rl * (ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1)
                    w = (r, us, ps)
            else:  # left rarefaction
                shl = ul - cl
                cs = cl * (ps / pl) ** ((g - 1) / (2 * g))
                stl = us - cs
                if s <= shl:
                    w = (rl, ul, pl)
                elif s >= stl:
                    w = (rl * (ps / pl) ** (1 / g), us, ps)
                else:
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    r = rl * (c / cl) ** (2 / (g - 1))
                    w = (r, u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:  # right of contact
            if ps > pr:  # right shock
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= sr:
                    w = (rr, ur, pr)
                else:
                    r = rr * (ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1)
                    w = (r, us, ps)
            else:  # right rarefaction
                shr = ur + cr
                cs = cr * (ps / pr) ** ((g - 1) / (2 * g))
                str_ = us + cs
                if s >= shr:
                    w = (rr, ur, pr)
                elif s <= str_:
                    w = (rr * (ps / pr) ** (1 / g), us, ps)
                else:
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    r = rr * (c / cr) ** (2 / (g - 1))
                    w = (r, u, pr * (c / cr) ** (2 * g / (g - 1)))
        out[:, n] = w
    return out


def cell_average_density(n, t, x0, left, right, g, sub=16):
    """Cell averages of density on n uniform cells of [0, 1] (midpoint rule
    with ``sub`` sub-samples per cell)."""
    xs = (np.arange(n * sub) + 0.5) / (n * sub)
    r = sample(xs, t, x0, left, right, g)[0]
    return r.reshape(n, sub).mean(axis=1)
