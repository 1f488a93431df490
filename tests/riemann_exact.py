"""Textbook exact Riemann solver for the 1D Euler equations of an ideal gas
(two-shock/two-rarefaction pressure function with a scalar root find), used
to pin the coarse Rusanov propagator against the exact Sod solution.

For the monatomic gas of the paper's Euler limit, E = rho|u|^2/2 + 3/2 p,
i.e. gamma = 5/3 and p = rho theta.
"""
import numpy as np
from scipy.optimize import brentq


def _fk(p, rk, pk, g):
    ak = np.sqrt(g * pk / rk)
    if p > pk:
        A = 2.0 / ((g + 1) * rk)
        B = (g - 1) / (g + 1) * pk
        return (p - pk) * np.sqrt(A / (p + B))
    return 2 * ak / (g - 1) * ((p / pk) ** ((g - 1) / (2 * g)) - 1)


def star_state(L, R, g):
    rl, ul, pl = L
    rr, ur, pr = R
    fn = lambda p: _fk(p, rl, pl, g) + _fk(p, rr, pr, g) + ur - ul
    ps = brentq(fn, 1e-12, 10 * max(pl, pr), xtol=1e-15, rtol=1e-15)
    us = 0.5 * (ul + ur) + 0.5 * (_fk(ps, rr, pr, g) - _fk(ps, rl, pl, g))
    return ps, us


def sample(L, R, g, xi):
    """Density, velocity and pressure at similarity coordinate xi = (x-x0)/t."""
    rl, ul, pl = L
    rr, ur, pr = R
    ps, us = star_state(L, R, g)
    al, ar = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    gm = (g - 1) / (g + 1)
    out = np.empty((len(xi), 3))
    for n, s in enumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                rs = rl * ((ps / pl + gm) / (gm * ps / pl + 1))
                S = ul - al * np.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                out[n] = (rl, ul, pl) if s < S else (rs, us, ps)
            else:  # left rarefaction
                rs = rl * (ps / pl) ** (1 / g)
                a_s = al * (ps / pl) ** ((g - 1) / (2 * g))
                if s < ul - al:
                    out[n] = (rl, ul, pl)
                elif s > us - a_s:
                    out[n] = (rs, us, ps)
                else:
                    c = 2 / (g + 1) + gm / al * (ul - s)
                    out[n] = (rl * c ** (2 / (g - 1)),
                              2 / (g + 1) * (al + (g - 1) / 2 * ul + s),
                              pl * c ** (2 * g / (g - 1)))
        else:  # right of contact
            if ps > pr:  # right shock
                rs = rr * ((ps / pr + gm) / (gm * ps / pr + 1))
                S = ur + ar * np.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                out[n] = (rr, ur, pr) if s > S else (rs, us, ps)
            else:  # right rarefaction
                rs = rr * (ps / pr) ** (1 / g)
                a_s = ar * (ps / pr) ** ((g - 1) / (2 * g))
                if s > ur + ar:
                    out[n] = (rr, ur, pr)
                elif s < us + a_s:
                    out[n] = (rs, us, ps)
                else:
                    c = 2 / (g + 1) - gm / ar * (ur - s)
                    out[n] = (rr * c ** (2 / (g - 1)),
                              2 / (g + 1) * (-ar + (g - 1) / 2 * ur + s),
                              pr * c ** (2 * g / (g - 1)))
    return out
