"""Exact solution of the 1D Riemann problem of the Euler equations for an
ideal gas: the inviscid reference the paper plots beside its shock-tube
results (Sec. IV, "Riemann solution for the inviscid case").

TEST INFRASTRUCTURE ONLY (see the package docstring).

The star-region pressure p* solves f_L(p) + f_R(p) + (u_R - u_L) = 0, where
f_K is the velocity change across the left / right wave: a shock (p > p_K,
Rankine-Hugoniot) or a rarefaction (p <= p_K, isentropic with the Riemann
invariant u +- 2c/(gamma - 1) constant).  The root is bracketed and
bisected to machine precision.  The self-similar solution is then sampled at
xi = (x - x0)/t.  The standard construction of Godunov's exact solver
(e.g. E. F. Toro, Riemann Solvers and Numerical Methods for Fluid Dynamics,
ch. 4), written from its equations.
"""
import math

import numpy as np


def _wave_jump(p, rho_k, p_k, c_k, g):
    """Velocity change f_K(p) across the wave facing state K."""
    if p > p_k:                                    # shock
        a = 2.0 / ((g + 1.0) * rho_k)
        b = (g - 1.0) / (g + 1.0) * p_k
        return (p - p_k) * math.sqrt(a / (p + b))
    return 2.0 * c_k / (g - 1.0) * ((p / p_k) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def star_state(left, right, gamma=1.4):
    """(p*, u*) of the Riemann problem with states (rho, p, u)."""
    (rl, pl, ul), (rr, pr, ur) = left, right
    g = gamma
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        raise ValueError("the data generate vacuum")

    def f(p):
        return _wave_jump(p, rl, pl, cl, g) + _wave_jump(p, rr, pr, cr, g) + (ur - ul)

    lo, hi = 0.0, max(pl, pr)
    while f(hi) < 0.0:                             # f increases with p
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) < 0.0:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 1e-15 * hi:
            break
    p = 0.5 * (lo + hi)
    u = 0.5 * (ul + ur) + 0.5 * (_wave_jump(p, rr, pr, cr, g) - _wave_jump(p, rl, pl, cl, g))
    return p, u


def sample(left, right, xi, gamma=1.4):
    """(rho, u, p) at the similarity coordinates xi = (x - x0)/t (array)."""
    (rl, pl, ul), (rr, pr, ur) = left, right
    g = gamma
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, gamma)
    gm = (g - 1.0) / (g + 1.0)
    xi = np.asarray(xi, dtype=np.float64)
    rho, u, p = np.empty_like(xi), np.empty_like(xi), np.empty_like(xi)
    for k, s in np.ndenumerate(xi):
        if s <= us:                                # left of the contact
            if ps > pl:                            # left shock
                sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
                if s <= sl:
                    st = (rl, ul, pl)
                else:
                    st = (rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps)
            else:                                  # left rarefaction
                head = ul - cl
                cs = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
                tail = us - cs
                if s <= head:
                    st = (rl, ul, pl)
                elif s >= tail:
                    st = (rl * (ps / pl) ** (1.0 / g), us, ps)
                else:
                    uf = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s)
                    cf = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - s))
                    st = (rl * (cf / cl) ** (2.0 / (g - 1.0)), uf, pl * (cf / cl) ** (2.0 * g / (g - 1.0)))
        else:                                      # right of the contact
            if ps > pr:                            # right shock
                sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
                if s >= sr:
                    st = (rr, ur, pr)
                else:
                    st = (rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps)
            else:                                  # right rarefaction
                head = ur + cr
                cs = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
                tail = us + cs
                if s >= head:
                    st = (rr, ur, pr)
                elif s <= tail:
                    st = (rr * (ps / pr) ** (1.0 / g), us, ps)
                else:
                    uf = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + s)
                    cf = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - s))
                    st = (rr * (cf / cr) ** (2.0 / (g - 1.0)), uf, pr * (cf / cr) ** (2.0 * g / (g - 1.0)))
        rho[k], u[k], p[k] = st
    return rho, u, p


def wave_speeds(left, right, gamma=1.4):
    """Speeds of the left wave (its head and tail), the contact and the right
    wave (tail and head); a shock has head = tail."""
    (rl, pl, ul), (rr, pr, ur) = left, right
    g = gamma
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, gamma)
    if ps > pl:
        sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
        lw = (sl, sl)
    else:
        lw = (ul - cl, us - cl * (ps / pl) ** ((g - 1.0) / (2.0 * g)))
    if ps > pr:
        sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
        rw = (sr, sr)
    else:
        rw = (us + cr * (ps / pr) ** ((g - 1.0) / (2.0 * g)), ur + cr)
    return {"left": lw, "contact": us, "right": rw}
