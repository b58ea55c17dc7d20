"""ORACLE — test infrastructure, not product code.

Exact solution of the Riemann problem of the one-dimensional Euler equations
of an ideal gas (the B = 0 limit of the ideal-MHD system of the paper's
Eq. (mhd) with the EOS of Eq. (Energy)). Used to pin the scheme on shock-tube
problems. Written from the classical construction (two nonlinear waves, each
a shock or a rarefaction, around a contact): the star pressure is the root of
f_L(p) + f_R(p) + (u_R - u_L) = 0, found by Newton iteration, and the
solution is sampled along x/t.

Pinned in the tests by the Rankine-Hugoniot jump conditions across each shock
and by the Riemann invariants across each rarefaction.
"""
from __future__ import annotations

import math

import numpy as np


def _f_and_df(p, rho_k, p_k, c_k, g):
    """Velocity change across the k-wave as a function of the star pressure."""
    if p > p_k:  # shock: from the Rankine-Hugoniot conditions
        A = 2.0 / ((g + 1.0) * rho_k)
        B = (g - 1.0) / (g + 1.0) * p_k
        s = math.sqrt(A / (p + B))
        f = (p - p_k) * s
        df = s * (1.0 - 0.5 * (p - p_k) / (p + B))
    else:  # rarefaction: isentropic, Riemann invariant conserved
        pr = p / p_k
        f = 2.0 * c_k / (g - 1.0) * (pr ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho_k * c_k) * pr ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, g):
    """Return (p*, u*) of the Riemann problem."""
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated")
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(200):
        fl, dfl = _f_and_df(p, rl, pl, cl, g)
        fr, dfr = _f_and_df(p, rr, pr, cr, g)
        step = (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(1e-14, p - step)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_and_df(p, rl, pl, cl, g)
    fr, _ = _f_and_df(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(rl, ul, pl, rr, ur, pr, g, xi):
    """(rho, u, p) at similarity coordinates xi = (x - x0) / t (array)."""
    xi = np.asarray(xi, dtype=np.float64)
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    out = np.zeros((3,) + xi.shape)
    gm = (g - 1.0) / (g + 1.0)
    for idx, s in np.ndenumerate(xi):
        if s <= us:  # left of the contact
            if ps > pl:  # left shock
                rs = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
                sl = ul - cl * math.sqrt((g + 1.0) / (2 * g) * ps / pl + (g - 1.0) / (2 * g))
                val = (rl, ul, pl) if s <= sl else (rs, us, ps)
            else:  # left rarefaction
                rs = rl * (ps / pl) ** (1.0 / g)
                cs = cl * (ps / pl) ** ((g - 1.0) / (2 * g))
                shead, stail = ul - cl, us - cs
                if s <= shead:
                    val = (rl, ul, pl)
                elif s >= stail:
                    val = (rs, us, ps)
                else:
                    u = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s)
                    c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - s))
                    r = rl * (c / cl) ** (2.0 / (g - 1.0))
                    val = (r, u, pl * (c / cl) ** (2.0 * g / (g - 1.0)))
        else:  # right of the contact
            if ps > pr:  # right shock
                rs = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
                sr = ur + cr * math.sqrt((g + 1.0) / (2 * g) * ps / pr + (g - 1.0) / (2 * g))
                val = (rr, ur, pr) if s >= sr else (rs, us, ps)
            else:  # right rarefaction
                rs = rr * (ps / pr) ** (1.0 / g)
                cs = cr * (ps / pr) ** ((g - 1.0) / (2 * g))
                shead, stail = ur + cr, us + cs
                if s >= shead:
                    val = (rr, ur, pr)
                elif s <= stail:
                    val = (rs, us, ps)
                else:
                    u = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + s)
                    c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - s))
                    r = rr * (c / cr) ** (2.0 / (g - 1.0))
                    val = (r, u, pr * (c / cr) ** (2.0 * g / (g - 1.0)))
        out[(slice(None),) + idx] = val
    return out


def wave_structure(rl, ul, pl, rr, ur, pr, g):
    """Star state plus the density on each side of the contact and the wave
    speeds (shock speed, or rarefaction head/tail), for the jump-condition pins."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    gm = (g - 1.0) / (g + 1.0)
    res = {"p": ps, "u": us}
    if ps > pl:
        res["rho_l"] = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
        res["left"] = ("shock", ul - cl * math.sqrt((g + 1.0) / (2 * g) * ps / pl + (g - 1.0) / (2 * g)))
    else:
        res["rho_l"] = rl * (ps / pl) ** (1.0 / g)
        res["left"] = ("rarefaction", ul - cl, us - cl * (ps / pl) ** ((g - 1.0) / (2 * g)))
    if ps > pr:
        res["rho_r"] = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
        res["right"] = ("shock", ur + cr * math.sqrt((g + 1.0) / (2 * g) * ps / pr + (g - 1.0) / (2 * g)))
    else:
        res["rho_r"] = rr * (ps / pr) ** (1.0 / g)
        res["right"] = ("rarefaction", ur + cr, us + cr * (ps / pr) ** ((g - 1.0) / (2 * g)))
    return res
