"""Exact solution of the Riemann problem for the 1-D Euler equations of an
ideal gas (textbook construction: shock / rarefaction wave curves joined at the
contact, pressure from Newton iteration, self-similar sampling in x/t).

Used as an independent check of the oracle's low-Mach shock tube; it contains
none of the lattice Boltzmann arithmetic."""
from __future__ import annotations

import math

import numpy as np


def _wave_curve(p, rho_k, p_k, c_k, g):
    """Velocity jump across the left/right wave and its derivative in p."""
    if p > p_k:  # shock (Rankine-Hugoniot)
        A = 2.0 / ((g + 1.0) * rho_k)
        B = (g - 1.0) / (g + 1.0) * p_k
        s = math.sqrt(A / (p + B))
        f = (p - p_k) * s
        df = s * (1.0 - 0.5 * (p - p_k) / (p + B))
    else:  # rarefaction (isentropic, Riemann invariant)
        e = (g - 1.0) / (2.0 * g)
        f = 2.0 * c_k / (g - 1.0) * ((p / p_k) ** e - 1.0)
        df = 1.0 / (rho_k * c_k) * (p / p_k) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, g):
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    p = 0.5 * (pl + pr)
    for _ in range(100):
        fl, dl = _wave_curve(p, rl, pl, cl, g)
        fr, dr = _wave_curve(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dl + dr)
        p = max(p - dp, 1e-12)
        if abs(dp) < 1e-14 * p:
            break
    fl, _ = _wave_curve(p, rl, pl, cl, g)
    fr, _ = _wave_curve(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(xi, rl, ul, pl, rr, ur, pr, g):
    """(rho, u, p) at similarity coordinate xi = x/t (left state assumed to the
    left of the diaphragm, left wave a rarefaction and right wave a shock when
    pl > pr, as in the tube considered)."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    cl = math.sqrt(g * pl / rl)
    out = np.zeros((3, len(xi)))
    for i, s in enumerate(xi):
        if s <= us:  # left of contact
            if ps <= pl:  # left rarefaction
                cs = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
                head, tail = ul - cl, us - cs
                if s <= head:
                    r, u, p = rl, ul, pl
                elif s >= tail:
                    r, u, p = rl * (ps / pl) ** (1.0 / g), us, ps
                else:
                    u = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s)
                    c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - s))
                    r = rl * (c / cl) ** (2.0 / (g - 1.0))
                    p = pl * (c / cl) ** (2.0 * g / (g - 1.0))
            else:
                raise NotImplementedError("left shock")
        else:  # right of contact
            if ps > pr:  # right shock
                q = ps / pr
                rs = rr * (q + (g - 1.0) / (g + 1.0)) / ((g - 1.0) / (g + 1.0) * q + 1.0)
                cr = math.sqrt(g * pr / rr)
                sh = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * q + (g - 1.0) / (2.0 * g))
                if s >= sh:
                    r, u, p = rr, ur, pr
                else:
                    r, u, p = rs, us, ps
            else:
                raise NotImplementedError("right rarefaction")
        out[:, i] = (r, u, p)
    return out


def shock_speed(rl, ul, pl, rr, ur, pr, g):
    ps, _ = star_state(rl, ul, pl, rr, ur, pr, g)
    q = ps / pr
    cr = math.sqrt(g * pr / rr)
    return ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * q + (g - 1.0) / (2.0 * g))
