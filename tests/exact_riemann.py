"""Exact solution of the Riemann problem of the 1D Euler equations for an ideal
gas (two-wave pressure function solved by Newton iteration, then sampled
along x/t), written from the mathematics of the Riemann problem.  Used to pin
the Euler limit of the oracle (tau -> 0, gamma = 3 in 1D)."""
import math

import numpy as np


def _pressure_function(p, rho, pk, ck, g):
    """value and derivative of the wave curve f_K(p) for state K"""
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(A / (p + B))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction
    r = p / pk
    return (2.0 * ck / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0),
            r ** (-(g + 1.0) / (2.0 * g)) / (rho * ck))


def star_state(left, right, g):
    """(p*, u*) of the Riemann problem; states are (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dl = _pressure_function(p, rl, pl, cl, g)
        fr, dr = _pressure_function(p, rr, pr, cr, g)
        pn = p - (fl + fr + ur - ul) / (dl + dr)
        pn = max(pn, 1e-14)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _pressure_function(p, rl, pl, cl, g)
    fr, _ = _pressure_function(p, rr, pr, cr, g)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(left, right, g, s):
    """(rho, u, p) at similarity coordinate s = (x - x0)/t."""
    ps, us = star_state(left, right, g)
    gm = (g - 1.0) / (g + 1.0)
    if s <= us:
        rk, uk, pk = left
        ck = math.sqrt(g * pk / rk)
        if ps > pk:
            sk = uk - ck * math.sqrt((g + 1) / (2 * g) * ps / pk + (g - 1) / (2 * g))
            if s <= sk:
                return rk, uk, pk
            return rk * (ps / pk + gm) / (gm * ps / pk + 1.0), us, ps
        sh = uk - ck
        cs = ck * (ps / pk) ** ((g - 1) / (2 * g))
        st = us - cs
        if s <= sh:
            return rk, uk, pk
        if s > st:
            return rk * (ps / pk) ** (1.0 / g), us, ps
        u = 2.0 / (g + 1) * (ck + 0.5 * (g - 1) * uk + s)
        c = 2.0 / (g + 1) * (ck + 0.5 * (g - 1) * (uk - s))
        return rk * (c / ck) ** (2 / (g - 1)), u, pk * (c / ck) ** (2 * g / (g - 1))
    rk, uk, pk = right
    ck = math.sqrt(g * pk / rk)
    if ps > pk:
        sk = uk + ck * math.sqrt((g + 1) / (2 * g) * ps / pk + (g - 1) / (2 * g))
        if s >= sk:
            return rk, uk, pk
        return rk * (ps / pk + gm) / (gm * ps / pk + 1.0), us, ps
    sh = uk + ck
    cs = ck * (ps / pk) ** ((g - 1) / (2 * g))
    st = us + cs
    if s >= sh:
        return rk, uk, pk
    if s < st:
        return rk * (ps / pk) ** (1.0 / g), us, ps
    u = 2.0 / (g + 1) * (-ck + 0.5 * (g - 1) * uk + s)
    c = 2.0 / (g + 1) * (ck - 0.5 * (g - 1) * (uk - s))
    return rk * (c / ck) ** (2 / (g - 1)), u, pk * (c / ck) ** (2 * g / (g - 1))


def solution(left, right, g, x, t, x0=0.5):
    """arrays (rho, u, p) at the points x and time t > 0"""
    out = np.array([sample(left, right, g, (xi - x0) / t) for xi in np.asarray(x)])
    return out[:, 0], out[:, 1], out[:, 2]
