"""Oracle (test infrastructure only): exact Riemann solver for the 1-D Euler
equations of an ideal gas.

Used to pin the forward scheme on a shock tube (the paper's solver is a
Godunov-type finite-volume scheme, Sec. 2.3; a Godunov scheme must converge to
the exact Riemann solution).  This is the classical construction: the star
pressure p* solves f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the shock
(Rankine-Hugoniot) branch for p > p_K and the isentropic rarefaction branch
otherwise; Newton's method from the two-rarefaction guess; then the solution
is sampled on rays x/t.
"""
from __future__ import annotations

import math

import numpy as np


def _f_and_df(p, rho, pk, ck, gamma):
    if p > pk:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (p + B))
    # rarefaction
    e = (gamma - 1.0) / (2.0 * gamma)
    f = 2.0 * ck / (gamma - 1.0) * ((p / pk) ** e - 1.0)
    df = (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma)) / (rho * ck)
    return f, df


def star_state(left, right, gamma=1.4, tol=1e-14, maxit=100):
    """(p*, u*) for left/right primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    if 2.0 * (cl + cr) / (gamma - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated")
    e = (gamma - 1.0) / (2.0 * gamma)
    p = ((cl + cr - 0.5 * (gamma - 1.0) * (ur - ul)) / (cl / pl**e + cr / pr**e)) ** (1.0 / e)
    p = max(p, tol)
    for _ in range(maxit):
        fl, dfl = _f_and_df(p, rl, pl, cl, gamma)
        fr, dfr = _f_and_df(p, rr, pr, cr, gamma)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(pn, tol)
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_and_df(p, rl, pl, cl, gamma)
    fr, _ = _f_and_df(p, rr, pr, cr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, xi, gamma=1.4):
    """Primitive solution (rho, u, p) on the rays xi = (x - x0)/t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, gamma)
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    xi = np.asarray(xi, dtype=np.float64)
    out = np.empty(xi.shape + (3,))
    for idx, s in np.ndenumerate(xi):
        if s <= us:  # left of the contact
            if ps > pl:  # left shock
                sl = ul - cl * math.sqrt((gamma + 1) / (2 * gamma) * ps / pl + (gamma - 1) / (2 * gamma))
                if s <= sl:
                    w = (rl, ul, pl)
                else:
                    w = (rl * (ps / pl + g1) / (g1 * ps / pl + 1.0), us, ps)
            else:  # left rarefaction
                head = ul - cl
                csl = cl * (ps / pl) ** ((gamma - 1) / (2 * gamma))
                tail = us - csl
                if s <= head:
                    w = (rl, ul, pl)
                elif s >= tail:
                    w = (rl * (ps / pl) ** (1.0 / gamma), us, ps)
                else:
                    c = 2.0 / (gamma + 1) * (cl + 0.5 * (gamma - 1) * (ul - s))
                    u = 2.0 / (gamma + 1) * (cl + 0.5 * (gamma - 1) * ul + s)
                    r = rl * (c / cl) ** (2.0 / (gamma - 1))
                    w = (r, u, pl * (c / cl) ** (2.0 * gamma / (gamma - 1)))
        else:  # right of the contact
            if ps > pr:  # right shock
                sr = ur + cr * math.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
                if s >= sr:
                    w = (rr, ur, pr)
                else:
                    w = (rr * (ps / pr + g1) / (g1 * ps / pr + 1.0), us, ps)
            else:  # right rarefaction
                head = ur + cr
                csr = cr * (ps / pr) ** ((gamma - 1) / (2 * gamma))
                tail = us + csr
                if s >= head:
                    w = (rr, ur, pr)
                elif s <= tail:
                    w = (rr * (ps / pr) ** (1.0 / gamma), us, ps)
                else:
                    c = 2.0 / (gamma + 1) * (cr - 0.5 * (gamma - 1) * (ur - s))
                    u = 2.0 / (gamma + 1) * (-cr + 0.5 * (gamma - 1) * ur + s)
                    r = rr * (c / cr) ** (2.0 / (gamma - 1))
                    w = (r, u, pr * (c / cr) ** (2.0 * gamma / (gamma - 1)))
        out[idx] = w
    return out


def cell_averages(left, right, x0, t, edges, gamma=1.4, sub=64):
    """Cell averages of the exact solution over cells [edges[k], edges[k+1]]
    by a midpoint rule with `sub` sub-cells per cell."""
    edges = np.asarray(edges, dtype=np.float64)
    n = len(edges) - 1
    frac = (np.arange(sub) + 0.5) / sub
    xs = edges[:-1, None] + (edges[1:] - edges[:-1])[:, None] * frac[None, :]
    w = sample(left, right, (xs - x0) / t, gamma)
    return w.reshape(n, sub, 3).mean(axis=1)
