"""Test infrastructure (with the rest of oracle/): the oracle's reverse-mode
adjoint of a march over given states, a step at a time, each step on row
bands that run on threads.

A step's adjoint at a cell gathers the cotangents of the outputs within two
cells, and an output two or more rows inside a block of the grid is computed
there exactly as on the whole grid (its stencil never reaches the block's
own walls).  So the adjoint of a block that extends a band of rows by four
rows on each side (the walls where the grid has them) equals the whole
grid's adjoint on the band, to the bit: the block computes the same
operations in the same order (tests/test_oracle_pins.py checks both).  The
oracle's tape is per thread, and its C calls release the GIL.
"""
from __future__ import annotations

import ctypes
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from oracle.rto import Oracle, Problem

MARGIN = 4


def _block_oracle(o: Oracle, b0: int, b1: int) -> Oracle:
    p = Problem.from_buffer_copy(o.prob)
    dy = o.prob.ly / o.prob.ny
    p.ny = b1 - b0
    p.ly = (b1 - b0) * dy
    p.nb = 1
    return Oracle(p)


def banded_vjp(o: Oracle, U, dt, lam_next, band: int = 16, ex: ThreadPoolExecutor | None = None):
    """lam = (dPhi_dt/dU)(U)^T lam_next for one member ([1][4][ny][nx]) by
    bands of `band` rows."""
    ny = o.prob.ny
    U = np.ascontiguousarray(U, dtype=np.float64)
    lam_next = np.ascontiguousarray(lam_next, dtype=np.float64)
    out = np.empty_like(lam_next)
    jobs = []
    for r0 in range(0, ny, band):
        r1 = min(ny, r0 + band)
        b0, b1 = max(0, r0 - MARGIN), min(ny, r1 + MARGIN)
        jobs.append((r0, r1, b0, b1))

    def run(job):
        r0, r1, b0, b1 = job
        ob = _block_oracle(o, b0, b1)
        lb = ob.step_vjp(np.ascontiguousarray(U[:, :, b0:b1]), dt, np.ascontiguousarray(lam_next[:, :, b0:b1]))
        out[:, :, r0:r1] = lb[:, :, r0 - b0:r1 - b0]

    if ex is None:
        for j in jobs:
            run(j)
    else:
        list(ex.map(run, jobs))
    return out


def adjoint_chain(o: Oracle, state_at, dts, lam_end, workers: int = 8, band: int = 16):
    """lambda^0 from lambda^N = lam_end through the steps n = N-1 .. 0, with
    state_at(n) giving U^n ([1][4][ny][nx]) and dts[n] the step."""
    lam = np.ascontiguousarray(lam_end, dtype=np.float64)
    with ThreadPoolExecutor(workers) as ex:
        for n in range(len(dts) - 1, -1, -1):
            lam = banded_vjp(o, state_at(n), float(dts[n]), lam, band=band, ex=ex)
    return lam


def terminal_adjoint_R(o: Oracle, UN, ke0: float):
    """lambda^N = dR/dU^N of R = KE(U^N)/KE0 with KE0 fixed: (1/KE0)
    (-|m|^2/(2 rho^2), m_x/rho, m_y/rho, 0) dx dy (closed form of c-11)."""
    dV = (o.prob.lx / o.prob.nx) * (o.prob.ly / o.prob.ny)
    r, mx, my = UN[:, 0], UN[:, 1], UN[:, 2]
    u, v = mx / r, my / r
    lam = np.zeros_like(UN)
    lam[:, 0] = -0.5 * (u * u + v * v) * dV / ke0
    lam[:, 1] = u * dV / ke0
    lam[:, 2] = v * dV / ke0
    return lam


def initial_adjoint_R(o: Oracle, uv0, lam0, R: float, ke0: float):
    """dR/d(u0, v0) = rho0 (lambda_m + u0 lambda_E) - (R/KE0) rho0 u0 dx dy
    (and v), the closed form of c-11 (masked components zero)."""
    rho0, _ = o.background()
    dV = (o.prob.lx / o.prob.nx) * (o.prob.ly / o.prob.ny)
    r0 = rho0[None, :, None]
    g = np.zeros((1, 2) + lam0.shape[2:])
    for k, mask in ((0, 1), (1, 2)):
        if o.prob.comp_mask & mask:
            q = uv0[:, k]
            g[:, k] = r0 * (lam0[:, 1 + k] + q * lam0[:, 3]) - (R / ke0) * r0 * q * dV
    return g
