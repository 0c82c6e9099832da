"""Projected L-BFGS with a non-monotone Armijo line search (Sec. 3.4).

The paper maximises its objective over the constraint set with a projected
limited-memory quasi-Newton method: a search direction from the m most
recent displacement / gradient-change pairs (m = 10, Tab. params), a trial
point rescaled onto the constraint set by the projection P of Eq. 11, and a
non-monotone Armijo backtracking line search that tolerates temporary
decreases; convergence is followed through the stationarity measure chi of
Appendix A.  This module states that method for the maximisation of f:

    g_k   = grad f(x_k)
    d_k   = H_k g_k            (two-loop recursion on the pairs (s_i, y_i) of
                                the ascent problem: s = x_{i+1} - x_i,
                                y = g_i - g_{i+1}; a pair enters only if
                                <s, y> > 0; H_0 = <s, y>/<y, y> of the newest
                                pair, or a scaled gradient step without pairs)
    x+    = P(x_k + lam d_k),  lam = 1, 1/2, 1/4, ...
    accept when f(x+) >= min(f of the last M accepted iterates)
                          + c <g_k, x+ - x_k>
    chi_k = || P(x_k + g_k) - x_k ||_inf

Every member of a batch is an independent problem; scalars are per member
(numpy arrays of length B).  Field arithmetic goes through a backend object,
so the same code runs on the HIP library's device fields and, in the tests,
on numpy arrays:

    backend.dot(a, b) -> [B]           backend.axpy(x, alpha[B], y) -> x + alpha y
    backend.project(x) -> P(x)         backend.max_abs(x) -> [B]
    backend.where(mask[B], a, b)       backend.value(x) -> f[B]
    backend.value_and_grad(x) -> (f[B], grad f)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class LBFGSLog:
    f: list = field(default_factory=list)          # [iter][B] accepted objective
    chi: list = field(default_factory=list)        # [iter][B] stationarity measure
    grad_norm: list = field(default_factory=list)  # [iter][B] Euclidean norm of the gradient
    backtracks: list = field(default_factory=list) # [iter][B]
    resets: list = field(default_factory=list)     # [iter][B] memory dropped (no ascent direction)
    evals: int = 0
    grads: int = 0


class _Memory:
    """Curvature pairs of every member, kept apart per member.

    Pairs are stored batched (one field per pair for all members) with a
    per-member validity mask; a pair that is not valid for a member enters
    its recursion with rho = 0 and contributes an exact zero.  Each member
    keeps its own `memory` newest valid pairs (the oldest of its own goes
    first) and takes H0 from its own newest valid pair, so a member's
    search direction is the one it would get searching alone."""

    def __init__(self, memory: int, B: int):
        self.memory, self.B = memory, B
        self.pairs = []  # (s, y, rho[B], valid[B], sy[B], yy[B]), oldest first

    def has(self) -> np.ndarray:
        out = np.zeros(self.B, dtype=bool)
        for *_, valid, _, _ in self.pairs:
            out |= valid
        return out

    def drop(self, members: np.ndarray):
        """Forget every pair of the members where `members` is True."""
        for k, (s, y, rho, valid, sy, yy) in enumerate(self.pairs):
            keep = valid & ~members
            self.pairs[k] = (s, y, np.where(keep, rho, 0.0), keep, sy, yy)
        self._compact()

    def push(self, be, s, y, good: np.ndarray, sy: np.ndarray, yy: np.ndarray):
        """Append (s, y) for the members where good is True (the other
        members' entries are stored as zeros)."""
        if self.memory <= 0 or not good.any():
            return
        s = be.where(good, s, be.axpy(s, -1.0, s))
        y = be.where(good, y, be.axpy(y, -1.0, y))
        self.pairs.append((s, y, np.where(good, 1.0 / np.where(good, sy, 1.0), 0.0), good.copy(), sy, yy))
        count = np.zeros(self.B, dtype=int)
        for *_, valid, _, _ in self.pairs:
            count += valid
        for k, (s_, y_, rho, valid, sy_, yy_) in enumerate(self.pairs):
            over = valid & (count > self.memory)  # this member's oldest pair beyond its memory
            if over.any():
                self.pairs[k] = (s_, y_, np.where(over, 0.0, rho), valid & ~over, sy_, yy_)
                count -= over
        self._compact()

    def _compact(self):
        self.pairs = [p for p in self.pairs if p[3].any()]

    def gamma(self) -> np.ndarray:
        """H0 = <s, y>/<y, y> of each member's newest valid pair (0 without)."""
        g = np.zeros(self.B)
        seen = np.zeros(self.B, dtype=bool)
        for *_, valid, sy, yy in reversed(self.pairs):
            new = valid & ~seen
            g = np.where(new, sy / np.where(yy > 0.0, yy, 1.0) * (yy > 0.0), g)
            seen |= valid
        return g

    def two_loop(self, be, g):
        """H g for the ascent problem (two-loop recursion, newest pair first)."""
        q = g
        alphas = []
        for s, y, rho, *_ in reversed(self.pairs):
            a = rho * be.dot(s, q)
            alphas.append(a)
            q = be.axpy(q, -a, y)
        r = be.axpy(q, self.gamma() - 1.0, q)  # gamma * q
        for (s, y, rho, *_), a in zip(self.pairs, reversed(alphas)):
            b = rho * be.dot(y, r)
            r = be.axpy(r, a - b, s)
        return r


def lbfgs_max(be, x0, iters: int, memory: int = 10, nonmonotone: int = 10, c_armijo: float = 1e-4,
              max_backtracks: int = 12, on_iter=None, log: LBFGSLog | None = None, grad_at_trials: bool = True):
    """Maximise f over the constraint set from x0 (projected first).
    Returns (x, f[B], g, log).  grad_at_trials: each trial point is
    evaluated with its gradient (the accepted one's is the next iterate's),
    else with f alone and the gradient afterwards at the accepted point; the
    iterates are the same (the backend's f must be the same in both).

    Safeguards (per member): the quasi-Newton direction is replaced by a
    gradient step, and the memory dropped, when the projected step
    P(x + d) - x is not an ascent direction (<g, P(x + d) - x> <= 0); a line
    search that finds no acceptable point within max_backtracks halvings
    leaves x unchanged and drops the memory.  Without memory the step is a
    gradient step scaled by the Barzilai-Borwein length <s, s>/|<s, y>| of
    the last move (0.1 ||x|| / ||g|| before the first, 1 / ||g|| at x = 0)."""
    log = log or LBFGSLog()
    x = be.project(x0)
    f, g = be.value_and_grad(x)
    log.grads += 1
    B = len(f)
    hist = [f.copy()]
    mem = _Memory(memory, B)
    gn = np.maximum(np.sqrt(be.dot(g, g)), 1e-300)
    xn = np.sqrt(be.dot(x, x))
    step0 = np.where(xn > 0.0, 0.1 * xn, 1.0) / gn
    for it in range(iters):
        d = be.axpy(g, step0 - 1.0, g)  # step0 * g
        reset = np.zeros(B, dtype=bool)
        have = mem.has()  # member has curvature pairs in memory
        if have.any():
            dq = mem.two_loop(be, g)
            ok = have & (be.dot(g, be.axpy(be.project(be.axpy(x, 1.0, dq)), -1.0, x)) > 0.0)
            reset = have & ~ok
            d = be.where(ok, dq, d)
        ref = np.min(np.stack(hist[-nonmonotone:]), axis=0)
        lam = np.ones(B)
        accepted = np.zeros(B, dtype=bool)
        x_new, f_new, g_new = x, f.copy(), g
        nback = np.zeros(B, dtype=int)
        for bt in range(max_backtracks + 1):
            trial = be.project(be.axpy(x, lam, d))
            if grad_at_trials:
                ft, gt = be.value_and_grad(trial)
                log.grads += 1
            else:
                ft = be.value(trial)
                log.evals += 1
            gd = be.dot(g, be.axpy(trial, -1.0, x))
            ok = ~accepted & (ft >= ref + c_armijo * gd)
            if ok.any():
                x_new = be.where(ok, trial, x_new)
                f_new = np.where(ok, ft, f_new)
                if grad_at_trials:
                    g_new = be.where(ok, gt, g_new)
                accepted |= ok
            if accepted.all():
                break
            nback += ~accepted
            lam = np.where(accepted, lam, 0.5 * lam)
        failed = ~accepted
        if grad_at_trials:
            f2, g2 = f_new, g_new  # a member that found no point keeps x, f and g
        else:
            f2, g2 = be.value_and_grad(x_new)
            log.grads += 1
        s = be.axpy(x_new, -1.0, x)
        y = be.axpy(g, -1.0, g2)  # gradient change of the minimisation of -f
        ss, sy, yy = be.dot(s, s), be.dot(s, y), be.dot(y, y)
        good = accepted & (sy > 1e-12 * np.sqrt(ss * yy))
        drop = reset | failed
        if drop.any():
            mem.drop(drop)
        mem.push(be, s, y, good, sy, yy)
        # Barzilai-Borwein length for the next gradient step
        gn2 = np.sqrt(be.dot(g2, g2))
        base = np.sqrt(be.dot(x_new, x_new)) / np.maximum(gn2, 1e-300)
        bb = ss / np.maximum(np.abs(sy), 1e-300)
        step0 = np.where(accepted & (ss > 0.0), np.clip(bb, 1e-10 * base, 1e10 * base),
                         np.where(failed, 0.1 * step0, step0))
        x, f, g = x_new, f2, g2
        hist.append(f.copy())
        chi = be.max_abs(be.axpy(be.project(be.axpy(x, 1.0, g)), -1.0, x))
        log.f.append(f.tolist())
        log.chi.append(np.asarray(chi).tolist())
        log.grad_norm.append(gn2.tolist())
        log.backtracks.append(nback.tolist())
        log.resets.append((reset | failed).tolist())
        if on_iter is not None:
            on_iter(it, f, log)
    return x, f, g, log
