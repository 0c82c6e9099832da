"""The benchmark workloads, each returning a dict of measured results.

    fwd_64x128            forward march to T = 2 of one RMS-1e-3 Gaussian seed; R and cell-updates/s
    ensemble_64x128x256   64 members (32 Gaussian seeds, 32 single Fourier modes kx = 1..16, two
                          phases), velocity L2 norm 1e-3, T = 2, all members in one launch per step
    cnop_8x512x1024       SPG CNOP search, 8 restarts, T = 1 or 4, binomial checkpointing <= 16 GB
                          (bench.py's step is one iteration of it)
    grad_1024x2048        forward + adjoint, T = 3, binomial checkpointing <= 64 GB; top-5 horizontal
                          mode energy of the sphere-projected gradient; adjoint/forward time ratio
    fd_64x128             the full central-difference gradient (2 n_dof batched forwards) vs the adjoint
    paper_cnop_128        the paper's own search on its physics: J of Eq. 8 over C <= 1e-6, projected L-BFGS
                          (m = 10) against the memory-free driver (SPG) at equal gradient budget
    paper_compare_128     the paper's forward comparison suite: CNOP, Random, 5modes and 2-D 90% reconstructions
                          marched together, KE(t) and mixing width h_mix(t)

The 256x512 gradient iteration (snapshot every 32 steps, T = 2) is bench.py --workload grad_256x512.
All inputs are seeded synthetic fields (see inputs.py); the paper uses no dataset.
Run: python -m paper_2608_04085_amd.workloads <name> [--iters K] [--T T]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import cnop, inputs, optim
from .config import CKPT_REVOLVE, CKPT_UNIFORM, NORM_L2, NORM_RHO_KE, SET_SPHERE, RTConfig, paper_preset
from .rtcnop import Context, Policy


def _sync():
    torch.cuda.synchronize()


def _timed(fn):
    _sync()
    t0 = time.perf_counter()
    out = fn()
    _sync()
    return out, time.perf_counter() - t0


def fwd_64x128(T: float = 2.0, reps: int = 5) -> dict:
    cfg = RTConfig(nx=64, ny=128)
    rt = Context(cfg, max_steps=8192)
    U0 = rt.init_state(inputs.seed_batch(cfg, [0], rms=1e-3))
    rt.autotune(U0)
    rt.integrate(U0, T)
    times = []
    for _ in range(reps):
        (UT, t, n, _), el = _timed(lambda: rt.integrate(U0, T))
        times.append(el)
    ke = rt.kinetic_energy(UT) / rt.kinetic_energy(U0)
    el = float(np.median(times))
    return {"workload": "fwd_64x128", "T": T, "nsteps": int(n.item()), "R": float(ke.item()),
            "cell_updates_per_s": cfg.cells * int(n.item()) / el, "seconds": el, "tiles": rt.tile}


def ensemble_64x128x256(T: float = 2.0, reps: int = 2) -> dict:
    cfg = RTConfig(nx=128, ny=256, batch=64)
    rt = Context(cfg, max_steps=8192)
    uv = inputs.ensemble_batch(cfg, 1e-3)
    U0 = rt.init_state(uv)
    rt.autotune(U0)
    times = []
    for _ in range(reps):
        (UT, t, n, _), el = _timed(lambda: rt.integrate(U0, T))
        times.append(el)
    R = (rt.kinetic_energy(UT) / rt.kinetic_energy(U0)).cpu().numpy()
    el = float(np.median(times))
    ns = n.cpu().numpy()
    return {"workload": "ensemble_64x128x256", "T": T, "batch": 64, "nsteps_min": int(ns.min()),
            "nsteps_max": int(ns.max()), "R_gaussian": R[:32].tolist(), "R_fourier_kx_phase": R[32:].tolist(),
            "aggregate_cell_updates_per_s": float(cfg.nx * cfg.ny * ns.sum() / el), "seconds": el,
            "tiles": rt.tile}


def _revolve_pool(rt: Context, budget_bytes: int) -> torch.Tensor:
    state = 8 * 4 * rt.cfg.cells * rt.cfg.batch
    slots = max(2, budget_bytes // state)
    return torch.empty(slots * state + 256, dtype=torch.uint8, device=rt.device)


def grad_1024x2048(T: float = 3.0, budget_gb: float = 64.0) -> dict:
    cfg = RTConfig(nx=1024, ny=2048)
    rt = Context(cfg, max_steps=65536)
    uv = inputs.seed_batch(cfg, [0], rms=1e-3)
    U0 = rt.init_state(uv)
    rt.autotune(U0, reps=5)
    (UT, t, n, _), t_fwd = _timed(lambda: rt.integrate(U0, T))
    pool = _revolve_pool(rt, int(budget_gb * 2**30))
    (R, g, ng), t_grad = _timed(lambda: rt.grad_u0(uv, T, Policy(CKPT_REVOLVE, 1), pool=pool))
    gp, _ = rt.project_to_constraint(g, math.sqrt(float((torch.as_tensor(uv) ** 2).sum()) * cfg.dx * cfg.dy),
                                     NORM_L2, SET_SPHERE)
    v = gp[0, 1].cpu().numpy()
    row = cnop.peak_row(v)
    E = rt.row_spectrum(gp, row, component=1)[0].cpu().numpy()  # Eq. 12 on the device
    return {"workload": "grad_1024x2048", "T": T, "nsteps": int(n.item()), "R": float(R.item()),
            "forward_seconds": t_fwd, "gradient_seconds": t_grad, "adjoint_over_forward": t_grad / t_fwd,
            "pool_slots": int(pool.numel() // (8 * 4 * cfg.cells)), "peak_row": row,
            "top5_kx_energy_fraction": cnop.top5_fraction(E), "tiles": rt.tile}


def cnop_8x512x1024(T: float = 1.0, iters: int = 50, budget_gb: float = 16.0, groups: int = 2) -> dict:
    """The 8 restarts as `groups` independent searches (cnop.GroupedSPG: own
    context, stream and share of the budget each, one host thread each;
    every member takes the iterates of one search of all 8), default tiles
    (measured fastest for the whole split binomial sweep, which the
    autotuner, timing each kernel alone, does not see)."""
    cfg = RTConfig(nx=512, ny=1024, batch=8)
    delta = 1e-3
    uv = inputs.seed_batch(cfg, range(8), l2=delta)
    t0 = time.perf_counter()
    search = cnop.GroupedSPG(cfg, uv, T, delta, groups=groups, pool_bytes=int(budget_gb * 2**30),
                             max_steps=65536, policy=Policy(CKPT_REVOLVE, 1))
    t_init = time.perf_counter() - t0
    R_init = search.R.tolist()

    def progress(k, it):
        print(f"cnop T={T} group {k} iter {it + 1}/{iters} {time.perf_counter() - t0:.1f}s", file=sys.stderr,
              flush=True)

    _, el = _timed(lambda: search.step(iters, on_iter=progress))
    R = search.R
    # finite-difference alternative (extrapolated): 2 n_dof central
    # differences plus the point itself per member and iteration, at the
    # measured rate of one batched forward of all members
    rt = Context(cfg, max_steps=65536)
    _, t_fwd = _timed(lambda: cnop.ke_ratio(rt, search.u, T))
    n_dof = 2 * cfg.cells
    fd_iter_s = t_fwd * (2 * n_dof + 1)  # each batched forward serves every member once
    chi = [c for s in search.searches for c in (s.log.chi[-1] if s.log.chi else [])]
    return {"workload": "cnop_8x512x1024", "T": T, "iters": iters, "groups": len(search.searches),
            "seconds": el, "iters_per_s": iters / el, "initial_gradient_seconds": t_init,
            "forward_batch_seconds": t_fwd, "fd_iters_per_s_extrapolated": 1.0 / fd_iter_s,
            "adjoint_vs_fd_speedup": fd_iter_s / (el / iters),
            "R_initial": R_init, "R_final": [float(x) for x in R.tolist()], "best_R": float(max(R.tolist())),
            "chi_final": chi, "gradient_evals_per_group": search.grads, "tiles": rt.tile}


def _fd_ratio(rtb: Context, uv: torch.Tensor, dofs: np.ndarray, h: float, T: float) -> np.ndarray:
    """Central differences (R(u + h e_k) - R(u - h e_k)) / 2h of the objective
    as computed (the adaptive march, every member with its own CFL steps)
    for the flat entries `dofs` of uv, in batched marches of B members
    (two per entry)."""
    B = rtb.cfg.batch
    per = B // 2
    out = np.empty(len(dofs))
    flat = uv.reshape(1, -1)
    for k0 in range(0, len(dofs), per):
        ks = dofs[k0:k0 + per]
        pert = flat.repeat(B, 1)
        rows = torch.arange(len(ks), device=uv.device)
        kk = torch.as_tensor(ks, device=uv.device)
        pert[2 * rows, kk] += h
        pert[2 * rows + 1, kk] -= h
        R = rtb.objective_ratio(pert.reshape(B, *uv.shape[1:]), T).cpu().numpy()
        out[k0:k0 + len(ks)] = (R[0:2 * len(ks):2] - R[1:2 * len(ks):2]) / (2.0 * h)
    return out


def fd_64x128(T: float = 2.0, batch: int = 256, hs=(1e-6, 1e-7, 1e-8, 1e-9), sample: int = 256) -> dict:
    """The finite-difference gradient iteration, measured: the central-
    difference gradient of R = KE(T)/KE(0) as computed (the adaptive march,
    2 n_dof marches of 64x128 to T = 2, `batch` per launch) against the
    library's adjoint gradients.  The step h (absolute, on one velocity
    entry of the RMS-1e-3 seed) is the best of `hs` on a sample of entries
    (the largest gradient entries and random ones); then every entry is
    differenced with it.  Errors are max |FD - g| / max |g| over all
    entries, against the gradient of the adaptive march (time steps
    differentiated: the map FD differences) and against the frozen-step
    one."""
    cfg = RTConfig(nx=64, ny=128)
    n_dof = 2 * cfg.cells
    uv = torch.from_numpy(inputs.seed_batch(cfg, [0], rms=1e-3)).cuda()
    rt1 = Context(cfg, max_steps=8192)
    out = {"workload": "fd_64x128", "T": T, "n_dof": n_dof, "fd_batch": batch}
    grads = {}
    for mode in ("differentiated", "frozen"):
        rt1.set_dt_mode(mode)
        rt1.grad_u0(uv, T)
        ts = []
        for _ in range(3):
            (R, g, n), el = _timed(lambda: rt1.grad_u0(uv, T))
            ts.append(el)
        grads[mode] = g.cpu().numpy().ravel()
        out[f"adjoint_gradient_seconds_{mode}"] = float(np.median(ts))
    _, t_fwd = _timed(lambda: rt1.objective_ratio(uv, T))
    gd = grads["differentiated"]
    gmax = float(np.max(np.abs(gd)))
    out["frozen_vs_differentiated"] = float(np.max(np.abs(grads["frozen"] - gd)) / gmax)
    rtb = Context(cfg.with_(batch=batch), max_steps=8192)
    rng = np.random.default_rng(77)
    top = np.argsort(-np.abs(gd), kind="stable")[: sample // 2]
    rest = np.setdiff1d(np.arange(n_dof), top)
    samp = np.concatenate([top, rng.choice(rest, size=sample - len(top), replace=False)])
    _fd_ratio(rtb, uv, samp[: batch // 2], hs[0], T)  # warm-up (graph capture)
    errs = {}
    for h in hs:
        fd = _fd_ratio(rtb, uv, samp, h, T)
        errs[h] = float(np.max(np.abs(fd - gd[samp])) / gmax)
    h_best = min(errs, key=errs.get)
    out["sample_errors_by_h"] = {f"{h:g}": e for h, e in errs.items()}
    out["h"] = h_best
    (fd, t_fd) = _timed(lambda: _fd_ratio(rtb, uv, np.arange(n_dof), h_best, T))
    out["fd_gradient_seconds"] = t_fd
    out["fd_marches"] = 2 * n_dof
    out["fd_error_vs_differentiated"] = float(np.max(np.abs(fd - gd)) / gmax)
    out["fd_error_vs_frozen"] = float(np.max(np.abs(fd - grads["frozen"])) / float(np.max(np.abs(grads["frozen"]))))
    rel = np.abs(fd - gd) / gmax
    out["fd_error_quantiles"] = {q: float(np.quantile(rel, float(q))) for q in ("0.5", "0.9", "0.99", "0.999")}
    # one iteration = one gradient plus one evaluation of the trial point
    # for FD; the adjoint iteration evaluates its trial with its gradient
    out["forward_seconds"] = t_fwd
    out["fd_iters_per_s"] = 1.0 / (t_fd + t_fwd)
    out["adjoint_iters_per_s"] = 1.0 / out["adjoint_gradient_seconds_frozen"]
    out["adjoint_speedup"] = out["adjoint_iters_per_s"] / out["fd_iters_per_s"]
    return out


def paper_cnop_128(T: float = 2.0, iters: int = 20, restarts: int = 4) -> dict:
    """The paper's own search (Sec. 3; run T2_N128 of its run table): J of
    Eq. 8 over C <= 1e-6 (Eq. 9, ball projection of Eq. 11), u_y-only seeds
    localised at the interface (width 0.1 L), paper physics on 128 x 128,
    projected L-BFGS with m = 10 against the same driver without memory (the
    spectral projected gradient method) at equal gradient budget; restarts
    are batch members.  UNIFORM(32) checkpoints."""
    cfg = paper_preset(128, batch=restarts)
    rt = Context(cfg, max_steps=16384)
    uv = inputs.paper_seed_batch(cfg, range(restarts))
    rt.autotune(rt.init_state(uv), reps=10)
    pol = Policy(CKPT_UNIFORM, 32)
    out = {"workload": "paper_cnop_128", "T": T, "eps": 1e-6, "restarts": restarts, "iters": iters,
           "tiles": rt.tile}
    for name, mem in (("lbfgs_m10", 10), ("spg_m0", 0)):
        t0 = time.perf_counter()

        def progress(k, f, lg, name=name, t0=t0):
            print(f"{name} iter {k + 1}/{iters} {time.perf_counter() - t0:.1f}s max J {float(np.max(f)):.4g}",
                  file=sys.stderr, flush=True)

        ekb = rt.baseline_ek(T)
        u0, _ = rt.project_to_constraint(rt.as_dev(uv), 1e-6, NORM_RHO_KE, SET_SPHERE)
        be = cnop.LibraryBackend(rt, T, ekb, 1e-6, pol)
        (u, J, g, log), el = _timed(lambda: optim.lbfgs_max(be, u0, iters, memory=mem, on_iter=progress))
        out[name] = {"seconds": el, "iters_per_s": iters / el, "gradient_evals": log.grads,
                     "forward_evals": log.evals, "J_first": log.f[0], "J_final": [float(x) for x in J],
                     "J_history_max": [float(np.max(x)) for x in log.f], "chi_final": log.chi[-1],
                     "resets": int(np.sum(log.resets))}
    return out


def paper_compare_128(T: float = 2.0, iters: int = 20, n_snap: int = 20) -> dict:
    """The forward comparison suite of the paper (run design of Sec. 3.3,
    diagnostics of Sec. 4.3-4.4) on its physics at 128 x 128: a CNOP from
    `iters` projected-gradient iterations on J (Eq. 8, C <= 1e-6), then the
    CNOP, a localised random seed, the CNOP's 5-mode reduction and its
    90%-power 2-D reconstruction, all at C = 1e-6, marched together to T
    with n_snap uniformly spaced KE and mixing-width diagnostics."""
    cfg = paper_preset(128, batch=1)
    rt = Context(cfg, max_steps=16384)
    uv = inputs.paper_seed_batch(cfg, [0])
    pol = Policy(CKPT_UNIFORM, 32)
    t0 = time.perf_counter()
    ekb = rt.baseline_ek(T)
    u0, _ = rt.project_to_constraint(rt.as_dev(uv), 1e-6, NORM_RHO_KE, SET_SPHERE)
    be = cnop.LibraryBackend(rt, T, ekb, 1e-6, pol)
    u, J, g, log = optim.lbfgs_max(be, u0, iters, memory=0)
    t_search = time.perf_counter() - t0
    seeds = cnop.comparison_seeds(cfg, u[0, 1].cpu().numpy(), rt=rt)
    rc = Context(cfg.with_(batch=4), max_steps=16384)
    (res, el) = _timed(lambda: cnop.comparison_runs(rc, seeds, 1e-6, T, n_snap))
    ke = np.array(res["ke"])
    hm = np.array(res["h_mix"])
    return {"workload": "paper_compare_128", "T": T, "search_iters": iters, "search_seconds": t_search,
            "J_cnop": float(J[0]), "kinds": list(cnop.COMPARISON_KINDS),
            "dominant_modes": cnop.dominant_modes(u[0, 1].cpu().numpy()).tolist(),
            "ke_ratio_T": (ke[-1] / ke[0]).tolist(), "h_mix_0": hm[0].tolist(), "h_mix_T": hm[-1].tolist(),
            "ke_series": res["ke"], "h_mix_series": res["h_mix"], "t": res["t"], "steps": res["steps"],
            "suite_seconds": el}


WORKLOADS = {f.__name__: f for f in (fwd_64x128, ensemble_64x128x256, grad_1024x2048, cnop_8x512x1024, fd_64x128,
                                     paper_cnop_128, paper_compare_128)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name", choices=sorted(WORKLOADS))
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--T", type=float, default=None)
    a = ap.parse_args()
    kw = {}
    if a.iters is not None:
        kw["iters"] = a.iters
    if a.T is not None:
        kw["T"] = a.T
    print(json.dumps(WORKLOADS[a.name](**kw)), flush=True)


if __name__ == "__main__":
    main()
