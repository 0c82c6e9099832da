"""Benchmark of the CNOP hot path on one MI355X.

One step = one projected-gradient iteration of the CNOP search on the
gradient workload (256 x 512 FP64 cells, T = 2, about 4.8k CFL steps, a
snapshot every 32 steps with re-computation in between):
    u+ = P(u + alpha g)                   (constraint projection, Eq. 11)
    R, g+ = KE ratio and its gradient     (init_state, CFL march with
                                           snapshots, kinetic energy, adjoint
                                           sweep, initial adjoint)
    alpha = <s,s>/|<s,y>|                 (dot products for the next step)
All of it runs in the library's HIP kernels; torch provides memory and the
stream.  Inputs are seeded synthetic velocity fields (envelope-masked
Gaussian noise); the paper uses no dataset.

value = (forward + adjoint) cell-updates per second of the whole iteration:
2 * N_t * nx * ny / (seconds per iteration).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FP64 cell-updates/s (fwd, adjoint) and CNOP grad iters/s vs FD-gradient, % HBM"
HBM_PEAK_GBS = 8000.0
FWD_BYTES_PER_CELL = 64.0   # read U^n, write U^{n+1}
ADJ_BYTES_PER_CELL = 96.0   # read U^n and lambda^{n+1}, write lambda^n


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--ny", type=int, default=512)
    ap.add_argument("--T", type=float, default=2.0)
    ap.add_argument("--interval", type=int, default=32)
    ap.add_argument("--tile", default=None, help="tile variant of both kernels (default: the library's choice)")
    ap.add_argument("--tiles", default=None, help="STEP/ADJOINT tile variants (overrides --tile)")
    ap.add_argument("--fold", type=int, choices=(0, 1), default=None,
                    help="1: folded reverse sweep (one kernel per adjoint step), 0: two kernels (default: the library's choice)")
    ap.add_argument("--autotune", action="store_true",
                    help="run the kernel autotuner, then keep the fastest of its pick and two fixed pairs on a "
                         "full gradient each (default: the library's measured defaults, so that a profile of "
                         "this command sees the same kernels)")
    ap.add_argument("--dt-mode", choices=("frozen", "differentiated"), default="frozen",
                    help="time steps in the gradient: held at the forward run's (default) or differentiated")
    ap.add_argument("--recon", choices=("primitive", "balanced"), default="primitive",
                    help="reconstruction: primitive MC (default) or the well-balanced variant")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--kernel-launches", type=int, default=300)
    ap.add_argument("--workload", default="grad_256x512",
                    help="grad_256x512 (default, the JSON line) or a name from paper_2608_04085_amd.workloads")
    return ap.parse_args()


def cpu_baseline(cfg, T, seconds):
    """The oracle as it stands (single-threaded C++), timed on a bounded
    sample of the same workload: forward steps and reverse-mode adjoint steps
    on the same grid from the same seed."""
    from oracle.rto import Oracle
    from paper_2608_04085_amd import inputs

    o = Oracle.from_config(cfg)
    U = o.init_state(inputs.seed_batch(cfg, [0], rms=1e-3))
    cells = cfg.nx * cfg.ny
    t0 = time.perf_counter()
    nf = 0
    while time.perf_counter() - t0 < 0.6 * seconds:
        U = o.step(U, o.cfl_dt(U))
        nf += 1
    tf = (time.perf_counter() - t0) / (nf * cells)
    lam = np.ones_like(U) * 1e-3
    t1 = time.perf_counter()
    na = 0
    dt = o.cfl_dt(U)
    while time.perf_counter() - t1 < 0.4 * seconds or na == 0:
        lam = o.step_vjp(U, dt, lam)
        na += 1
    ta = (time.perf_counter() - t1) / (na * cells)
    return {
        "value": 2.0 / (tf + ta),
        "unit": "cell-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{nf} forward steps + {na} adjoint steps of the {cfg.nx}x{cfg.ny} grid from the same seed; "
                  f"value = 2/(t_fwd + t_adj) per cell (forward {1.0 / tf:.3e}, adjoint {1.0 / ta:.3e} cell-updates/s)",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the independent members of a "
              f"batch shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.workload != "grad_256x512":
        from paper_2608_04085_amd import workloads

        print(json.dumps(workloads.WORKLOADS[args.workload]()), flush=True)
        return

    from paper_2608_04085_amd import inputs
    from paper_2608_04085_amd.config import CKPT_UNIFORM, NORM_L2, SET_SPHERE, RTConfig
    from paper_2608_04085_amd.rtcnop import Context, Policy

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    from paper_2608_04085_amd.config import RECON_BALANCED, RECON_PRIMITIVE

    cfg = RTConfig(nx=args.nx, ny=args.ny, recon=RECON_BALANCED if args.recon == "balanced" else RECON_PRIMITIVE)
    # the committed counter runs cover the default kernels only
    counters_apply = args.dt_mode == "frozen" and args.recon == "primitive"
    T = args.T
    ctx = Context(cfg, max_steps=16384, tile=args.tile)
    if args.tiles:
        ctx.set_tiles(*args.tiles.split("/"))
    if args.fold is not None:
        ctx.set_fold(bool(args.fold))
    ctx.set_dt_mode(args.dt_mode)
    cells = cfg.nx * cfg.ny

    # seed and step count
    u = torch.from_numpy(inputs.seed_batch(cfg, [0], rms=1e-3)).cuda()
    delta = float(math.sqrt(float((u * u).sum()) * cfg.dx * cfg.dy))
    U0 = ctx.init_state(u)
    _, _, n, log = ctx.integrate(U0, T, log_cap=16384)
    nt = int(n.item())
    pol = Policy(CKPT_UNIFORM, args.interval)
    pool = torch.empty(ctx.pool_bytes(CKPT_UNIFORM, args.interval, nt + 64) + 256, dtype=torch.uint8, device="cuda")
    tuning = {}
    if args.autotune:
        # kernel-level autotuning, then the sweep decides: the autotuner's
        # pick against two fixed pairs, one gradient each (all give the same
        # bits; only the speed differs)
        ctx.autotune(U0, reps=20)
        cands = [(ctx.tile, ctx.fold), ("32x8w/32x8", False), ("32x8/32x8", False)]
        for tiles, fold in cands:
            ctx.set_tiles(*tiles.split("/"))
            ctx.set_fold(fold)
            ctx.grad_u0(u, T, pol, pool=pool)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.grad_u0(u, T, pol, pool=pool)
            torch.cuda.synchronize()
            tuning[f"{tiles}{'+fold' if fold else ''}"] = time.perf_counter() - t0
        best = min(tuning, key=tuning.get)
        ctx.set_tiles(*best.split("+")[0].split("/"))
        ctx.set_fold(best.endswith("+fold"))
    R, g, _ = ctx.grad_u0(u, T, pol, pool=pool)
    alpha = 0.1 * delta / float(g.norm() * math.sqrt(cfg.dx * cfg.dy))

    def iteration(u, g, alpha):
        ut = ctx.axpy(u, alpha, g)
        ut, _ = ctx.project_to_constraint(ut, delta, NORM_L2, SET_SPHERE)
        R, gt, n = ctx.grad_u0(ut, T, pol, pool=pool)
        s = ctx.axpy(ut, -1.0, u)
        y = ctx.axpy(gt, -1.0, g)
        ss, sy = ctx.dot(s, s), ctx.dot(s, y)
        a = float(ss.item()) / max(abs(float(sy.item())), 1e-300)
        return ut, gt, min(max(a, 1e-10 * alpha), 1e10 * alpha), R, n

    for _ in range(args.warmup):
        u, g, alpha, R, n = iteration(u, g, alpha)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nsteps_total = 0
    for _ in range(args.steps):
        u, g, alpha, R, n = iteration(u, g, alpha)
        nsteps_total += int(n.item())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    per_iter = elapsed / args.steps
    nt_mean = nsteps_total / args.steps
    value = 2.0 * nt_mean * cells / per_iter

    # forward-only march (adaptive CFL, one launch per step, no snapshots)
    torch.cuda.synchronize()
    tf0 = time.perf_counter()
    _, _, nf, _ = ctx.integrate(U0, T)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - tf0
    fwd_rate = int(nf.item()) * cells / t_fwd

    # finite-difference gradient for comparison: n_dof + 1 forward marches
    # (one-sided differences), run as batches of 8 members; one batch timed
    fd_b = 8
    ctx_fd = Context(cfg.with_(batch=fd_b), max_steps=16384)
    Ufd = ctx_fd.init_state(np.repeat(inputs.seed_batch(cfg, [0], rms=1e-3), fd_b, axis=0))
    ctx_fd.autotune(Ufd, reps=10)
    ctx_fd.integrate(Ufd, T)
    torch.cuda.synchronize()
    tb0 = time.perf_counter()
    ctx_fd.integrate(Ufd, T)
    torch.cuda.synchronize()
    t_fd_batch = time.perf_counter() - tb0
    del ctx_fd, Ufd
    n_dof = 2 * cells
    fd_iter_s = t_fd_batch * (n_dof + 1) / fd_b

    # per-launch durations of the kernels as the iteration launches them,
    # from HIP events on the library's stream around back-to-back launches
    Uk = ctx.integrate(U0, 0.5)[0]
    kt = ctx.kernel_times(Uk, reps=args.kernel_launches)
    t_given, t_march, t_adj = (kt["step_given_us"] * 1e-6, kt["step_march_us"] * 1e-6,
                               kt["adjoint_sweep_us"] * 1e-6)
    # per iteration: nt march steps, nt (interval-1)/interval re-computed
    # steps, nt adjoint steps (one kernel each)
    fw_share = nt_mean * (t_march + t_given * (1 - 1.0 / args.interval))
    adj_share = t_adj * nt_mean
    if adj_share >= fw_share:
        dom = {"kernel": ("adjoint step (k_adj_a with the folded limiter gather)" if ctx.fold
                          else "adjoint step (k_adj_a + k_adj_b)"),
               "bytes_per_cell": ADJ_BYTES_PER_CELL, "t": t_adj,
               "traffic_key": "adjoint_folded" if ctx.fold else "adjoint"}
    else:
        dom = {"kernel": "fused forward step (k_step, march)", "bytes_per_cell": FWD_BYTES_PER_CELL, "t": t_march,
               "traffic_key": "step"}
    achieved = dom["bytes_per_cell"] * cells / dom["t"] / 1e9
    from paper_2608_04085_amd import profiling

    traffic = (profiling.traffic_for(f"grad_{cfg.nx}x{cfg.ny}", dom["traffic_key"], ctx.tile)
               if counters_apply else None)
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 2),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 5),
        "traffic": None if traffic is None else round(traffic, 1),
        "algorithmic_bytes_per_launch": dom["bytes_per_cell"] * cells,
        "kernel": dom["kernel"],
        "launch_us": round(dom["t"] * 1e6, 3),
        "kernel_times_us": {k: round(v, 3) for k, v in kt.items()},
        **({} if args.dt_mode == "frozen" else
           {"note": "launch_us and kernel_times_us time the frozen-step kernels; the differentiated sweep adds its "
                    "step-size partial sums to kernel A and one small kernel per step"}),
        "fwd_share_of_iteration": round(fw_share / per_iter, 3),
        "adj_share_of_iteration": round(adj_share / per_iter, 3),
    }
    # the fused forward step of the march beside it, on the same terms
    t_step_traffic = (profiling.traffic_for(f"grad_{cfg.nx}x{cfg.ny}", "step_march", ctx.tile)
                      if counters_apply else None)
    achieved_step = FWD_BYTES_PER_CELL * cells / t_march / 1e9
    roofline_step = {
        "bound": "hbm",
        "achieved": round(achieved_step, 2),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved_step / HBM_PEAK_GBS, 5),
        "traffic": None if t_step_traffic is None else round(t_step_traffic, 1),
        "algorithmic_bytes_per_launch": FWD_BYTES_PER_CELL * cells,
        "kernel": "fused forward step (k_step with the CFL epilogue, march)",
        "launch_us": round(t_march * 1e6, 3),
    }
    # the out-of-cache point: 8 members of 1024 x 2048 (537 MB per state,
    # above the last-level cache), the same kernels timed the same way
    cfg8 = RTConfig(nx=1024, ny=2048, batch=8)
    ctx8 = Context(cfg8, max_steps=64)
    U8 = ctx8.init_state(inputs.seed_batch(cfg8, range(8), rms=1e-3))
    kt8 = ctx8.kernel_times(U8, reps=10)
    cells8 = cfg8.nx * cfg8.ny * cfg8.batch
    scale_point = {"workload": "8 x 1024 x 2048, one launch per step", "tile": ctx8.tile}
    for key, bpc, t_us, tkey in (("step", FWD_BYTES_PER_CELL, kt8["step_march_us"], "step_march"),
                                 ("adjoint", ADJ_BYTES_PER_CELL, kt8["adjoint_two_kernel_us"], "adjoint")):
        gbs = bpc * cells8 / (t_us * 1e-6) / 1e9
        tr = profiling.traffic_for("step_8x1024x2048", tkey, ctx8.tile)
        scale_point[key] = {"launch_us": round(t_us, 3), "cell_updates_per_s": cells8 / (t_us * 1e-6),
                            "achieved_GBps": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                            "traffic": None if tr is None else round(tr, 1)}
    del ctx8, U8
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": per_iter * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"grad_{cfg.nx}x{cfg.ny}: forward + discrete-adjoint gradient of KE(T)/KE(0), T={T}, "
                        f"snapshot every {args.interval} steps, one projected-gradient iteration per step",
            "nx": cfg.nx, "ny": cfg.ny, "batch": 1, "T": T, "nsteps": nt_mean, "tile": ctx.tile,
            "adjoint_folded": ctx.fold,
            "dt_in_gradient": ctx.dt_mode, "reconstruction": "primitive MC" if cfg.recon == 0 else "well-balanced",
            "sweep_tuning_seconds": {k: round(v, 4) for k, v in tuning.items()},
        },
        "grad_iters_per_s": 1.0 / per_iter,
        "fwd_cell_updates_per_s": fwd_rate,
        "fd_grad_iters_per_s_extrapolated": 1.0 / fd_iter_s,
        "fd_batch8_forward_seconds": t_fd_batch,
        "adjoint_vs_fd_speedup": fd_iter_s / per_iter,
        "R": float(R.item()),
        "roofline": roofline,
        "roofline_step": roofline_step,
        "scale_point": scale_point,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, T, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
