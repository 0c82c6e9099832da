"""Benchmark of the CNOP hot path on one MI355X.

One step = one iteration of the CNOP search on the largest workload that
fits one GPU: 8 restarts of the spectral projected-gradient ascent on the
sphere ||u0|| = 1e-3 (Sec. 3.4, Eq. 11) at 512 x 1024 FP64 cells, T = 1
(about 4.8k CFL steps per march), with binomial checkpointing under a
16 GiB pool:
    u+ = P(u + alpha g)                trial point on the sphere (Eq. 11)
    R+, g+ = R(u+) and dR/du(u+)       init_state, CFL march with level-1
                                       snapshots, kinetic energy, the
                                       reverse sweep (re-computation and
                                       discrete adjoint), initial adjoint
    accept (non-monotone test), alpha = <s,s>/|<s,y>| (dot products)
All of it runs in the library's HIP kernels; torch provides memory and the
stream.  Inputs are seeded synthetic velocity fields (envelope-masked
Gaussian noise); the paper uses no dataset.

value = algorithmic cell-updates per second: 2 B nx ny N_t per gradient
evaluation (one forward and one adjoint sweep over each member's N_t
steps), summed over the timed iterations, over their wall time.
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
FP64_PEAK_TFLOPS = 78.6                   # 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4     # wave64 instructions/s: one per 4 cycles per SIMD
FWD_BYTES_PER_CELL = 64.0   # read U^n, write U^{n+1}
ADJ_BYTES_PER_CELL = 96.0   # read U^n and lambda^{n+1}, write lambda^n
# Algorithmic FP64 operations per cell and step (the oracle's scheme counted
# operation by operation; tests/test_oracle_pins.py holds them to the count):
# the step plus the signal speed of the new state; the adjoint re-computes
# the step and does one multiply-add per edge of its computational graph.
FWD_FLOPS_PER_CELL = 324.0
ADJ_FLOPS_PER_CELL = 1400.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--T", type=float, default=1.0)
    ap.add_argument("--budget-gib", type=float, default=16.0, help="checkpoint pool of the binomial checkpointing")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline (no FD measurement, 256x512 and out-of-cache legs)")
    ap.add_argument("--kernel-launches", type=int, default=20)
    ap.add_argument("--groups", type=int, default=2,
                    help="independent searches the 8 restarts run as (own context, stream, host thread each)")
    ap.add_argument("--workload", default="cnop_8x512x1024",
                    help="cnop_8x512x1024 (default, the JSON line), grad_256x512, or a name from "
                         "paper_2608_04085_amd.workloads")
    return ap.parse_args()


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return model, int(cores or 1)


def cpu_baseline(cfg, seconds):
    """The oracle as it stands (C++, -O2), timed on the host CPU beside the GPU on a
    bounded sample of the same grid and seed: forward steps on one thread
    and with OpenMP over rows on every core the process may use, and
    reverse-mode adjoint steps of the whole grid on row bands on the same
    cores (oracle/chain.py: each band's adjoint is the whole grid's on it to
    the bit) and on one thread."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import chain, rto
    from oracle.rto import Oracle
    from paper_2608_04085_amd import inputs

    model, cores = host_info()
    c1 = cfg.with_(batch=1)
    o = Oracle.from_config(c1)
    U = o.init_state(inputs.seed_batch(c1, [0], l2=1e-3))
    cells = c1.nx * c1.ny
    dt = o.cfl_dt(U)

    def fwd_rate(threads, budget):
        used = rto.set_threads(threads)
        t0 = time.perf_counter()
        n = 0
        V = U
        while time.perf_counter() - t0 < budget or n == 0:
            V = o.step(V, dt)
            n += 1
        return n, n * cells / (time.perf_counter() - t0), used

    def adj_rate(workers, budget):
        rto.set_threads(1)
        lam = np.full_like(U, 1e-3)
        with ThreadPoolExecutor(workers) as ex:
            t0 = time.perf_counter()
            n = 0
            while time.perf_counter() - t0 < budget or n == 0:
                lam = chain.banded_vjp(o, U, float(dt[0]), lam, band=32, ex=ex)
                n += 1
            return n, n * cells / (time.perf_counter() - t0)

    n1, r1, _ = fwd_rate(1, 0.2 * seconds)
    nm, rm, used = fwd_rate(cores, 0.2 * seconds)
    na, ra = adj_rate(used, 0.3 * seconds)
    na1, ra1 = adj_rate(1, 0.3 * seconds)
    value = 2.0 / (1.0 / rm + 1.0 / ra)
    return {
        "value": value,
        "unit": "cell-updates/s",
        "cores": used,
        "kind": "oracle",
        "sample": f"{c1.nx}x{c1.ny} grid, Gaussian seed 0: {nm} forward steps with OpenMP over rows on {used} threads "
                  f"({rm:.3e} cell-updates/s; one thread: {n1} steps, {r1:.3e}) and {na} reverse-mode adjoint steps "
                  f"of the whole grid on row bands on {used} threads ({ra:.3e}; one thread: {na1} steps, {ra1:.3e}); "
                  f"value = 2/(1/forward + 1/adjoint) per cell",
        "single_thread_value": 2.0 / (1.0 / r1 + 1.0 / ra1),
        "host_cpu": model,
        "host_cores_available": cores,
    }


def roofline(kind, kt_us, cells, traffic, counters):
    """Roofline object of the forward step or the adjoint pair: algorithmic
    FP64 flops over the event-timed launch against the FP64 vector peak
    (the kernels are bound by FP64 VALU issue), with the HBM view
    (algorithmic bytes) and, from the committed counters at this size, the
    VALU issue rate beside it."""
    flops = (FWD_FLOPS_PER_CELL if kind == "step" else ADJ_FLOPS_PER_CELL) * cells
    nbytes = (FWD_BYTES_PER_CELL if kind == "step" else ADJ_BYTES_PER_CELL) * cells
    t = kt_us * 1e-6
    tf = flops / t / 1e12
    gb = nbytes / t / 1e9
    out = {
        "bound": "alu",
        "achieved": round(tf, 3),
        "peak": FP64_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(tf / FP64_PEAK_TFLOPS, 5),
        "traffic": None if traffic is None else round(traffic, 1),
        "algorithmic_flops_per_launch": flops,
        "kernel": ("fused forward step (k_step with the CFL epilogue, march)" if kind == "step"
                   else "adjoint step (k_adj_a + k_adj_b)"),
        "launch_us": round(kt_us, 3),
        "hbm": {"achieved": round(gb, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gb / HBM_PEAK_GBS, 5),
                "algorithmic_bytes_per_launch": nbytes},
        "valu_issue": None,
    }
    if counters and counters.get("SQ_INSTS_VALU"):
        insts = counters["SQ_INSTS_VALU"]
        f64 = 64 * (counters.get("SQ_INSTS_VALU_ADD_F64", 0) + counters.get("SQ_INSTS_VALU_MUL_F64", 0)
                    + counters.get("SQ_INSTS_VALU_TRANS_F64", 0) + 2 * counters.get("SQ_INSTS_VALU_FMA_F64", 0))
        out["valu_issue"] = {"achieved": insts / t, "peak": VALU_ISSUE_PEAK, "unit": "wave-instructions/s",
                             "frac": round(insts / t / VALU_ISSUE_PEAK, 4), "instructions_per_launch": insts,
                             "per_64_cells": round(insts / (cells / 64), 1),
                             "executed_fp64_tflops": round(f64 / t / 1e12, 3)}
    return out


def grad_256x512_extra(steps: int = 5, interval: int = 32) -> dict:
    """The 256 x 512, T = 2 gradient iteration (snapshots every 32 steps):
    projected-gradient iterations per second and cell-updates/s."""
    import torch

    from paper_2608_04085_amd import inputs
    from paper_2608_04085_amd.config import CKPT_UNIFORM, NORM_L2, SET_SPHERE, RTConfig
    from paper_2608_04085_amd.rtcnop import Context, Policy

    cfg = RTConfig(nx=256, ny=512)
    T = 2.0
    ctx = Context(cfg, max_steps=16384)
    u = torch.from_numpy(inputs.seed_batch(cfg, [0], rms=1e-3)).cuda()
    delta = float(math.sqrt(float((u * u).sum()) * cfg.dx * cfg.dy))
    U0 = ctx.init_state(u)
    _, _, n, _ = ctx.integrate(U0, T)
    nt = int(n.item())
    pol = Policy(CKPT_UNIFORM, interval)
    pool = torch.empty(ctx.pool_bytes(CKPT_UNIFORM, interval, nt + 64) + 256, dtype=torch.uint8, device="cuda")
    R, g, _ = ctx.grad_u0(u, T, pol, pool=pool)
    alpha = 0.1 * delta / float(g.norm() * math.sqrt(cfg.dx * cfg.dy))

    def iteration(u, g, alpha):
        ut, _ = ctx.project_to_constraint(ctx.axpy(u, alpha, g), delta, NORM_L2, SET_SPHERE)
        R, gt, n = ctx.grad_u0(ut, T, pol, pool=pool)
        s, y = ctx.axpy(ut, -1.0, u), ctx.axpy(gt, -1.0, g)
        a = float(ctx.dot(s, s).item()) / max(abs(float(ctx.dot(s, y).item())), 1e-300)
        return ut, gt, min(max(a, 1e-10 * alpha), 1e10 * alpha), n

    u, g, alpha, n = iteration(u, g, alpha)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot = 0
    for _ in range(steps):
        u, g, alpha, n = iteration(u, g, alpha)
        tot += int(n.item())
    torch.cuda.synchronize()
    per = (time.perf_counter() - t0) / steps
    torch.cuda.synchronize()
    tf0 = time.perf_counter()
    _, _, nf, _ = ctx.integrate(U0, T)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - tf0
    kt = ctx.kernel_times(ctx.integrate(U0, 0.5)[0], reps=100)
    return {"workload": "grad_256x512: forward + discrete-adjoint gradient of KE(T)/KE(0), T=2, snapshot every 32 "
                        "steps, one projected-gradient iteration", "grad_iters_per_s": 1.0 / per,
            "cell_updates_per_s": 2.0 * (tot / steps) * cfg.cells / per, "nsteps": tot / steps,
            "fwd_cell_updates_per_s": int(nf.item()) * cfg.cells / t_fwd, "gradient_over_forward": per / t_fwd,
            "kernel_times_us": {k: round(v, 3) for k, v in kt.items()}, "tile": ctx.tile}


def scale_point(kernel_launches: int = 10) -> dict:
    """Out-of-cache kernel times: 8 members of 1024 x 2048 (537 MB a state)."""
    from paper_2608_04085_amd import inputs, profiling
    from paper_2608_04085_amd.config import RTConfig
    from paper_2608_04085_amd.rtcnop import Context

    cfg8 = RTConfig(nx=1024, ny=2048, batch=8)
    ctx8 = Context(cfg8, max_steps=64)
    U8 = ctx8.init_state(inputs.seed_batch(cfg8, range(8), rms=1e-3))
    kt8 = ctx8.kernel_times(U8, reps=kernel_launches)
    cells8 = cfg8.nx * cfg8.ny * cfg8.batch
    out = {"workload": "8 x 1024 x 2048, one launch per step", "tile": ctx8.tile}
    for key, t_us, tkey, parts in (("step", kt8["step_march_us"], "step_march", ["step_march"]),
                                   ("adjoint", kt8["adjoint_two_kernel_us"], "adjoint", ["adj_a", "adj_b"])):
        out[key] = roofline(key, t_us, cells8, profiling.traffic_for("step_8x1024x2048", tkey, ctx8.tile),
                            profiling.counters_for("8x1024x2048", parts, ctx8.tile))
        out[key]["cell_updates_per_s"] = cells8 / (t_us * 1e-6)
    return out


def workload_child(name: str) -> dict:
    """A workload (`--workload NAME`) in a process of its own.  The
    gradients of the 256x512 and 64x128 workloads overlap their reverse
    sweep on two streams, and HIP maps a process's streams onto a few
    hardware queues in the order they are created: after the searches'
    streams, their two streams can share one queue and run one after the
    other (measured 185 against 155 ms per 256x512 iteration, 22 against
    17.5 ms per 64x128 gradient)."""
    import subprocess

    r = subprocess.run([sys.executable, "-u", os.path.abspath(__file__), "--workload", name, "--steps", "5"],
                       capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        raise RuntimeError(f"{name} child failed ({r.returncode}): {r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the independent restarts of a batch "
              f"would shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.workload == "grad_256x512":
        torch.cuda.set_device(0)
        print(json.dumps(grad_256x512_extra(max(args.steps, 1))), flush=True)
        return
    if args.workload != "cnop_8x512x1024":
        from paper_2608_04085_amd import workloads

        print(json.dumps(workloads.WORKLOADS[args.workload]()), flush=True)
        return

    from paper_2608_04085_amd import cnop, inputs, profiling, rtcnop
    from paper_2608_04085_amd.config import CKPT_REVOLVE, RTConfig
    from paper_2608_04085_amd.rtcnop import Context, Policy

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cfg = RTConfig(nx=512, ny=1024, batch=8)
    B = cfg.batch
    cells = cfg.nx * cfg.ny * B
    T = args.T
    delta = 1e-3
    max_steps = int(math.ceil(6000 * T)) + 1024
    state_bytes = 8 * 4 * cells
    budget = int(args.budget_gib * 2**30)
    slots = budget // state_bytes
    uv = inputs.seed_batch(cfg, range(B), l2=delta)

    # the 8 restarts as `groups` independent searches, each on its own
    # context, stream and share of the checkpoint budget (same slots per
    # state), driven by its own host thread: every member takes the
    # iterates of one search of all 8, bit for bit
    search = cnop.GroupedSPG(cfg, uv, T, delta, groups=args.groups, pool_bytes=budget, max_steps=max_steps,
                             policy=Policy(CKPT_REVOLVE, 1))
    if args.warmup:
        search.step(args.warmup)
    torch.cuda.synchronize()
    cu0, gr0, it0 = search.cell_updates, sum(search.grads), len(search.backtracks)
    t0 = time.perf_counter()
    search.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    per_iter = elapsed / args.steps
    value = (search.cell_updates - cu0) / elapsed
    grads_timed = (sum(search.grads) - gr0) / len(search.grads)
    nsteps = search.last_nsteps
    nt = int(max(nsteps))
    backtracks = [row for row in search.backtracks[it0:]]

    # kernels at this size, as one launch of all 8 members (HIP events on
    # the library's stream), on a state half-way through the march
    ctx = Context(cfg, max_steps=max_steps)
    Umid, _, _, _ = ctx.integrate(ctx.init_state(search.u), 0.5 * T)
    kt = ctx.kernel_times(Umid, reps=args.kernel_launches)
    fw_total, interval, two = rtcnop.revolve_plan_stats(nt, slots, nt)
    t_fwd = nt * kt["step_march_us"] + (fw_total - nt) * kt["step_given_us"]
    t_adj = nt * kt["adjoint_two_kernel_us"]
    tkey = "cnop_8x512x1024"
    adj = roofline("adjoint", kt["adjoint_two_kernel_us"], cells, profiling.traffic_for(tkey, "adjoint", ctx.tile),
                   profiling.counters_for(tkey, ["adj_a", "adj_b"], ctx.tile))
    stp = roofline("step", kt["step_march_us"], cells, profiling.traffic_for(tkey, "step_march", ctx.tile),
                   profiling.counters_for(tkey, ["step_march"], ctx.tile))
    dom, other = (adj, stp) if t_adj >= t_fwd else (stp, adj)
    per_grad_s = per_iter * args.steps / max(grads_timed, 1)
    dom["fwd_share_of_gradient"] = round(t_fwd * 1e-6 / per_grad_s, 3)
    dom["adj_share_of_gradient"] = round(t_adj * 1e-6 / per_grad_s, 3)
    # time per phase of one gradient of all 8 restarts, from the kernels'
    # event times (the executor copies no states); the searches overlap the
    # phases on the GPU, so they add up to more than the measured gradient
    phases = {"forward_march_ms": nt * kt["step_march_us"] * 1e-3,
              "recompute_ms": (fw_total - nt) * kt["step_given_us"] * 1e-3,
              "adjoint_ms": t_adj * 1e-3, "state_copies_ms": 0.0,
              "measured_gradient_ms": per_grad_s * 1e3}

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
            "workload": f"cnop_8x512x1024: one iteration of the CNOP search (spectral projected gradient on the sphere "
                        f"||u0|| = 1e-3, non-monotone line search, each trial evaluated with its discrete-adjoint "
                        f"gradient) for 8 restarts, run as {len(search.searches)} independent searches on their own "
                        f"streams, 512x1024 cells, T={T}, binomial checkpointing under {args.budget_gib:g} GiB",
            "nx": cfg.nx, "ny": cfg.ny, "batch": B, "groups": len(search.searches), "T": T,
            "nsteps": int(np.mean(nsteps)),
            "pool_slots": slots, "level1_interval": interval, "two_level": two,
            "forward_steps_per_gradient": fw_total, "tile": ctx.tile,
        },
        "cnop_iters_per_s": 1.0 / per_iter,
        "gradient_evals_per_iter": grads_timed / args.steps,
        "backtracks": backtracks,
        "best_R": float(np.max(search.R)),
        "roofline": dom,
        "roofline_other": other,
        "kernel_times_us": {k: round(v, 3) for k, v in kt.items()},
        "phases_per_gradient": {k: round(v, 1) for k, v in phases.items()},
    }
    if not args.no_extras:
        out["fd_64x128_measured"] = workload_child("fd_64x128")
        # the FD gradient iteration at this size, extrapolated from a timed
        # march of the 8 members: 2 n_dof marches per member, each batched
        # march serving every member once
        torch.cuda.synchronize()
        tb = time.perf_counter()
        ctx.objective_ratio(search.u, T)
        torch.cuda.synchronize()
        t_march8 = time.perf_counter() - tb
        n_dof = 2 * cfg.nx * cfg.ny
        fd_iter = 2 * n_dof * t_march8 + t_march8
        out["fd_iters_per_s_extrapolated"] = 1.0 / fd_iter
        out["adjoint_vs_fd_speedup_extrapolated"] = fd_iter / per_iter
        out["forward_march_seconds_8_members"] = t_march8
        out["grad_256x512"] = workload_child("grad_256x512")
        out["scale_point"] = scale_point()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
