"""Counter runs of the hot-path kernels and their summaries.

    python -m paper_2608_04085_amd.profiling drive NX NY B K STEP_TILE ADJ_TILE
        K launches of the step kernel and K of the adjoint step at one grid,
        then K copies of a 2 GiB buffer (a plain copy of known size whose
        FETCH_SIZE / WRITE_SIZE calibrate the counters).  Run it under
        rocprofv3 (kernel trace, then --pmc FETCH_SIZE, then --pmc WRITE_SIZE).
    python -m paper_2608_04085_amd.profiling summarize WORKLOAD TRACE FETCH WRITE REQ OUT_MD
        Turns the rocprofv3 CSV directories (kernel trace; --pmc FETCH_SIZE;
        --pmc WRITE_SIZE; --pmc TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum
        TCC_EA0_RDREQ_128B_sum TCC_EA0_RDREQ_sum) into a short Markdown summary
        and records per-launch HBM bytes in profiles/traffic.json, keyed by the
        hash of the kernel sources (bench.py reports the traffic only while the
        kernels are unchanged).

FETCH_SIZE and WRITE_SIZE are scaled by what they read for the plain copy
(bytes moved / counted bytes).  On gfx950 the derived FETCH_SIZE counts a
128-byte read request as 64 bytes, so the copy (all 128-byte requests) reads
half its bytes; the request-size counters give the read bytes exactly
(32 n32 + 64 n64 + 128 n128) and are reported beside the scaled figure.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
KERNEL_SOURCES = ["csrc/rt_kernels.hip", "csrc/rt_device.h", "csrc/rt_kernels.h"]
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")
COPY_BYTES = 2 * 1024**3


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def drive(nx: int, ny: int, B: int, K: int, step_tile: str, adj_tile: str):
    import torch

    from . import inputs
    from .config import RTConfig
    from .rtcnop import Context

    cfg = RTConfig(nx=nx, ny=ny, batch=B)
    rt = Context(cfg, max_steps=64, tile=step_tile)
    U = rt.init_state(inputs.seed_batch(cfg, range(B), rms=1e-3))
    dt = rt.cfl_dt(U)
    Un = torch.empty_like(U)
    for _ in range(K):
        rt.step(U, dt, out=Un)
    rt.set_tile(adj_tile)
    lam = torch.empty_like(U).fill_(1e-3)
    lo = torch.empty_like(U)
    for _ in range(K):
        rt.step_adjoint(U, dt, lam, out=lo)
    n = COPY_BYTES // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
    flush = torch.empty(n, dtype=torch.float64, device="cuda").fill_(2.0)  # evicts a from the last-level cache
    b = torch.empty_like(a)
    for _ in range(K):
        b.copy_(a)
        flush.fill_(3.0)
    torch.cuda.synchronize()
    print(f"drive done {nx}x{ny}x{B} K={K} step={step_tile} adj={adj_tile}", flush=True)


def _rows(d: str, name: str):
    fs = glob.glob(os.path.join(d, "**", name), recursive=True)
    if not fs:
        raise FileNotFoundError(f"{name} under {d}")
    with open(fs[0]) as f:
        return list(csv.DictReader(f))


def _kind(name: str) -> str | None:
    if "k_step" in name:
        return "step"
    if "k_adj_a" in name:
        return "adj_a"
    if "k_adj_b" in name:
        return "adj_b"
    if "copy" in name.lower() and "rtk" not in name:
        return "copy"
    return None


def _counter_avgs(dirs):
    counters: dict = {}
    for d in dirs:
        if d is None:
            continue
        for r in _rows(d, "*counter_collection.csv"):
            k = _kind(r["Kernel_Name"])
            if k:
                counters.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return counters


def summarize(workload: str, trace: str, fetch: str, write: str, req: str | None, out_md: str, command: str = ""):
    stats = {}
    for r in _rows(trace, "*kernel_stats.csv"):
        k = _kind(r["Name"])
        if k and k != "copy":
            stats[k] = (int(r["Calls"]), float(r["AverageNs"]) / 1e3, r["Name"])
    counters = _counter_avgs([fetch, write, req])
    avg = {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in counters.items()}
    cp = avg.get("copy", {})
    kib = COPY_BYTES / 1024
    f_scale = kib / cp["FETCH_SIZE"] if cp.get("FETCH_SIZE") else None
    w_scale = kib / cp["WRITE_SIZE"] if cp.get("WRITE_SIZE") else None

    def req_bytes(c):
        if "TCC_EA0_RDREQ_128B_sum" not in c:
            return None
        return 32 * c["TCC_EA0_RDREQ_32B_sum"] + 64 * c["TCC_EA0_RDREQ_64B_sum"] + 128 * c["TCC_EA0_RDREQ_128B_sum"]

    lines = [f"# HBM traffic and kernel times: {workload}", "", "Commands (repository root):", "", "```"]
    lines += command.strip().split("\n") if command else []
    lines += ["```", "",
              "| kernel | launches | avg us | FETCH_SIZE KiB | WRITE_SIZE KiB | read KiB from request sizes "
              "(32/64/128 B requests) |", "|---|---|---|---|---|---|"]
    for k in ("step", "adj_a", "adj_b", "copy"):
        c = avg.get(k, {})
        name, calls, us = (stats[k][2][:58], stats[k][0], f"{stats[k][1]:.3f}") if k in stats else (k, "", "")
        rb = req_bytes(c)
        rq = "" if rb is None else (f"{rb / 1024:.1f} ({c['TCC_EA0_RDREQ_32B_sum']:.0f}/"
                                    f"{c['TCC_EA0_RDREQ_64B_sum']:.0f}/{c['TCC_EA0_RDREQ_128B_sum']:.0f})")
        lines.append(f"| `{name}` | {calls} | {us} | {c.get('FETCH_SIZE', float('nan')):.1f} | "
                     f"{c.get('WRITE_SIZE', float('nan')):.1f} | {rq} |")
    lines += ["", f"Calibration: a plain copy of {COPY_BYTES} B (reads {COPY_BYTES} B, writes {COPY_BYTES} B, "
              f"source evicted from the last-level cache before each copy) reads FETCH_SIZE "
              f"{cp.get('FETCH_SIZE', float('nan')):.1f} KiB and WRITE_SIZE {cp.get('WRITE_SIZE', float('nan')):.1f} KiB "
              f"per dispatch: scale factors fetch {f_scale}, write {w_scale}."]
    entry = {}
    for name, parts in (("step", ["step"]), ("adjoint", ["adj_a", "adj_b"])):
        if all(p in avg for p in parts):
            fb = sum(avg[p].get("FETCH_SIZE", 0.0) for p in parts) * 1024 * (f_scale or 1.0)
            wb = sum(avg[p].get("WRITE_SIZE", 0.0) for p in parts) * 1024 * (w_scale or 1.0)
            rbs = [req_bytes(avg[p]) for p in parts]
            rb = None if any(x is None for x in rbs) else sum(rbs)
            entry[name] = {"fetch_bytes_scaled": fb, "write_bytes_scaled": wb, "bytes_per_launch": fb + wb,
                           "read_bytes_request_sizes": rb}
            lines.append(f"Per launch, {name}: scaled fetch {fb / 2**20:.2f} MiB + write {wb / 2**20:.2f} MiB = "
                         f"{(fb + wb) / 2**20:.2f} MiB"
                         + ("" if rb is None else f"; read bytes from request sizes {rb / 2**20:.2f} MiB"))
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    data = {}
    if os.path.exists(TRAFFIC_JSON):
        with open(TRAFFIC_JSON) as f:
            data = json.load(f)
    data[workload] = {"source_hash": kernel_source_hash(), "kernels": entry, "fetch_scale": f_scale,
                      "write_scale": w_scale,
                      "kernel_names": {k: v[2] for k, v in stats.items()}}
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(data, f, indent=1)
    print("\n".join(lines))


def traffic_for(workload: str, kernel: str) -> float | None:
    """Per-launch HBM bytes of `kernel` from the committed counters, or None
    if there are none or the kernel sources changed since they were taken."""
    try:
        with open(TRAFFIC_JSON) as f:
            d = json.load(f)[workload]
    except (OSError, KeyError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else float(k["bytes_per_launch"])


if __name__ == "__main__":
    if sys.argv[1] == "drive":
        nx, ny, B, K = (int(x) for x in sys.argv[2:6])
        drive(nx, ny, B, K, sys.argv[6], sys.argv[7])
    elif sys.argv[1] == "summarize":
        cmd = os.environ.get("RT_PROFILE_COMMAND", "")
        summarize(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6] or None, sys.argv[7], cmd)
    else:
        raise SystemExit(__doc__)
