"""Counter runs of the hot-path kernels and their summaries.

    python -m paper_2608_04085_amd.profiling drive NX NY B K STEP_TILE ADJ_TILE
        (STEP_TILE "auto": the autotuner's choice, as bench.py makes it.)
        The library's kernel-timing hook (K launches each of the step at a
        given dt, the march step, the folded adjoint step and the two-kernel
        adjoint step on one grid), then K copies of a 2 GiB buffer: a plain
        copy of known size whose FETCH_SIZE / WRITE_SIZE calibrate the
        counters.  Run it under rocprofv3: --kernel-trace, then --pmc
        FETCH_SIZE, then --pmc WRITE_SIZE, then --pmc TCC_EA0_RDREQ_32B_sum
        TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum TCC_EA0_RDREQ_sum.
    python -m paper_2608_04085_amd.profiling summarize WORKLOAD TRACE FETCH WRITE REQ OUT_MD
        Turns the four rocprofv3 CSV directories into a short Markdown summary
        and records per-launch HBM bytes in profiles/traffic.json, keyed by the
        hash of the kernel sources (bench.py reports the traffic only while the
        kernels are unchanged).  The command lines go in via the environment
        variable RT_PROFILE_COMMAND.
    python -m paper_2608_04085_amd.profiling stats TITLE TRACE OUT_MD
        Kernel times of a --kernel-trace run as Markdown, per kernel and grid.
    python -m paper_2608_04085_amd.profiling counters [--tiles=STEP/ADJ] TITLE DIR... OUT_MD
        Per-dispatch averages of the counters of --pmc runs, per kernel class,
        as Markdown and in profiles/counters.json under TITLE (keyed by the
        kernel-source hash and the tile variants, as the traffic is).

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
COUNTERS_JSON = os.path.join(ROOT, "profiles", "counters.json")
COPY_BYTES = 2 * 1024**3
CATEGORIES = ["step_given", "step_march", "adj_a_folded", "adj_a", "adj_b", "copy"]


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
    rt = Context(cfg, max_steps=64)
    U = rt.init_state(inputs.seed_batch(cfg, range(B), rms=1e-3))
    if step_tile == "auto":
        rt.autotune(U, reps=20)
    else:
        rt.set_tiles(step_tile, adj_tile)
    times = rt.kernel_times(U, reps=K)
    print(json.dumps({"grid": f"{nx}x{ny}x{B}", "tiles": rt.tile, "fold": rt.fold, "times_us": times}), flush=True)
    n = COPY_BYTES // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
    flush = torch.empty(n, dtype=torch.float64, device="cuda").fill_(2.0)  # evicts a from the last-level cache
    b = torch.empty_like(a)
    for _ in range(K):
        b.copy_(a)
        flush.fill_(3.0)
    torch.cuda.synchronize()
    print(f"drive done {nx}x{ny}x{B} K={K} tiles={rt.tile} {json.dumps(times)}", flush=True)


def _rows(d: str, name: str):
    fs = glob.glob(os.path.join(d, "**", name), recursive=True)
    if not fs:
        raise FileNotFoundError(f"{name} under {d}")
    with open(fs[0]) as f:
        return list(csv.DictReader(f))


def _classify(rows):
    """Category of each dispatch, in dispatch order: steps after the march
    set-up kernel are march steps; an adjoint kernel A followed by kernel B
    is the two-kernel form, otherwise the folded one; copies after the last
    library kernel are the calibration copies."""
    disp = {}
    for r in rows:
        disp.setdefault(int(r["Dispatch_Id"]), r["Kernel_Name"])
    order = sorted(disp)
    last_lib = max([d for d in order if "rtk::" in disp[d]], default=-1)
    cat = {}
    march = False
    for i, d in enumerate(order):
        n = disp[d]
        if "k_march_begin" in n:
            march = True
        if "k_step" in n:
            cat[d] = "step_march" if march else "step_given"
        elif "k_adj_a" in n:
            nxt = disp[order[i + 1]] if i + 1 < len(order) else ""
            cat[d] = "adj_a" if "k_adj_b" in nxt else "adj_a_folded"
        elif "k_adj_b" in n:
            cat[d] = "adj_b"
        elif "copyBuffer" in n and d > last_lib:
            cat[d] = "copy"  # the calibration copies come after every library kernel
    return cat


def summarize(workload: str, trace: str, fetch: str, write: str, req: str | None, out_md: str, command: str = "",
              tiles: str = ""):
    trows = _rows(trace, "*kernel_trace.csv")
    tcat = _classify(trows)
    dur: dict = {}
    meta: dict = {}
    tbig = max((int(r["Grid_Size_X"]) for r in trows if tcat.get(int(r["Dispatch_Id"])) == "copy"), default=0)
    for r in trows:
        c = tcat.get(int(r["Dispatch_Id"]))
        if c == "copy" and int(r["Grid_Size_X"]) < tbig:
            continue
        if c:
            dur.setdefault(c, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
            meta[c] = (r["Kernel_Name"], r["LDS_Block_Size"], r["VGPR_Count"], r["Workgroup_Size_X"])
    counters: dict = {}
    for d in (fetch, write, req):
        if not d:
            continue
        crows = _rows(d, "*counter_collection.csv")
        ccat = _classify(crows)
        # calibration copies: the largest copy dispatches only
        big = max((int(r["Grid_Size"]) for r in crows if ccat.get(int(r["Dispatch_Id"])) == "copy"), default=0)
        for r in crows:
            c = ccat.get(int(r["Dispatch_Id"]))
            if c == "copy" and int(r["Grid_Size"]) < big:
                continue
            if c:
                counters.setdefault(c, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
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
              "| kernel (launch form) | name | threads | LDS B | VGPR | launches | avg us | FETCH_SIZE KiB | "
              "WRITE_SIZE KiB | read KiB from request sizes (n32/n64/n128) |",
              "|---|---|---|---|---|---|---|---|---|---|"]
    for k in CATEGORIES:
        if k not in dur and k not in avg:
            continue
        c = avg.get(k, {})
        name, lds, vgpr, wg = meta.get(k, ("", "", "", ""))
        name = name.replace("rtk::(anonymous namespace)::", "").split("(")[0]
        ds = dur.get(k, [])
        us = f"{sum(ds) / len(ds):.3f}" if ds else ""
        rb = req_bytes(c)
        rq = "" if rb is None else (f"{rb / 1024:.1f} ({c['TCC_EA0_RDREQ_32B_sum']:.0f}/"
                                    f"{c['TCC_EA0_RDREQ_64B_sum']:.0f}/{c['TCC_EA0_RDREQ_128B_sum']:.0f})")
        lines.append(f"| {k} | `{name}` | {wg} | {lds} | {vgpr} | {len(ds)} | {us} | "
                     f"{c.get('FETCH_SIZE', float('nan')):.1f} | {c.get('WRITE_SIZE', float('nan')):.1f} | {rq} |")
    lines += ["", f"Calibration: a plain copy of {COPY_BYTES} B (reads {COPY_BYTES} B, writes {COPY_BYTES} B, "
              f"source evicted from the last-level cache before each copy) reads FETCH_SIZE "
              f"{cp.get('FETCH_SIZE', float('nan')):.1f} KiB and WRITE_SIZE {cp.get('WRITE_SIZE', float('nan')):.1f} "
              f"KiB per dispatch: scale factors fetch {f_scale}, write {w_scale}.", ""]
    entry = {}
    for name, parts in (("step", ["step_given"]), ("step_march", ["step_march"]), ("adjoint", ["adj_a", "adj_b"]),
                        ("adjoint_folded", ["adj_a_folded"])):
        if all(p in avg for p in parts):
            fb = sum(avg[p].get("FETCH_SIZE", 0.0) for p in parts) * 1024 * (f_scale or 1.0)
            wb = sum(avg[p].get("WRITE_SIZE", 0.0) for p in parts) * 1024 * (w_scale or 1.0)
            rbs = [req_bytes(avg[p]) for p in parts]
            rb = None if any(x is None for x in rbs) else sum(rbs)
            us = sum(sum(dur[p]) / len(dur[p]) for p in parts if p in dur)
            entry[name] = {"fetch_bytes_scaled": fb, "write_bytes_scaled": wb, "bytes_per_launch": fb + wb,
                           "read_bytes_request_sizes": rb, "avg_us": us}
            lines.append(f"Per launch, {name}: {us:.3f} us; scaled fetch {fb / 2**20:.2f} MiB + write "
                         f"{wb / 2**20:.2f} MiB = {(fb + wb) / 2**20:.2f} MiB"
                         + ("" if rb is None else f"; read bytes from request sizes {rb / 2**20:.2f} MiB"))
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    data = {}
    if os.path.exists(TRAFFIC_JSON):
        with open(TRAFFIC_JSON) as f:
            data = json.load(f)
    data[workload] = {"source_hash": kernel_source_hash(), "tiles": tiles, "kernels": entry, "fetch_scale": f_scale,
                      "write_scale": w_scale, "kernel_names": {k: v[0] for k, v in meta.items()}}
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(data, f, indent=1)
    print("\n".join(lines))


def traffic_for(workload: str, kernel: str, tiles: str | None = None) -> float | None:
    """Per-launch HBM bytes of `kernel` from the committed counters, or None
    if there are none, the kernel sources changed since they were taken, or
    they were taken with other tile variants than `tiles`."""
    try:
        with open(TRAFFIC_JSON) as f:
            d = json.load(f)[workload]
    except (OSError, KeyError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    if tiles is not None and d.get("tiles") and d["tiles"] != tiles:
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else float(k["bytes_per_launch"])


def stats_md(title: str, trace: str, out_md: str, command: str = "", top: int = 14):
    """Kernel statistics of a --kernel-trace run as Markdown, one row per
    kernel and launch grid (so that launches over different batch sizes are
    not averaged together)."""
    rows = _rows(trace, "*kernel_trace.csv")
    groups: dict = {}
    total = 0.0
    for r in rows:
        key = (r["Kernel_Name"], f"{r['Grid_Size_X']}x{r['Grid_Size_Y']}x{r['Grid_Size_Z']}", r["Workgroup_Size_X"])
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
        groups.setdefault(key, []).append(d)
        total += d
    order = sorted(groups, key=lambda k: -sum(groups[k]))
    lines = [f"# Kernel time: {title}", "", "Command (repository root):", "", "```"]
    lines += command.strip().split("\n") if command else []
    lines += ["```", "", "One row per kernel and launch grid (threads: grid size in threads x, y, z).", "",
              "| kernel | grid (threads) | block | calls | total ms | avg us | min us | max us | share % |",
              "|---|---|---|---|---|---|---|---|---|"]
    for k in order[:top]:
        v = groups[k]
        name = k[0].replace("rtk::(anonymous namespace)::", "").split("(")[0]
        lines.append(f"| `{name[:60]}` | {k[1]} | {k[2]} | {len(v)} | {sum(v) * 1e-3:.3f} | {sum(v) / len(v):.3f} | "
                     f"{min(v):.3f} | {max(v):.3f} | {100 * sum(v) / total:.2f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def counters_md(title: str, dirs: list, out_md: str, command: str = "", tiles: str = ""):
    """Per-dispatch averages of every collected counter, per kernel class."""
    per: dict = {}
    for d in dirs:
        rows = _rows(d, "*counter_collection.csv")
        cat = _classify(rows)
        for r in rows:
            c = cat.get(int(r["Dispatch_Id"]))
            if c and c != "copy":
                per.setdefault(c, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    names = sorted({n for v in per.values() for n in v})
    lines = [f"# Counters: {title}" + (f" (tiles {tiles})" if tiles else ""), "", "Commands (repository root):", "",
             "```"]
    lines += command.strip().split("\n") if command else []
    lines += ["```", "", "Per-dispatch averages.", "", "| counter | " + " | ".join(k for k in CATEGORIES if k in per) + " |",
              "|---|" + "---|" * len([k for k in CATEGORIES if k in per])]
    for n in names:
        vals = []
        for k in CATEGORIES:
            if k in per:
                v = per[k].get(n)
                vals.append("" if not v else f"{sum(v) / len(v):.4g}")
        lines.append(f"| {n} | " + " | ".join(vals) + " |")
    # where the wavefronts' cycles go, when the run has the wait counters
    fr = ["SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_SCA", "SQ_ACTIVE_INST_LDS", "SQ_WAIT_INST_ANY",
          "SQ_WAIT_ANY", "SQ_WAIT_INST_LDS"]
    ks = [k for k in CATEGORIES if k in per and "SQ_WAVE_CYCLES" in per[k] and "SQ_WAIT_ANY" in per[k]]
    if ks:
        lines += ["", "Fractions of SQ_WAVE_CYCLES (per dispatch):", "", "| counter / SQ_WAVE_CYCLES | " + " | ".join(ks) +
                  " |", "|---|" + "---|" * len(ks)]
        for n in fr:
            vals = []
            for k in ks:
                v, w = per[k].get(n), per[k]["SQ_WAVE_CYCLES"]
                vals.append("" if not v else f"{(sum(v) / len(v)) / (sum(w) / len(w)):.3f}")
            lines.append(f"| {n} | " + " | ".join(vals) + " |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    data = {}
    if os.path.exists(COUNTERS_JSON):
        with open(COUNTERS_JSON) as f:
            data = json.load(f)
    data[title] = {"source_hash": kernel_source_hash(), "tiles": tiles,
                   "per_dispatch": {k: {n: sum(v) / len(v) for n, v in d.items()} for k, d in per.items()}}
    with open(COUNTERS_JSON, "w") as f:
        json.dump(data, f, indent=1)
    print("\n".join(lines))


def counters_for(title: str, parts, tiles: str | None = None) -> dict | None:
    """Per-launch sums over the kernel classes `parts` of the counters of
    the committed --pmc runs titled `title`, or None if there are none, the
    kernel sources changed since they were taken, or they were taken with
    other tile variants than `tiles`."""
    try:
        with open(COUNTERS_JSON) as f:
            d = json.load(f)[title]
    except (OSError, KeyError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    if tiles is not None and d.get("tiles") and d["tiles"] != tiles:
        return None
    per = d.get("per_dispatch", {})
    if not all(p in per for p in parts):
        return None
    names = set().union(*(per[p].keys() for p in parts))
    return {n: sum(per[p].get(n, 0.0) for p in parts) for n in names}


if __name__ == "__main__":
    if sys.argv[1] == "drive":
        nx, ny, B, K = (int(x) for x in sys.argv[2:6])
        drive(nx, ny, B, K, sys.argv[6], sys.argv[7])
    elif sys.argv[1] == "summarize":
        cmd = os.environ.get("RT_PROFILE_COMMAND", "")
        tiles = sys.argv[8] if len(sys.argv) > 8 else ""
        summarize(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6] or None, sys.argv[7], cmd, tiles)
    elif sys.argv[1] == "stats":
        stats_md(sys.argv[2], sys.argv[3], sys.argv[4], os.environ.get("RT_PROFILE_COMMAND", ""))
    elif sys.argv[1] == "counters":
        args = sys.argv[2:]
        tl = args.pop(0)[len("--tiles="):] if args and args[0].startswith("--tiles=") else ""
        counters_md(args[0], args[1:-1], args[-1], os.environ.get("RT_PROFILE_COMMAND", ""), tl)
    else:
        raise SystemExit(__doc__)
