"""CPU-side checks of the C-ABI library: it loads, exports every call that
include/rtcnop.h declares, rejects bad arguments without touching a GPU, and
its binomial checkpoint schedule is optimal (against a brute-force dynamic
program) and consistent."""
import ctypes
import functools
import os
import re

import pytest

from paper_2608_04085_amd import rtcnop

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "rtcnop.h")).read()
    return sorted(set(re.findall(r"\b(rt_[a-z0-9_]+)\s*\(", text)))


def test_header_calls_are_exported():
    L = rtcnop.load()
    names = _declared()
    assert "rt_grad_u0" in names and "rt_integrate" in names
    for n in names:
        assert hasattr(L, n), n
    for n in rtcnop.EXPORTED:
        assert n in names, n


def test_create_rejects_bad_grid_without_gpu():
    L = rtcnop.load()
    h = ctypes.c_void_p()
    g = rtcnop.RtGrid(2, 8, 1, 0, 0.5, 1.0)
    p = rtcnop.RtPhys(1.4, -0.1, 2.0, 1.0, 0.5, 0.01, 2.5, 0.4, 3, 0)
    assert L.rt_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == -1
    assert b"grid" in L.rt_last_error()
    g = rtcnop.RtGrid(8, 8, 1, 0, 0.5, 1.0)
    p.gamma = 1.0
    assert L.rt_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == -1
    p.gamma = 1.4
    p.recon = 2
    assert L.rt_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == -1
    assert b"recon" in L.rt_last_error()
    p.recon = 0
    assert L.rt_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == 0
    # calls that need a workspace refuse to run without one
    assert L.rt_kinetic_energy(h, ctypes.c_void_p(8), ctypes.c_void_p(8)) == -5
    # the gradient's time-step mode: frozen by default, two valid values
    mode = ctypes.c_int32(-1)
    assert L.rt_get_dt_mode(h, ctypes.byref(mode)) == 0 and mode.value == rtcnop.DT_MODES["frozen"]
    assert L.rt_set_dt_mode(h, 2) == -1 and b"dt mode" in L.rt_last_error()
    assert L.rt_set_dt_mode(h, rtcnop.DT_MODES["differentiated"]) == 0
    assert L.rt_get_dt_mode(h, ctypes.byref(mode)) == 0 and mode.value == 1
    assert L.rt_set_dt_mode(None, 0) == -1
    n = ctypes.c_size_t()
    assert L.rt_workspace_bytes(h, 100, ctypes.byref(n)) == 0 and n.value > 8 * 8 * 4 * 8 * 4
    assert L.rt_destroy(h) == 0


@functools.lru_cache(maxsize=None)
def _dp(l, c):
    # Brute force over recursive schedules: advance m steps, snapshot, reverse
    # the right part with one slot fewer, then the left part.
    if l <= 1:
        return 0
    if c <= 1:
        return l * (l - 1) // 2
    return min(m + _dp(l - m, c - 1) + _dp(m, c) for m in range(1, l))


@pytest.mark.parametrize("c", [1, 2, 3, 4, 5, 6])
def test_revolve_is_optimal_against_brute_force(c):
    for l in range(1, 41):
        fw, opt = rtcnop.revolve_stats(l, c)
        assert opt == _dp(l, c), (l, c)
        assert fw == opt, (l, c, fw, opt)


def test_revolve_large_schedules_are_consistent():
    # the march lengths of the benchmark workloads
    for l, c in [(1210, 8), (4838, 119), (19350, 119), (29024, 953), (5000, 2)]:
        fw, opt = rtcnop.revolve_stats(l, c)
        assert fw == opt
    # with as many slots as steps nothing is recomputed beyond one pass
    fw, _ = rtcnop.revolve_stats(100, 100)
    assert fw == 99


@functools.lru_cache(maxsize=None)
def _dp_cost(l, c):
    # the same brute force, for the segments of the two-level plan
    return _dp(l, c)


@pytest.mark.parametrize("n,c,n_est", [(1, 2, 1), (7, 2, 7), (40, 3, 40), (40, 5, 20), (120, 6, 100),
                                       (37, 4, 37), (200, 6, 30)])
def test_two_level_revolve_plan_is_consistent_and_segmentwise_optimal(n, c, n_est):
    # The plan of RT_CKPT_REVOLVE: the objective's march leaves snapshots
    # every I steps; each segment is reversed by a binomial schedule on the
    # free slots.  The replay inside the call checks that every step is
    # reversed once, in order, from the right state.  Its forward steps are
    # the march's n plus, per segment (last first), the brute-force optimum
    # for its length and the slots free then -- or, when that is dearer or
    # the snapshots do not fit, n plus the single binomial schedule.
    fw, I, two = rtcnop.revolve_plan_stats(n, c, n_est)
    K = -(-n // I)
    if two:
        free, seg = c - K, 0
        for k in range(K - 1, -1, -1):
            seg += _dp_cost(min(I, n - k * I), 1 + free)
            free += 1
        assert fw == n + seg
        assert K <= c - 1
    else:
        assert fw == n + _dp(n, c)
    assert fw <= n + _dp(n, c)


def test_two_level_revolve_at_the_workload_sizes():
    # The binomial checkpointing workloads (8 x 512 x 1024 under 16 GB: 119
    # states; 1024 x 2048 under 64 GB: 1024 states).  Against counting the
    # steps first and then one binomial schedule (n + t(n, c)), the two-level
    # plan saves re-computation, and an underestimated step count falls back
    # to that schedule.
    for n, c in [(4838, 119), (19350, 119), (29025, 1024), (1210, 8)]:
        fw, I, two = rtcnop.revolve_plan_stats(n, c, n)
        _, opt = rtcnop.revolve_stats(n, c)
        assert two and fw < n + opt, (n, c, fw, n + opt)
        print(f"revolve n={n} c={c}: interval {I}, forward steps {fw} ({fw / n:.2f} n) "
              f"against {n + opt} ({(n + opt) / n:.2f} n) counting first")
    # estimate far below the actual count: the snapshots overflow, fall back
    fw, I, two = rtcnop.revolve_plan_stats(4838, 119, 1000)
    _, opt = rtcnop.revolve_stats(4838, 119)
    assert not two and fw == 4838 + opt


def test_argument_validation_without_gpu():
    # every rejection below is decided on the host before any HIP call
    L = rtcnop.load()
    h = ctypes.c_void_p()
    p = rtcnop.RtPhys(1.4, -0.1, 2.0, 1.0, 0.5, 0.01, 2.5, 0.4, 3, 0)
    bad_grids = [rtcnop.RtGrid(8, 8, 0, 0, 0.5, 1.0),         # empty batch
                 rtcnop.RtGrid(8, 1, 1, 0, 0.5, 1.0),         # one row
                 rtcnop.RtGrid(16384, 16384, 1, 0, 0.5, 1.0),  # 2^28 cells: 32-bit plane offsets overflow
                 rtcnop.RtGrid(8, 8, 1, 0, -0.5, 1.0),        # negative length
                 rtcnop.RtGrid(8, 8, 1, 0, 0.5, 0.0)]         # zero length
    for g in bad_grids:
        assert L.rt_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == -1
    g = rtcnop.RtGrid(8, 8, 1, 0, 0.5, 1.0)
    for field, value in [("comp_mask", 0), ("comp_mask", 4), ("cfl", 0.0), ("h", 0.0), ("rho_l", -1.0)]:
        q = rtcnop.RtPhys(1.4, -0.1, 2.0, 1.0, 0.5, 0.01, 2.5, 0.4, 3, 0)
        setattr(q, field, value)
        assert L.rt_create(ctypes.byref(g), ctypes.byref(q), None, ctypes.byref(h)) == -1, field
    # the largest grid below the limit is accepted (nothing is allocated)
    big = rtcnop.RtGrid(16384, 16383, 1, 0, 0.5, 1.0)
    assert L.rt_create(ctypes.byref(big), ctypes.byref(p), None, ctypes.byref(h)) == 0
    assert L.rt_destroy(h) == 0
    assert L.rt_create(ctypes.byref(g), ctypes.byref(p), None, ctypes.byref(h)) == 0
    n = ctypes.c_size_t()
    assert L.rt_workspace_bytes(h, 0, ctypes.byref(n)) == -1
    assert L.rt_workspace_bytes(h, 64, ctypes.byref(n)) == 0
    # workspace: misaligned or too small, refused before it is touched
    assert L.rt_set_workspace(h, ctypes.c_void_p(256 + 8), n.value, 64) == -1
    assert b"aligned" in L.rt_last_error()
    assert L.rt_set_workspace(h, ctypes.c_void_p(256), n.value - 1, 64) == -3
    # checkpoint pools: unknown kind, bad interval
    assert L.rt_pool_bytes(h, 7, 32, 100, ctypes.byref(n)) == -1
    assert L.rt_pool_bytes(h, 1, 0, 100, ctypes.byref(n)) == -1
    assert L.rt_set_tiles(h, 0, 99) == -1 and L.rt_set_tile(h, -1) == -1
    # spectrum: a row outside -1 .. ny - 1
    assert L.rt_row_spectrum(h, ctypes.c_void_p(256), 64, 8, ctypes.c_void_p(256)) == -1
    assert L.rt_row_spectrum(h, ctypes.c_void_p(256), 64, -2, ctypes.c_void_p(256)) == -1
    assert L.rt_destroy(h) == 0
    # and a row wider than its LDS twiddle table
    wide = rtcnop.RtGrid(8192, 4, 1, 0, 0.5, 1.0)
    assert L.rt_create(ctypes.byref(wide), ctypes.byref(p), None, ctypes.byref(h)) == 0
    assert L.rt_row_spectrum(h, ctypes.c_void_p(256), 8192 * 4, -1, ctypes.c_void_p(256)) == -1
    assert b"4096" in L.rt_last_error()
    assert L.rt_destroy(h) == 0


def test_committed_counters_belong_to_the_kernel_sources():
    # profiles/traffic.json records the hash of the kernel sources it was
    # measured on; the benchmark reports its HBM traffic only while they match
    # and the tile variants (the defaults at each size)
    from paper_2608_04085_amd import profiling
    for workload, kernels, tiles in (("grad_256x512", ("step", "step_march", "adjoint"), "32x16/32x8"),
                                     ("cnop_8x512x1024", ("step_march", "adjoint"), "16x15/16x15"),
                                     ("step_8x1024x2048", ("step", "adjoint"), "16x15/16x15")):
        for k in kernels:
            t = profiling.traffic_for(workload, k, tiles)
            assert t is not None and t > 0, (workload, k)
    assert profiling.traffic_for("grad_256x512", "adjoint", "16x8/32x8") is None  # other tiles
    for title, tiles in (("cnop_8x512x1024", "16x15/16x15"), ("8x1024x2048", "16x15/16x15")):
        c = profiling.counters_for(title, ["adj_a", "adj_b"], tiles)
        assert c is not None and c["SQ_INSTS_VALU"] > 0, title
        assert profiling.counters_for(title, ["adj_a"], "32x16/32x8") is None


def test_header_declares_every_exported_call():
    # the C ABI is what the header declares: no call is defined without a
    # declaration there
    src = open(os.path.join(ROOT, "paper_2608_04085_amd", "csrc", "rt_api.hip")).read()
    defined = set(re.findall(r"^(?:int|const char\*)\s+(rt_[a-z0-9_]+)\s*\(", src[src.index('extern "C" {'):], re.M))
    assert defined and defined <= set(_declared()), sorted(defined - set(_declared()))
