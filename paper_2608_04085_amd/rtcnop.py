"""Thin Python binding of ``librtcnop.so`` (the C ABI of include/rtcnop.h).

Argument marshalling only: torch supplies device memory and the stream, and
every step of the hot path runs in the library's HIP kernels.  There is no
CPU fallback: :func:`load` raises if the library is missing, and every call
raises :class:`RTError` on a non-zero status.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import torch

from .config import (CKPT_REVOLVE, CKPT_STORE_ALL, CKPT_UNIFORM, NORM_L2, SET_SPHERE, RTConfig)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtcnop.so")

STATUS = {0: "RT_OK", -1: "RT_EINVAL", -2: "RT_EHIP", -3: "RT_ENOMEM", -4: "RT_EUNPHYS", -5: "RT_ESTATE"}
TILES = {"16x16": 0, "32x8": 1, "64x4": 2, "16x16w": 3, "32x8w": 4, "16x8": 5, "8x8": 6, "16x8w": 7, "8x8w": 8, "32x16": 9,
         "16x15": 10, "15x16": 11}
DT_MODES = {"frozen": 0, "differentiated": 1}
DT_MODES_BY_ID = {v: k for k, v in DT_MODES.items()}


class RTError(RuntimeError):
    def __init__(self, code: int, call: str, msg: str):
        super().__init__(f"{call}: {STATUS.get(code, code)}: {msg}")
        self.code = code


class RtGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("lx", ctypes.c_double), ("ly", ctypes.c_double)]


class RtPhys(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("g_y", ctypes.c_double), ("rho_h", ctypes.c_double),
                ("rho_l", ctypes.c_double), ("y0", ctypes.c_double), ("h", ctypes.c_double),
                ("p_int", ctypes.c_double), ("cfl", ctypes.c_double), ("comp_mask", ctypes.c_int32),
                ("recon", ctypes.c_int32)]


class RtCkptPolicy(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("interval", ctypes.c_int32), ("pool", ctypes.c_void_p),
                ("pool_bytes", ctypes.c_size_t)]


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32


def load():
    """Load the HIP library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2608_04085_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "rt_create": [ctypes.POINTER(RtGrid), ctypes.POINTER(RtPhys), _vp, ctypes.POINTER(_vp)],
        "rt_destroy": [_vp],
        "rt_set_stream": [_vp, _vp],
        "rt_set_tile": [_vp, _i32],
        "rt_get_tile": [_vp, ctypes.POINTER(_i32)],
        "rt_get_tiles": [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
        "rt_autotune": [_vp, _vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
        "rt_workspace_bytes": [_vp, _i32, ctypes.POINTER(ctypes.c_size_t)],
        "rt_set_workspace": [_vp, _vp, ctypes.c_size_t, _i32],
        "rt_init_state": [_vp, _vp, _vp],
        "rt_cfl_dt": [_vp, _vp, _vp],
        "rt_step": [_vp, _vp, _vp, _vp, _vp],
        "rt_integrate": [_vp, _vp, ctypes.c_double, _vp, _vp, _vp, _i32],
        "rt_kinetic_energy": [_vp, _vp, _vp],
        "rt_ke_ratio": [_vp, _vp, _vp, _vp],
        "rt_ke_ratio_noalloc": [_vp, _vp, _vp, _vp],
        "rt_step_adjoint": [_vp, _vp, _vp, _vp, _vp],
        "rt_grad_u0": [_vp, _vp, ctypes.c_double, ctypes.POINTER(RtCkptPolicy), _vp, _vp, _vp],
        "rt_pool_bytes": [_vp, _i32, _i32, _i32, ctypes.POINTER(ctypes.c_size_t)],
        "rt_project_to_constraint": [_vp, _vp, ctypes.c_double, _i32, _i32, _vp],
        "rt_dot": [_vp, _vp, _vp, _vp],
        "rt_max_abs": [_vp, _vp, _vp],
        "rt_set_graphs": [_vp, _i32],
        "rt_set_overlap": [_vp, _i32],
        "rt_kernel_times": [_vp, _vp, _i32, ctypes.POINTER(ctypes.c_double)],
        "rt_set_fold": [_vp, _i32],
        "rt_set_tiles": [_vp, _i32, _i32],
        "rt_ek_field": [_vp, _vp, _vp],
        "rt_mix_width": [_vp, _vp, _vp],
        "rt_row_spectrum": [_vp, _vp, ctypes.c_int64, _i32, _vp],
        "rt_power_spectrum_2d": [_vp, _vp, ctypes.c_int64, _vp],
        "rt_ek_anomaly": [_vp, _vp, _vp, _vp],
        "rt_grad_ek_anomaly": [_vp, _vp, ctypes.c_double, _vp, _vp, _vp, _vp, _vp],
        "rt_get_fold": [_vp, ctypes.POINTER(_i32)],
        "rt_set_dt_mode": [_vp, _i32],
        "rt_get_dt_mode": [_vp, ctypes.POINTER(_i32)],
        "rt_axpy": [_vp, _vp, _vp, _vp, _vp],
        "rt_check_error": [_vp],
        "rt_revolve_stats": [_i32, _i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
        "rt_revolve_plan_stats": [_i32, _i32, _i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_i32),
                                  ctypes.POINTER(_i32)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.rt_last_error.argtypes = []
    L.rt_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


EXPORTED = ["rt_create", "rt_destroy", "rt_set_stream", "rt_workspace_bytes", "rt_set_workspace",
            "rt_init_state", "rt_cfl_dt", "rt_step", "rt_integrate", "rt_kinetic_energy", "rt_step_adjoint",
            "rt_grad_u0", "rt_pool_bytes", "rt_project_to_constraint", "rt_dot", "rt_axpy", "rt_check_error",
            "rt_last_error", "rt_set_tile", "rt_get_tiles", "rt_autotune", "rt_max_abs", "rt_set_graphs",
            "rt_set_overlap", "rt_kernel_times", "rt_set_fold", "rt_get_fold",
            "rt_set_tiles", "rt_ek_field", "rt_ek_anomaly", "rt_grad_ek_anomaly",
            "rt_mix_width", "rt_set_dt_mode", "rt_get_dt_mode", "rt_get_tile", "rt_revolve_stats",
            "rt_row_spectrum", "rt_ke_ratio", "rt_revolve_plan_stats", "rt_ke_ratio_noalloc",
            "rt_power_spectrum_2d"]


def _check(rc: int, call: str):
    if rc != 0:
        msg = load().rt_last_error()
        raise RTError(rc, call, msg.decode() if msg else "")


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA/HIP tensors"
    return ctypes.c_void_p(t.data_ptr())


def revolve_stats(nsteps: int, slots: int):
    """(forward steps of the library's binomial schedule, the closed-form
    minimum) for reversing `nsteps` steps with `slots` checkpoint slots; the
    call also checks the schedule's consistency (host only, no GPU)."""
    fw = ctypes.c_int64()
    opt = ctypes.c_int64()
    _check(load().rt_revolve_stats(nsteps, slots, ctypes.byref(fw), ctypes.byref(opt)), "rt_revolve_stats")
    return fw.value, opt.value


def revolve_plan_stats(nsteps: int, slots: int, n_est: int):
    """(forward steps of the whole gradient, level-1 interval, two-level
    plan used) of RT_CKPT_REVOLVE for a march of nsteps steps with `slots`
    slots when the initial CFL step suggested n_est steps; the plan is also
    checked for consistency (host only, no GPU)."""
    fw = ctypes.c_int64()
    iv = ctypes.c_int32()
    two = ctypes.c_int32()
    _check(load().rt_revolve_plan_stats(nsteps, slots, n_est, ctypes.byref(fw), ctypes.byref(iv), ctypes.byref(two)),
           "rt_revolve_plan_stats")
    return fw.value, iv.value, bool(two.value)


@dataclass
class Policy:
    kind: int = CKPT_UNIFORM
    interval: int = 32
    pool_bytes: int | None = None  # None: what the policy needs for max_steps


class Context:
    """One grid / physics / stream; owns its workspace tensor."""

    def __init__(self, cfg: RTConfig, max_steps: int = 65536, device: str | int = "cuda", tile: str | None = None):
        self.cfg = cfg
        dev = torch.device(device) if not isinstance(device, int) else torch.device("cuda", device)
        if dev.type != "cuda":
            raise ValueError(f"the library runs on a HIP device, not {dev}")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.max_steps = int(max_steps)
        self._own_pool = None  # checkpoint pool of gradient calls made without one
        L = load()
        grid = RtGrid(cfg.nx, cfg.ny, cfg.batch, 0, cfg.lx, cfg.ly)
        phys = RtPhys(cfg.gamma, cfg.g_y, cfg.rho_h, cfg.rho_l, cfg.y0, cfg.h, cfg.p_int, cfg.cfl, cfg.comp_mask,
                      cfg.recon)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):  # rt_set_workspace launches its set-up on the current device
            _check(L.rt_create(ctypes.byref(grid), ctypes.byref(phys), self._stream(), ctypes.byref(h)),
                   "rt_create")
            self._h = h
            if tile is not None:
                _check(L.rt_set_tile(h, TILES[tile]), "rt_set_tile")
            n = ctypes.c_size_t()
            _check(L.rt_workspace_bytes(h, self.max_steps, ctypes.byref(n)), "rt_workspace_bytes")
            self.ws = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
            off = (-self.ws.data_ptr()) % 256
            self._ws_ptr = ctypes.c_void_p(self.ws.data_ptr() + off)
            _check(L.rt_set_workspace(h, self._ws_ptr, n.value, self.max_steps), "rt_set_workspace")

    def __del__(self):
        try:
            if getattr(self, "_h", None) is not None and _lib is not None:
                _lib.rt_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def _stream(self):
        if not torch.cuda.is_available():
            return None
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def _sync_stream(self):
        # the library launches on the current device: refuse to run on another
        if torch.cuda.current_device() != self.device.index:
            raise RuntimeError(f"the context lives on {self.device}; make it the current device "
                               f"(torch.cuda.set_device) before calling it")
        _check(load().rt_set_stream(self._h, self._stream()), "rt_set_stream")

    # ---------------------------------------------------------------- shapes
    @property
    def shape_u(self):
        return (self.cfg.batch, 4, self.cfg.ny, self.cfg.nx)

    @property
    def shape_uv(self):
        return (self.cfg.batch, 2, self.cfg.ny, self.cfg.nx)

    def _f64(self, shape):
        return torch.empty(shape, dtype=torch.float64, device=self.device)

    def as_dev(self, a) -> torch.Tensor:
        if isinstance(a, torch.Tensor):
            return a.to(device=self.device, dtype=torch.float64).contiguous()
        return torch.as_tensor(a, dtype=torch.float64, device=self.device).contiguous()

    @property
    def tile(self) -> str:
        """Tile variants in use, "step/adjoint"."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(load().rt_get_tiles(self._h, ctypes.byref(a), ctypes.byref(b)), "rt_get_tiles")
        names = {v: k for k, v in TILES.items()}
        return f"{names[a.value]}/{names[b.value]}"

    def set_tile(self, name: str):
        _check(load().rt_set_tile(self._h, TILES[name]), "rt_set_tile")

    def set_tiles(self, step: str, adjoint: str):
        _check(load().rt_set_tiles(self._h, TILES[step], TILES[adjoint]), "rt_set_tiles")

    def set_graphs(self, on: bool):
        _check(load().rt_set_graphs(self._h, 1 if on else 0), "rt_set_graphs")

    def kernel_times(self, U, reps: int = 100) -> dict:
        """Per-launch microseconds of the selected variants (HIP events on the
        context's stream): given-dt step, march step, folded adjoint step
        (the reverse sweep's kernel), rt_step_adjoint (two kernels)."""
        self._sync_stream()
        U = self.as_dev(U)
        out = (ctypes.c_double * 5)()
        _check(load().rt_kernel_times(self._h, _ptr(U), int(reps), out), "rt_kernel_times")
        return {"step_given_us": out[0], "step_march_us": out[1], "adjoint_folded_us": out[2],
                "adjoint_two_kernel_us": out[3], "adjoint_sweep_us": out[4]}

    @property
    def fold(self) -> bool:
        """Reverse sweep with the limiter gather folded into the next adjoint kernel."""
        v = ctypes.c_int32()
        _check(load().rt_get_fold(self._h, ctypes.byref(v)), "rt_get_fold")
        return bool(v.value)

    def set_fold(self, on: bool):
        _check(load().rt_set_fold(self._h, 1 if on else 0), "rt_set_fold")

    @property
    def dt_mode(self) -> str:
        """"frozen" (the forward run's steps held fixed in the gradient, the
        default) or "differentiated" (the gradient of the adaptive march)."""
        v = ctypes.c_int32()
        _check(load().rt_get_dt_mode(self._h, ctypes.byref(v)), "rt_get_dt_mode")
        return DT_MODES_BY_ID[v.value]

    def set_dt_mode(self, mode: str):
        _check(load().rt_set_dt_mode(self._h, DT_MODES[mode]), "rt_set_dt_mode")

    def set_overlap(self, on: bool):
        """Second stream in the reverse sweep (default on): the UNIFORM policy re-computes the next segment on
        it, REVOLVE runs half of the members on it; results are identical."""
        _check(load().rt_set_overlap(self._h, 1 if on else 0), "rt_set_overlap")

    def autotune(self, U, reps: int = 20) -> str:
        """Time every kernel variant on U and keep the fastest (bitwise-identical results)."""
        self._sync_stream()
        U = self.as_dev(U)
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(load().rt_autotune(self._h, _ptr(U), int(reps), ctypes.byref(a), ctypes.byref(b)), "rt_autotune")
        return self.tile

    # ---------------------------------------------------------------- calls
    def init_state(self, uv0) -> torch.Tensor:
        self._sync_stream()
        uv0 = self.as_dev(uv0).reshape(self.shape_uv)
        U = self._f64(self.shape_u)
        _check(load().rt_init_state(self._h, _ptr(uv0), _ptr(U)), "rt_init_state")
        return U

    def cfl_dt(self, U) -> torch.Tensor:
        self._sync_stream()
        U = self.as_dev(U)
        dt = self._f64((self.cfg.batch,))
        _check(load().rt_cfl_dt(self._h, _ptr(U), _ptr(dt)), "rt_cfl_dt")
        return dt

    def _dt(self, dt) -> torch.Tensor:
        """Per-member step sizes as a device [B] tensor (passed through when it already is one)."""
        if (isinstance(dt, torch.Tensor) and dt.is_cuda and dt.dtype == torch.float64 and dt.is_contiguous()
                and dt.numel() == self.cfg.batch):
            return dt
        return self.as_dev(torch.as_tensor(dt, dtype=torch.float64).expand(self.cfg.batch).clone())

    def step(self, U, dt=None, want_next: bool = False, out: torch.Tensor | None = None):
        self._sync_stream()
        U = self.as_dev(U)
        Un = torch.empty_like(U) if out is None else out
        dtp = None
        if dt is not None:
            dtp = self._dt(dt)
        nxt = self._f64((self.cfg.batch,)) if want_next else None
        _check(load().rt_step(self._h, _ptr(U), _ptr(Un), _ptr(dtp), _ptr(nxt)), "rt_step")
        return (Un, nxt) if want_next else Un

    def integrate(self, U, T: float, log_cap: int = 0):
        """(U(T), t, nsteps, dt_log or None); U is not modified."""
        self._sync_stream()
        U = self.as_dev(U).clone()
        t = self._f64((self.cfg.batch,))
        n = torch.empty((self.cfg.batch,), dtype=torch.int32, device=self.device)
        log = self._f64((self.cfg.batch, log_cap)) if log_cap > 0 else None
        _check(load().rt_integrate(self._h, _ptr(U), float(T), _ptr(t), _ptr(n), _ptr(log), int(log_cap)),
               "rt_integrate")
        return U, t, n, log

    def kinetic_energy(self, U) -> torch.Tensor:
        self._sync_stream()
        U = self.as_dev(U)
        ke = self._f64((self.cfg.batch,))
        _check(load().rt_kinetic_energy(self._h, _ptr(U), _ptr(ke)), "rt_kinetic_energy")
        return ke

    def ke_ratio(self, U0, UT) -> torch.Tensor:
        """R[B] = KE(UT)/KE(U0) (the library's rt_ke_ratio)."""
        self._sync_stream()
        U0 = self.as_dev(U0)
        UT = self.as_dev(UT)
        R = self._f64((self.cfg.batch,))
        _check(load().rt_ke_ratio(self._h, _ptr(U0), _ptr(UT), _ptr(R)), "rt_ke_ratio")
        return R

    def ke_ratio_noalloc(self, U0, UT, out: torch.Tensor) -> torch.Tensor:
        """rt_ke_ratio_noalloc: R[B] into `out` (device, [B]) with the
        library's static scratch; U0 and UT must already be contiguous
        float64 device tensors (nothing is allocated)."""
        self._sync_stream()
        _check(load().rt_ke_ratio_noalloc(self._h, _ptr(U0), _ptr(UT), _ptr(out)), "rt_ke_ratio_noalloc")
        return out

    def objective_ratio(self, uv0, T: float) -> torch.Tensor:
        """R = KE(U(T))/KE(U(0)) of every member for the perturbation uv0
        (forward march only)."""
        U0 = self.init_state(uv0)
        UT, _, _, _ = self.integrate(U0, T)
        return self.ke_ratio(U0, UT)

    def step_adjoint(self, U, dt, lam_next, out: torch.Tensor | None = None) -> torch.Tensor:
        self._sync_stream()
        U = self.as_dev(U)
        lam_next = self.as_dev(lam_next)
        dtp = self._dt(dt)
        lam = torch.empty_like(lam_next) if out is None else out
        _check(load().rt_step_adjoint(self._h, _ptr(U), _ptr(dtp), _ptr(lam_next), _ptr(lam)), "rt_step_adjoint")
        return lam

    def pool_bytes(self, kind: int, interval: int, nsteps_max: int) -> int:
        n = ctypes.c_size_t()
        _check(load().rt_pool_bytes(self._h, kind, interval, nsteps_max, ctypes.byref(n)), "rt_pool_bytes")
        return n.value

    def grad_u0(self, uv0, T: float, policy: Policy | None = None, pool: torch.Tensor | None = None):
        """(R[B], grad[B][2][ny][nx], nsteps[B]) on the device.  Without a
        pool the context sizes one for the run (see _pool) and keeps it."""
        self._sync_stream()
        policy = policy or Policy()
        uv0 = self.as_dev(uv0).reshape(self.shape_uv)
        if pool is None:
            return self._with_own_pool(policy, uv0, T, lambda pl, pol: load().rt_grad_u0(
                self._h, _ptr(uv0), float(T), ctypes.byref(pol), _ptr(pl[0]), _ptr(pl[1]), _ptr(pl[2])),
                "rt_grad_u0")
        pool, pol = self._pool(policy, pool)
        R = self._f64((self.cfg.batch,))
        g = self._f64(self.shape_uv)
        n = torch.empty((self.cfg.batch,), dtype=torch.int32, device=self.device)
        _check(load().rt_grad_u0(self._h, _ptr(uv0), float(T), ctypes.byref(pol), _ptr(R), _ptr(g), _ptr(n)),
               "rt_grad_u0")
        return R, g, n

    def _step_estimate(self, uv0, T: float) -> int:
        """Steps a march of uv0 to T will take, with room to spare: 1.25 T /
        dt0 + 64 from the CFL step dt0 of the initial state (the signal
        speeds of these runs are set by the background's sound speed, so
        dt changes little along the march)."""
        dt0 = float(self.cfl_dt(self.init_state(uv0)).min())
        return min(self.max_steps, int(math.ceil(1.25 * T / dt0)) + 64)

    def _with_own_pool(self, policy, uv0, T, call, name):
        """Run a gradient call with a pool the context sizes and keeps:
        policy.pool_bytes if given, else what the policy needs for the
        estimated step count; on RT_ENOMEM (more steps than estimated) once
        more with the exact count from a forward march."""
        out = (self._f64((self.cfg.batch,)), self._f64(self.shape_uv),
               torch.empty((self.cfg.batch,), dtype=torch.int32, device=self.device))
        need = policy.pool_bytes or self.pool_bytes(policy.kind, policy.interval, self._step_estimate(uv0, T))
        for attempt in range(2):
            if self._own_pool is None or self._own_pool.numel() < need + 256:
                self._own_pool = None
                self._own_pool = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
            _, pol = self._pool(policy, self._own_pool)
            rc = call(out, pol)
            if rc != -3 or attempt == 1 or policy.pool_bytes:
                _check(rc, name)
                return out
            _, _, n, _ = self.integrate(self.init_state(uv0), T)
            need = self.pool_bytes(policy.kind, policy.interval, int(n.max().item()))
        return out

    def _pool(self, policy, pool):
        if pool is None:
            nbytes = policy.pool_bytes or self.pool_bytes(policy.kind, policy.interval, self.max_steps)
            pool = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        if pool.device != self.device or not pool.is_contiguous():
            raise ValueError("the checkpoint pool must be a contiguous tensor on the context's device")
        off = (-pool.data_ptr()) % 256
        nbytes = pool.numel() * pool.element_size() - off
        if nbytes <= 0:
            raise ValueError("checkpoint pool too small")
        return pool, RtCkptPolicy(policy.kind, policy.interval, ctypes.c_void_p(pool.data_ptr() + off), nbytes)

    def ek_field(self, U) -> torch.Tensor:
        """Kinetic-energy density e_k = |m|^2/(2 rho) of every cell, [B][ny][nx] (Eq. 7)."""
        self._sync_stream()
        U = self.as_dev(U)
        ek = self._f64((self.cfg.batch, self.cfg.ny, self.cfg.nx))
        _check(load().rt_ek_field(self._h, _ptr(U), _ptr(ek)), "rt_ek_field")
        return ek

    def mix_width(self, U) -> torch.Tensor:
        """Mixing-layer width h_mix[B] of Eqs. 13-14."""
        self._sync_stream()
        U = self.as_dev(U)
        h = self._f64((self.cfg.batch,))
        _check(load().rt_mix_width(self._h, _ptr(U), _ptr(h)), "rt_mix_width")
        return h

    def row_spectrum(self, field, row: int = -1, component: int | None = None) -> torch.Tensor:
        """E[B][nx/2 + 1] of Eq. 12 before normalisation: the squared modulus
        of each row's horizontal Fourier coefficients, summed over all rows
        (row = -1) or of one row.  field is [B][ny][nx], or a velocity field
        [B][2][ny][nx] with `component` 0 (u) or 1 (v)."""
        self._sync_stream()
        f = self.as_dev(field)
        N = self.cfg.nx * self.cfg.ny
        if component is None:
            f = f.reshape(self.cfg.batch, self.cfg.ny, self.cfg.nx)
            base, stride = f.data_ptr(), N
        else:
            if component not in (0, 1):
                raise ValueError("component must be 0 (u) or 1 (v)")
            f = f.reshape(self.shape_uv)
            base, stride = f.data_ptr() + 8 * N * int(component), 2 * N
        E = self._f64((self.cfg.batch, self.cfg.nx // 2 + 1))
        _check(load().rt_row_spectrum(self._h, ctypes.c_void_p(base), stride, int(row), _ptr(E)), "rt_row_spectrum")
        return E

    def _field_ptr(self, field, component):
        f = self.as_dev(field)
        N = self.cfg.nx * self.cfg.ny
        if component is None:
            f = f.reshape(self.cfg.batch, self.cfg.ny, self.cfg.nx)
            return f, f.data_ptr(), N
        if component not in (0, 1):
            raise ValueError("component must be 0 (u) or 1 (v)")
        f = f.reshape(self.shape_uv)
        return f, f.data_ptr() + 8 * N * int(component), 2 * N

    def power_spectrum_2d(self, field, component: int | None = None) -> torch.Tensor:
        """E[B][ny][nx/2 + 1] = |F(q, k)|^2, the 2-D power spectrum of a field
        [B][ny][nx] or of one component of a velocity field (App. B)."""
        self._sync_stream()
        f, base, stride = self._field_ptr(field, component)
        E = self._f64((self.cfg.batch, self.cfg.ny, self.cfg.nx // 2 + 1))
        _check(load().rt_power_spectrum_2d(self._h, ctypes.c_void_p(base), stride, _ptr(E)), "rt_power_spectrum_2d")
        return E

    def baseline_ek(self, T: float) -> torch.Tensor:
        """e_k field of the unperturbed run at time T: the reference of Eq. 8."""
        U0 = self.init_state(torch.zeros(self.shape_uv, dtype=torch.float64, device=self.device))
        UT, _, _, _ = self.integrate(U0, T)
        return self.ek_field(UT)

    def ek_anomaly(self, U, ek_base) -> torch.Tensor:
        """J[B] of Eq. 8 for the state U against the baseline field."""
        self._sync_stream()
        U = self.as_dev(U)
        ekb = self.as_dev(ek_base).expand(self.cfg.batch, self.cfg.ny, self.cfg.nx).contiguous()
        J = self._f64((self.cfg.batch,))
        _check(load().rt_ek_anomaly(self._h, _ptr(U), _ptr(ekb), _ptr(J)), "rt_ek_anomaly")
        return J

    def grad_ek_anomaly(self, uv0, T: float, ek_base, policy: Policy | None = None,
                        pool: torch.Tensor | None = None):
        """(J[B], grad[B][2][ny][nx], nsteps[B]) of Eq. 8 on the device."""
        self._sync_stream()
        policy = policy or Policy()
        uv0 = self.as_dev(uv0).reshape(self.shape_uv)
        ekb = self.as_dev(ek_base).expand(self.cfg.batch, self.cfg.ny, self.cfg.nx).contiguous()
        if pool is None:
            return self._with_own_pool(policy, uv0, T, lambda pl, pol: load().rt_grad_ek_anomaly(
                self._h, _ptr(uv0), float(T), ctypes.byref(pol), _ptr(ekb), _ptr(pl[0]), _ptr(pl[1]),
                _ptr(pl[2])), "rt_grad_ek_anomaly")
        pool, pol = self._pool(policy, pool)
        J = self._f64((self.cfg.batch,))
        g = self._f64(self.shape_uv)
        n = torch.empty((self.cfg.batch,), dtype=torch.int32, device=self.device)
        _check(load().rt_grad_ek_anomaly(self._h, _ptr(uv0), float(T), ctypes.byref(pol), _ptr(ekb), _ptr(J),
                                         _ptr(g), _ptr(n)), "rt_grad_ek_anomaly")
        return J, g, n

    def project_to_constraint(self, uv, delta: float, norm: int = NORM_L2, kind: int = SET_SPHERE):
        """In-place on a copy: returns (projected uv, norm before scaling)."""
        self._sync_stream()
        uv = self.as_dev(uv).reshape(self.shape_uv).clone()
        m = self._f64((self.cfg.batch,))
        _check(load().rt_project_to_constraint(self._h, _ptr(uv), float(delta), int(norm), int(kind), _ptr(m)),
               "rt_project_to_constraint")
        return uv, m

    def dot(self, a, b) -> torch.Tensor:
        self._sync_stream()
        a = self.as_dev(a)
        b = self.as_dev(b)
        out = self._f64((self.cfg.batch,))
        _check(load().rt_dot(self._h, _ptr(a), _ptr(b), _ptr(out)), "rt_dot")
        return out

    def max_abs(self, a) -> torch.Tensor:
        self._sync_stream()
        a = self.as_dev(a)
        out = self._f64((self.cfg.batch,))
        _check(load().rt_max_abs(self._h, _ptr(a), _ptr(out)), "rt_max_abs")
        return out

    def axpy(self, x, alpha, y) -> torch.Tensor:
        self._sync_stream()
        x = self.as_dev(x)
        y = self.as_dev(y)
        al = self.as_dev(torch.as_tensor(alpha, dtype=torch.float64).expand(self.cfg.batch).clone())
        out = torch.empty_like(x)
        _check(load().rt_axpy(self._h, _ptr(x), _ptr(al), _ptr(y), _ptr(out)), "rt_axpy")
        return out

    def check_error(self):
        _check(load().rt_check_error(self._h), "rt_check_error")


class KERatio(torch.autograd.Function):
    """R = KE(U(T)) / KE(U(0)) as a differentiable function of the initial
    velocity perturbation.  When a gradient is wanted, forward runs the
    library's rt_grad_u0 (one march with checkpoints, then the discrete
    adjoint) and keeps dR/duv0; backward only scales it by grad_output.
    Otherwise forward marches once (rt_integrate, rt_ke_ratio)."""

    @staticmethod
    def forward(fctx, uv0: torch.Tensor, rt: Context, T: float, policy: Policy | None = None):
        if fctx.needs_input_grad[0]:
            R, g, _ = rt.grad_u0(uv0, T, policy)
            fctx.save_for_backward(g)
            return R
        fctx.save_for_backward(None)
        return rt.objective_ratio(uv0, T)

    @staticmethod
    def backward(fctx, gout):
        (g,) = fctx.saved_tensors
        return g * gout.reshape(-1, 1, 1, 1), None, None, None


__all__ = ["Context", "Policy", "KERatio", "RTError", "load", "revolve_stats", "EXPORTED",
           "CKPT_STORE_ALL", "CKPT_UNIFORM", "CKPT_REVOLVE"]
