"""Oracle (test infrastructure only): numpy wrapper over ``librtoracle.so``.

The oracle is a plain, slow FP64 CPU implementation of the CNOP hot path
(forward Euler-with-gravity march, kinetic-energy ratio, its exact gradient by
reverse-mode AD, and the constraint projection of Eq. 11).  Only the tests,
the smoke check and the CPU-baseline leg of the benchmark use it; the product
path never imports it.  It shares no code with the GPU implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "librtoracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)

ERRORS = {-1: "invalid argument", -3: "capacity too small", -4: "unphysical state"}

# Relative tie tolerance of the scheme's discrete decisions used by the
# workloads (Problem.tie_tol; 0 gives the plain limiter and Riemann-solver
# decisions).
TIE_TOL = 1e-10


class Problem(ctypes.Structure):
    """Mirror of the oracle's ``rto::Problem`` (plain numbers only)."""

    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nb", ctypes.c_int32),
        ("comp_mask", ctypes.c_int32),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double),
        ("gamma", ctypes.c_double), ("g_y", ctypes.c_double),
        ("rho_h", ctypes.c_double), ("rho_l", ctypes.c_double),
        ("y0", ctypes.c_double), ("h", ctypes.c_double),
        ("p_int", ctypes.c_double), ("cfl", ctypes.c_double),
        ("recon", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("tie_tol", ctypes.c_double),
    ]


class OracleError(RuntimeError):
    pass


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise OracleError(f"{_LIB_PATH} is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(Problem)
        sig = {
            "rto_init_state": [P, _dp, _dp],
            "rto_cfl_dt": [P, _dp, _dp],
            "rto_step": [P, _dp, _dp, _dp],
            "rto_integrate": [P, _dp, ctypes.c_double, _dp, _ip, _dp, ctypes.c_int32],
            "rto_kinetic_energy": [P, _dp, _dp],
            "rto_step_jvp": [P, _dp, _dp, _dp, _dp, _dp],
            "rto_step_vjp": [P, _dp, _dp, _dp, _dp],
            "rto_grad_u0": [P, _dp, ctypes.c_double, _dp, _dp, _ip, _dp, ctypes.c_int32],
            "rto_ke_ratio_frozen": [P, _dp, _dp, _ip, ctypes.c_int32, _dp],
            "rto_project_to_constraint": [P, _dp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, _dp],
            "rto_ek_field": [P, _dp, _dp],
            "rto_mix_width": [P, _dp, _dp],
            "rto_row_spectrum": [P, _dp, ctypes.c_int64, ctypes.c_int32, _dp],
            "rto_power_spectrum_2d": [P, _dp, ctypes.c_int64, _dp],
            "rto_ek_anomaly_frozen": [P, _dp, _dp, _ip, ctypes.c_int32, _dp, _dp],
            "rto_grad_ek_anomaly": [P, _dp, ctypes.c_double, _dp, _dp, _dp, _ip, _dp, ctypes.c_int32],
            "rto_objective_adaptive": [P, _dp, ctypes.c_double, _dp, _dp, _ip],
            "rto_grad_adaptive": [P, _dp, ctypes.c_double, _dp, _dp, _dp, _ip],
            "rto_hllc": [ctypes.c_double, _dp, _dp, _dp],
            "rto_mc_slope": [ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp],
            "rto_slopes": [P, _dp, _dp, _dp, ctypes.c_int32, _dp],
            "rto_predict": [P, _dp, _dp, _dp, ctypes.c_double, _dp],
            "rto_set_threads": [ctypes.c_int32],
            "rto_count_flops": [P, _dp, ctypes.c_double, _dp],
            "rto_background": [P, _dp, _dp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.rto_wall_pressure.argtypes = [ctypes.c_double, _dp, ctypes.c_int32]
        L.rto_wall_pressure.restype = ctypes.c_double
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _ipt(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_ip)


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what}: {ERRORS.get(rc, rc)}")


@dataclass
class Oracle:
    """Bound problem description; arrays are numpy float64, members stacked."""

    prob: Problem

    @classmethod
    def from_config(cls, cfg, nb: int | None = None, tie_tol: float | None = None):
        """The oracle for an RTConfig; tie_tol None takes the workloads'
        tolerance TIE_TOL, 0 the plain decisions (see rto_scheme.hpp)."""
        p = Problem(
            nx=cfg.nx, ny=cfg.ny, nb=cfg.batch if nb is None else nb, comp_mask=cfg.comp_mask,
            lx=cfg.lx, ly=cfg.ly, gamma=cfg.gamma, g_y=cfg.g_y, rho_h=cfg.rho_h, rho_l=cfg.rho_l,
            y0=cfg.y0, h=cfg.h, p_int=cfg.p_int, cfl=cfg.cfl, recon=getattr(cfg, "recon", 0),
            tie_tol=TIE_TOL if tie_tol is None else float(tie_tol),
        )
        return cls(p)

    @property
    def shape_u(self):
        return (self.prob.nb, 4, self.prob.ny, self.prob.nx)

    @property
    def shape_uv(self):
        return (self.prob.nb, 2, self.prob.ny, self.prob.nx)

    def init_state(self, uv0):
        uv0 = np.ascontiguousarray(uv0, dtype=np.float64).reshape(self.shape_uv)
        U = np.empty(self.shape_u)
        _check(lib().rto_init_state(ctypes.byref(self.prob), _p(uv0), _p(U)), "init_state")
        return U

    def cfl_dt(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        dt = np.empty(self.prob.nb)
        _check(lib().rto_cfl_dt(ctypes.byref(self.prob), _p(U), _p(dt)), "cfl_dt")
        return dt

    def step(self, U, dt):
        U = np.ascontiguousarray(U, dtype=np.float64)
        dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (self.prob.nb,)))
        Un = np.empty_like(U)
        _check(lib().rto_step(ctypes.byref(self.prob), _p(U), _p(Un), _p(dt)), "step")
        return Un

    def integrate(self, U, T, cap: int = 0):
        U = np.array(U, dtype=np.float64, copy=True, order="C")
        t = np.empty(self.prob.nb)
        n = np.empty(self.prob.nb, dtype=np.int32)
        log = np.zeros((self.prob.nb, max(cap, 1)))
        rc = lib().rto_integrate(ctypes.byref(self.prob), _p(U), float(T), _p(t), _ipt(n),
                                 _p(log) if cap > 0 else None, int(cap))
        _check(rc, "integrate")
        return U, t, n, (log[:, :] if cap > 0 else None)

    def kinetic_energy(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        ke = np.empty(self.prob.nb)
        _check(lib().rto_kinetic_energy(ctypes.byref(self.prob), _p(U), _p(ke)), "kinetic_energy")
        return ke

    def step_jvp(self, U, dU, dt):
        U = np.ascontiguousarray(U, dtype=np.float64)
        dU = np.ascontiguousarray(dU, dtype=np.float64)
        dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (self.prob.nb,)))
        Un, dUn = np.empty_like(U), np.empty_like(U)
        _check(lib().rto_step_jvp(ctypes.byref(self.prob), _p(U), _p(dU), _p(dt), _p(Un), _p(dUn)), "step_jvp")
        return Un, dUn

    def step_vjp(self, U, dt, lam_next):
        U = np.ascontiguousarray(U, dtype=np.float64)
        lam_next = np.ascontiguousarray(lam_next, dtype=np.float64)
        dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (self.prob.nb,)))
        lam = np.empty_like(U)
        _check(lib().rto_step_vjp(ctypes.byref(self.prob), _p(U), _p(dt), _p(lam_next), _p(lam)), "step_vjp")
        return lam

    def grad_u0(self, uv0, T, cap: int = 0):
        """(R, grad, nsteps, dt_log): KE ratio and its exact frozen-schedule gradient."""
        uv0 = np.ascontiguousarray(uv0, dtype=np.float64).reshape(self.shape_uv)
        R = np.empty(self.prob.nb)
        g = np.empty(self.shape_uv)
        n = np.empty(self.prob.nb, dtype=np.int32)
        log = np.zeros((self.prob.nb, max(cap, 1)))
        rc = lib().rto_grad_u0(ctypes.byref(self.prob), _p(uv0), float(T), _p(R), _p(g), _ipt(n),
                               _p(log) if cap > 0 else None, int(cap))
        _check(rc, "grad_u0")
        return R, g, n, (log if cap > 0 else None)

    def ke_ratio_frozen(self, uv0, dt_log, nsteps):
        uv0 = np.ascontiguousarray(uv0, dtype=np.float64).reshape(self.shape_uv)
        dt_log = np.ascontiguousarray(dt_log, dtype=np.float64)
        nsteps = np.ascontiguousarray(nsteps, dtype=np.int32)
        R = np.empty(self.prob.nb)
        rc = lib().rto_ke_ratio_frozen(ctypes.byref(self.prob), _p(uv0), _p(dt_log), _ipt(nsteps),
                                       int(dt_log.shape[1]), _p(R))
        _check(rc, "ke_ratio_frozen")
        return R

    def mix_width(self, U):
        """Mixing-layer width of Eqs. 13-14 for each member."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        h = np.empty(self.prob.nb)
        _check(lib().rto_mix_width(ctypes.byref(self.prob), _p(U), _p(h)), "mix_width")
        return h

    def row_spectrum(self, f, row: int = -1):
        """E[B][nx/2 + 1]: sum over the selected rows of |DFT_n of the row|^2
        for each member's field f [B][ny][nx] (Eq. 12 before normalisation)."""
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.prob.nb, self.prob.ny, self.prob.nx)
        E = np.empty((self.prob.nb, self.prob.nx // 2 + 1))
        _check(lib().rto_row_spectrum(ctypes.byref(self.prob), _p(f), self.prob.nx * self.prob.ny, int(row), _p(E)),
               "row_spectrum")
        return E

    def power_spectrum_2d(self, f):
        """E[B][ny][nx/2 + 1] = |2-D DFT of each member's field f [B][ny][nx]|^2
        (App. B's reconstruction keeps its strongest modes)."""
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.prob.nb, self.prob.ny, self.prob.nx)
        E = np.empty((self.prob.nb, self.prob.ny, self.prob.nx // 2 + 1))
        _check(lib().rto_power_spectrum_2d(ctypes.byref(self.prob), _p(f), self.prob.nx * self.prob.ny, _p(E)),
               "power_spectrum_2d")
        return E

    def ek_field(self, U):
        """Kinetic-energy density e_k = |m|^2/(2 rho) of every cell, [nb][ny][nx] (Eq. 7)."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        ek = np.empty((self.prob.nb, self.prob.ny, self.prob.nx))
        _check(lib().rto_ek_field(ctypes.byref(self.prob), _p(U), _p(ek)), "ek_field")
        return ek

    def _ekb(self, ek_base):
        return np.ascontiguousarray(np.broadcast_to(np.asarray(ek_base, dtype=np.float64),
                                                    (self.prob.nb, self.prob.ny, self.prob.nx)))

    def grad_ek_anomaly(self, uv0, T, ek_base, cap: int = 0):
        """(J, grad, nsteps, dt_log): objective of Eq. 8 against the baseline
        field ek_base and its exact frozen-schedule gradient."""
        uv0 = np.ascontiguousarray(uv0, dtype=np.float64).reshape(self.shape_uv)
        ekb = self._ekb(ek_base)
        J = np.empty(self.prob.nb)
        g = np.empty(self.shape_uv)
        n = np.empty(self.prob.nb, dtype=np.int32)
        log = np.zeros((self.prob.nb, max(cap, 1)))
        rc = lib().rto_grad_ek_anomaly(ctypes.byref(self.prob), _p(uv0), float(T), _p(ekb), _p(J), _p(g), _ipt(n),
                                       _p(log) if cap > 0 else None, int(cap))
        _check(rc, "grad_ek_anomaly")
        return J, g, n, (log if cap > 0 else None)

    def ek_anomaly_frozen(self, uv0, dt_log, nsteps, ek_base):
        uv0 = np.ascontiguousarray(uv0, dtype=np.float64).reshape(self.shape_uv)
        dt_log = np.ascontiguousarray(dt_log, dtype=np.float64)
        nsteps = np.ascontiguousarray(nsteps, dtype=np.int32)
        ekb = self._ekb(ek_base)
        J = np.empty(self.prob.nb)
        rc = lib().rto_ek_anomaly_frozen(ctypes.byref(self.prob), _p(uv0), _p(dt_log), _ipt(nsteps),
                                         int(dt_log.shape[1]), _p(ekb), _p(J))
        _check(rc, "ek_anomaly_frozen")
        return J

    def objective_adaptive(self, uv0, T, ek_base=None):
        """(value, nsteps): R = KE(T)/KE(0), or J of Eq. 8 when ek_base is
        given, after the adaptive march (every step from the CFL rule)."""
        uv0 = np.ascontiguousarray(uv0, dtype=np.float64).reshape(self.shape_uv)
        ekb = None if ek_base is None else self._ekb(ek_base)
        v = np.empty(self.prob.nb)
        n = np.empty(self.prob.nb, dtype=np.int32)
        rc = lib().rto_objective_adaptive(ctypes.byref(self.prob), _p(uv0), float(T),
                                          None if ekb is None else _p(ekb), _p(v), _ipt(n))
        _check(rc, "objective_adaptive")
        return v, n

    def grad_adaptive(self, uv0, T, ek_base=None):
        """(value, grad, nsteps): R (or J) and its gradient through the
        adaptive march, the state dependence of the CFL steps and of the
        clipped last step included."""
        uv0 = np.ascontiguousarray(uv0, dtype=np.float64).reshape(self.shape_uv)
        ekb = None if ek_base is None else self._ekb(ek_base)
        v = np.empty(self.prob.nb)
        g = np.empty(self.shape_uv)
        n = np.empty(self.prob.nb, dtype=np.int32)
        rc = lib().rto_grad_adaptive(ctypes.byref(self.prob), _p(uv0), float(T),
                                     None if ekb is None else _p(ekb), _p(v), _p(g), _ipt(n))
        _check(rc, "grad_adaptive")
        return v, g, n

    def baseline_ek(self, T):
        """e_k of the unperturbed run at time T (the reference field of Eq. 8)."""
        U0 = self.init_state(np.zeros(self.shape_uv))
        UT, _, _, _ = self.integrate(U0, T)
        return self.ek_field(UT)

    def project_to_constraint(self, uv, delta, norm: int = 0, kind: int = 0):
        uv = np.array(uv, dtype=np.float64, copy=True, order="C").reshape(self.shape_uv)
        m = np.empty(self.prob.nb)
        rc = lib().rto_project_to_constraint(ctypes.byref(self.prob), _p(uv), float(delta), int(norm),
                                             int(kind), _p(m))
        _check(rc, "project_to_constraint")
        return uv, m

    def background(self):
        r = np.empty(self.prob.ny)
        p = np.empty(self.prob.ny)
        _check(lib().rto_background(ctypes.byref(self.prob), _p(r), _p(p)), "background")
        return r, p


def hllc(gamma, left, right):
    """HLLC flux, face-normal order, for states (rho, normal vel., tangential vel., p)."""
    L = np.ascontiguousarray(left, dtype=np.float64)
    R = np.ascontiguousarray(right, dtype=np.float64)
    f = np.empty(4)
    lib().rto_hllc(float(gamma), _p(L), _p(R), _p(f))
    return f


def wall_pressure(gamma, state, interior_left: bool):
    s = np.ascontiguousarray(state, dtype=np.float64)
    return lib().rto_wall_pressure(float(gamma), _p(s), 1 if interior_left else 0)


def mc_slope(a, b, tol=0.0):
    """(slope, d slope/d a, d slope/d b) of the monotonized-central limiter
    for the differences a, b; |d| <= tol counts as zero."""
    out = np.empty(3)
    _check(lib().rto_mc_slope(float(a), float(b), float(tol), _p(out)), "mc_slope")
    return out[0], out[1], out[2]


def _w4(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(4))


def slopes(o: "Oracle", wm, w, wp, balanced: bool = False):
    """Limited slopes (rho, u, v, p) of the cell w between wm and wp."""
    s = np.empty(4)
    _check(lib().rto_slopes(ctypes.byref(o.prob), _p(_w4(wm)), _p(_w4(w)), _p(_w4(wp)), 1 if balanced else 0,
                            _p(s)), "slopes")
    return s


def predict(o: "Oracle", w, sx, sy, dt):
    """MUSCL-Hancock half step W^{n+1/2} of one cell (primitives, slopes per cell width)."""
    q = np.empty(4)
    _check(lib().rto_predict(ctypes.byref(o.prob), _p(_w4(w)), _p(_w4(sx)), _p(_w4(sy)), float(dt), _p(q)), "predict")
    return q


def set_threads(n: int) -> int:
    """Threads over the rows of the oracle's forward step (timing only;
    results do not depend on it).  Returns the count in force."""
    return int(lib().rto_set_threads(int(n)))


def count_flops(o: "Oracle", U, dt):
    """Algorithmic work of one step of member 0 of U at step dt, per cell:
    {"step": flops of the step, "cfl": flops of the signal speed of the new
    state, "edges": edges of the step's computational graph, "add", "mul",
    "div", "sqrt": the step's operations by kind} (see rto_count.hpp)."""
    U = np.ascontiguousarray(np.asarray(U, dtype=np.float64)[:1])
    out = np.empty(7)
    _check(lib().rto_count_flops(ctypes.byref(o.prob), _p(U), float(np.asarray(dt).ravel()[0]), _p(out)), "count_flops")
    n = o.prob.nx * o.prob.ny
    return {"step": out[0] / n, "cfl": out[1] / n, "edges": out[2] / n, "add": out[3] / n, "mul": out[4] / n,
            "div": out[5] / n, "sqrt": out[6] / n}
