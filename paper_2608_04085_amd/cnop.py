"""CNOP search: spectral projected-gradient ascent on the constraint sphere.

The paper maximises its objective over the perturbations that satisfy the
energy constraint (Sec. 3.1, Eq. 10) with a projected quasi-Newton method, a
projection that rescales a trial point onto the constraint (Eq. 11) and a
non-monotone Armijo line search that allows temporary decreases (Sec. 3.4).
This driver does the same with the spectral (Barzilai-Borwein) projected
gradient method:

    u+ = P(u_k + lam * alpha_k * g_k)              trial point on the sphere
    accept if R(u+) >= min(R of the last M accepted iterates)
                       + c * <g_k, u+ - u_k>       (non-monotone, ascent form)
    else lam <- lam / 2
    alpha_{k+1} = <s, s> / |<s, y>|,  s = u+ - u_k, y = g+ - g_k

and logs the stationarity measure chi_k = ||P(u_k + g_k) - u_k||_inf of
Appendix A (written for ascent).  Every member of the batch is an independent
restart; all members advance in the same launches.  The host only decides
acceptance and step sizes from per-member scalars; every field operation is
a library call (projection, axpy, dot products, forward march, gradient).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import optim
from .config import NORM_L2, NORM_RHO_KE, SET_BALL, SET_SPHERE
from .rtcnop import Context, Policy


@dataclass
class SPGLog:
    R: list = field(default_factory=list)          # [iter][B] accepted objective
    grad_norm: list = field(default_factory=list)  # [iter][B] ||g|| (L2 dV)
    chi: list = field(default_factory=list)        # [iter][B] stationarity measure
    backtracks: list = field(default_factory=list) # [iter][B]
    evals: int = 0                                 # forward evaluations
    grads: int = 0                                 # gradient evaluations


def _l2dv(rt: Context, x: torch.Tensor) -> np.ndarray:
    return np.sqrt(rt.dot(x, x).cpu().numpy() * rt.cfg.dx * rt.cfg.dy)


def ke_ratio(rt: Context, uv: torch.Tensor, T: float) -> torch.Tensor:
    """R = KE(T)/KE(0) of every member (forward march only)."""
    return rt.objective_ratio(uv, T)


class SPG:
    """The spectral projected-gradient search as an object that advances one
    iteration per step() (all members at once).  Each trial point is
    evaluated with its gradient (grad_at_trials, the default: an accepted
    trial needs no second march) or with a forward march and the gradient
    afterwards at the accepted point; both give the same iterates.

    cell_updates counts 2 B nx ny N_t per gradient call (one forward and one
    adjoint sweep over every member's N_t steps), the algorithmic work of
    the calls so far."""

    def __init__(self, rt: Context, uv0, T: float, delta: float, policy: Policy | None = None,
                 pool: torch.Tensor | None = None, memory: int = 10, c_armijo: float = 1e-4,
                 max_backtracks: int = 8, log: SPGLog | None = None, grad_at_trials: bool = True):
        self.rt, self.T, self.delta, self.policy, self.pool = rt, T, delta, policy, pool
        self.memory, self.c_armijo, self.max_backtracks = memory, c_armijo, max_backtracks
        self.grad_at_trials = grad_at_trials
        self.log = log or SPGLog()
        self.cell_updates = 0
        self.u, _ = rt.project_to_constraint(rt.as_dev(uv0), delta, NORM_L2, SET_SPHERE)
        R, self.g, _ = self._grad(self.u)
        self.R = R.cpu().numpy().copy()
        self.hist = [self.R.copy()]
        gn = _l2dv(rt, self.g)
        self.alpha = 0.1 * delta / np.maximum(gn, 1e-300)

    def _grad(self, u):
        R, g, n = self.rt.grad_u0(u, self.T, self.policy, pool=self.pool)
        self.log.grads += 1
        self.last_nsteps = n.cpu().numpy().tolist()
        self.cell_updates += 2 * int(sum(self.last_nsteps)) * self.rt.cfg.nx * self.rt.cfg.ny
        return R, g, n

    def step(self) -> np.ndarray:
        """One iteration; returns the accepted objective of every member."""
        rt, log, B = self.rt, self.log, self.rt.cfg.batch
        u, g, alpha, delta, T = self.u, self.g, self.alpha, self.delta, self.T
        lam = np.ones(B)
        accepted = np.zeros(B, dtype=bool)
        u_new = torch.empty_like(u)
        g2 = torch.empty_like(g)
        R_new = np.zeros(B)
        ref = np.min(np.stack(self.hist[-self.memory:]), axis=0)
        nback = np.zeros(B, dtype=int)
        for bt in range(self.max_backtracks + 1):
            trial = rt.axpy(u, lam * alpha, g)
            trial, _ = rt.project_to_constraint(trial, delta, NORM_L2, SET_SPHERE)
            if self.grad_at_trials:
                Rt_dev, gt, _ = self._grad(trial)
            else:
                Rt_dev = ke_ratio(rt, trial, T)
                log.evals += 1
            Rt = Rt_dev.cpu().numpy()
            d = rt.axpy(trial, -1.0, u)
            gd = rt.dot(g, d).cpu().numpy()
            ok = (Rt >= ref + self.c_armijo * gd) | (bt == self.max_backtracks)
            for b in range(B):
                if not accepted[b] and ok[b]:
                    accepted[b] = True
                    u_new[b] = trial[b]
                    R_new[b] = Rt[b]
                    if self.grad_at_trials:
                        g2[b] = gt[b]
            if accepted.all():
                break
            nback += ~accepted
            lam = np.where(accepted, lam, 0.5 * lam)
        if self.grad_at_trials:
            Rh = R_new.copy()
        else:
            R2, g2, _ = self._grad(u_new)
            Rh = R2.cpu().numpy().copy()
        s = rt.axpy(u_new, -1.0, u)
        y = rt.axpy(g2, -1.0, g)
        ss = rt.dot(s, s).cpu().numpy()
        sy = rt.dot(s, y).cpu().numpy()
        gn = _l2dv(rt, g2)
        base = delta / np.maximum(gn, 1e-300)
        self.alpha = np.clip(ss / np.maximum(np.abs(sy), 1e-300), 1e-10 * base, 1e10 * base)
        # stationarity measure chi = ||P(u + g) - u||_inf
        pg, _ = rt.project_to_constraint(rt.axpy(u_new, 1.0, g2), delta, NORM_L2, SET_SPHERE)
        chi = rt.max_abs(rt.axpy(pg, -1.0, u_new)).cpu().numpy()
        self.u, self.g, self.R = u_new, g2, Rh
        self.hist.append(Rh)
        log.R.append(Rh.tolist())
        log.grad_norm.append(gn.tolist())
        log.chi.append(chi.tolist())
        log.backtracks.append(nback.tolist())
        return Rh


class GroupedSPG:
    """The SPG search of B independent restarts run as `groups` searches of
    about B / groups members, each on its own context, stream and share of
    the checkpoint budget and driven by its own host thread.  The restarts
    never interact (every decision of the search is per member), so each
    takes the same iterates, bit for bit, as in one search of all B; the
    groups' marches and reverse sweeps overlap on the GPU instead of running
    one after the other.  `pool_bytes` is the whole budget; each group's
    pool holds the same number of its own states as one pool of
    `pool_bytes` holds of all B."""

    def __init__(self, cfg, uv0, T: float, delta: float, groups: int = 2, pool_bytes: int | None = None,
                 max_steps: int = 65536, policy: Policy | None = None, **kw):
        B = cfg.batch
        groups = max(1, min(groups, B))
        uv0 = np.asarray(uv0.cpu() if isinstance(uv0, torch.Tensor) else uv0)
        self.bounds = [(k * B // groups, (k + 1) * B // groups) for k in range(groups)]
        self.streams = [torch.cuda.Stream() for _ in range(groups)]
        self.searches: list[SPG] = []
        for (b0, b1), st in zip(self.bounds, self.streams):
            with torch.cuda.stream(st):
                gcfg = cfg.with_(batch=b1 - b0)
                rt = Context(gcfg, max_steps=max_steps)
                pool = None
                if pool_bytes is not None:
                    state = 8 * 4 * gcfg.nx * gcfg.ny
                    slots = int(pool_bytes) // (state * B)
                    pool = torch.empty(slots * state * (b1 - b0) + 256, dtype=torch.uint8, device=rt.device)
                self.searches.append(SPG(rt, uv0[b0:b1], T, delta, policy, pool, **kw))
        torch.cuda.synchronize()

    def step(self, n: int = 1, on_iter=None) -> np.ndarray:
        """n iterations of every group (the groups advance independently);
        on_iter(group, k), if given, is called from the group's thread after
        its iteration k.  Returns the accepted objectives of all members."""
        import threading
        errors = []

        def run(k):
            try:
                # a new thread starts on device 0: take the group's device first
                torch.cuda.set_device(self.searches[k].rt.device)
                with torch.cuda.stream(self.streams[k]):
                    for it in range(n):
                        self.searches[k].step()
                        if on_iter is not None:
                            on_iter(k, it)
                self.streams[k].synchronize()
            except BaseException as e:  # noqa: BLE001 -- re-raised below
                errors.append(e)

        threads = [threading.Thread(target=run, args=(k,)) for k in range(len(self.searches))]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        if errors:
            raise errors[0]
        return self.R

    @property
    def R(self) -> np.ndarray:
        return np.concatenate([s.R for s in self.searches])

    @property
    def u(self) -> torch.Tensor:
        return torch.cat([s.u for s in self.searches])

    @property
    def cell_updates(self) -> int:
        return sum(s.cell_updates for s in self.searches)

    @property
    def grads(self) -> list[int]:
        return [s.log.grads for s in self.searches]

    @property
    def last_nsteps(self) -> list[int]:
        return [n for s in self.searches for n in s.last_nsteps]

    @property
    def hist(self) -> np.ndarray:
        return np.concatenate([np.array(s.hist) for s in self.searches], axis=1)

    @property
    def backtracks(self) -> list[list[int]]:
        """Per iteration, the backtracks of every member."""
        rows = [s.log.backtracks for s in self.searches]
        return [sum((r[i] for r in rows), []) for i in range(min(len(r) for r in rows))]


def spg(rt: Context, uv0, T: float, delta: float, iters: int, policy: Policy | None = None,
        pool: torch.Tensor | None = None, memory: int = 10, c_armijo: float = 1e-4, max_backtracks: int = 8,
        log: SPGLog | None = None, on_iter=None, grad_at_trials: bool = True):
    """Run `iters` SPG iterations from uv0 (projected onto ||u|| = delta).
    on_iter(k, R, log), if given, is called after iteration k.
    grad_at_trials: see SPG.  Returns (u, R, g, log)."""
    search = SPG(rt, uv0, T, delta, policy, pool, memory, c_armijo, max_backtracks, log, grad_at_trials)
    for it in range(iters):
        Rh = search.step()
        if on_iter is not None:
            on_iter(it, Rh, search.log)
    return search.u, torch.as_tensor(search.R), search.g, search.log


class LibraryBackend:
    """Field operations of the projected L-BFGS search on the HIP library,
    for the paper's problem (Sec. 3.1): maximise J of Eq. 8 against the
    baseline field ek_base at time T over the ball C <= eps of Eq. 9, with
    the projection of Eq. 11."""

    def __init__(self, rt: Context, T: float, ek_base, eps: float, policy: Policy | None = None,
                 pool: torch.Tensor | None = None):
        self.rt, self.T, self.eps, self.policy, self.pool = rt, float(T), float(eps), policy, pool
        self.ek_base = rt.as_dev(ek_base).expand(rt.cfg.batch, rt.cfg.ny, rt.cfg.nx).contiguous()

    def dot(self, a, b):
        return self.rt.dot(a, b).cpu().numpy()

    def axpy(self, x, alpha, y):
        return self.rt.axpy(x, alpha, y)

    def project(self, x):
        return self.rt.project_to_constraint(x, self.eps, NORM_RHO_KE, SET_BALL)[0]

    def max_abs(self, x):
        return self.rt.max_abs(x).cpu().numpy()

    def where(self, mask, a, b):
        m = torch.as_tensor(np.asarray(mask), device=a.device).view(-1, 1, 1, 1)
        return torch.where(m, a, b)

    def value(self, x):
        U0 = self.rt.init_state(x)
        UT, _, _, _ = self.rt.integrate(U0, self.T)
        return self.rt.ek_anomaly(UT, self.ek_base).cpu().numpy()

    def value_and_grad(self, x):
        J, g, _ = self.rt.grad_ek_anomaly(x, self.T, self.ek_base, self.policy, pool=self.pool)
        return J.cpu().numpy(), g


def paper_cnop(rt: Context, uv0, T: float, eps: float, iters: int, policy: Policy | None = None,
               pool: torch.Tensor | None = None, memory: int = 10, on_iter=None):
    """The paper's search (Sec. 3): maximise J of Eq. 8 over C <= eps with
    projected L-BFGS (m = memory) and a non-monotone Armijo line search, from
    initial guesses uv0 scaled to C = eps.  Every member is an independent
    restart.  Returns (u, J, g, log, ek_base)."""
    ek_base = rt.baseline_ek(T)
    u0, _ = rt.project_to_constraint(rt.as_dev(uv0), eps, NORM_RHO_KE, SET_SPHERE)
    be = LibraryBackend(rt, T, ek_base, eps, policy, pool)
    u, J, g, log = optim.lbfgs_max(be, u0, iters, memory=memory, on_iter=on_iter)
    return u, J, g, log, ek_base


def spectrum_top5(v_row: np.ndarray) -> float:
    """Energy fraction of the 5 strongest horizontal modes n >= 1 of one row
    (Sec. 4.2, Eq. 12: E_n = |u_n|^2 / sum over the positive modes)."""
    c = np.fft.rfft(v_row)
    e = np.abs(c[1:]) ** 2
    e = e / np.sum(e)
    return float(np.sum(np.sort(e)[-5:]))


def top5_fraction(E_row) -> float:
    """The same fraction from a spectrum E[0 .. nx/2] as the library's
    rt_row_spectrum returns it (Eq. 12: normalised over n >= 1)."""
    e = np.asarray(E_row, dtype=np.float64)[1:]
    e = e / np.sum(e)
    return float(np.sum(np.sort(e)[-5:]))


def peak_row(v: np.ndarray) -> int:
    """Row whose rms along x is largest (lowest index on ties)."""
    return int(np.argmax(np.sqrt(np.mean(v * v, axis=1))))


# ---------------------------------------------------------------------------
# Forward comparison suite (Sec. 3.3 run design, Sec. 4.3-4.4 diagnostics)

def dominant_modes(v: np.ndarray, k: int = 5, E_row=None) -> np.ndarray:
    """Horizontal mode numbers n >= 1 of the k largest E_n (Eq. 12) at the
    peak row of v ([ny][nx]); E_row, if given, is that row's spectrum from
    the library's rt_row_spectrum (else numpy's rfft of the row)."""
    if E_row is None:
        e = np.abs(np.fft.rfft(v[peak_row(v)])[1:]) ** 2
    else:
        e = np.asarray(E_row, dtype=np.float64)[1:]
    return 1 + np.argsort(-e, kind="stable")[:k]


def five_mode_seed(v: np.ndarray, k: int = 5, E_row=None) -> np.ndarray:
    """The 5modes perturbation: every row of v keeps only the k dominant
    horizontal modes of the peak row, with their amplitudes and phases
    (rfft bins n and, implicitly, -n); the rest of each row is dropped."""
    modes = dominant_modes(v, k, E_row)
    c = np.fft.rfft(v, axis=1)
    keep = np.zeros(c.shape[1], dtype=bool)
    keep[modes] = True
    return np.fft.irfft(np.where(keep[None, :], c, 0.0), n=v.shape[1], axis=1)


def full_plane(E_half: np.ndarray, nx: int) -> np.ndarray:
    """The [ny][nx] power spectrum of a real field from its half plane
    [ny][nx/2 + 1] (E(q, k) = E(-q mod ny, nx - k))."""
    ny = E_half.shape[0]
    out = np.empty((ny, nx))
    nk = nx // 2 + 1
    out[:, :nk] = E_half
    k = np.arange(nk, nx)
    out[:, nk:] = E_half[(-np.arange(ny)) % ny][:, nx - k]
    return out


def power_reconstruction(v: np.ndarray, frac: float = 0.9, E2=None) -> np.ndarray:
    """The 2-D reconstruction of App. B: the fewest 2-D Fourier modes of v
    that hold `frac` of its spectral energy (strongest first), inverse
    transformed.  E2, if given, is the library's rt_power_spectrum_2d of v
    (half plane), which then ranks the modes."""
    F = np.fft.fft2(v)
    e = np.abs(F) ** 2 if E2 is None else full_plane(np.asarray(E2, dtype=np.float64), v.shape[1])
    order = np.argsort(-e, axis=None, kind="stable")
    csum = np.cumsum(e.ravel()[order])
    m = int(np.searchsorted(csum, frac * csum[-1]) + 1)
    mask = np.zeros(e.size, dtype=bool)
    mask[order[:m]] = True
    return np.real(np.fft.ifft2(np.where(mask.reshape(e.shape), F, 0.0)))


def library_spectra(rt: Context, v: np.ndarray):
    """(E of the peak row, the 2-D power spectrum) of the field v [ny][nx]
    from the library (rt_row_spectrum, rt_power_spectrum_2d), on a
    one-member context of rt's grid."""
    r1 = Context(rt.cfg.with_(batch=1), max_steps=8, device=rt.device)
    f = torch.as_tensor(np.ascontiguousarray(v)[None], dtype=torch.float64, device=rt.device)
    E_row = r1.row_spectrum(f, row=peak_row(v))[0].cpu().numpy()
    E2 = r1.power_spectrum_2d(f)[0].cpu().numpy()
    return E_row, E2


COMPARISON_KINDS = ("CNOP", "Random", "5modes", "2D90")


def comparison_seeds(cfg, v_cnop: np.ndarray, random_seed: int = 1000, rt: Context | None = None) -> np.ndarray:
    """[4][2][ny][nx] u_y-only perturbations of the comparison suite, unscaled:
    the CNOP itself, a localised Gaussian field (the optimiser's initial-guess
    construction), its 5-mode reduction and its 90%-power 2-D
    reconstruction.  With rt, the mode energies that pick the 5 modes and
    the 90 % of the power come from the library's spectra."""
    from . import inputs

    E_row, E2 = library_spectra(rt, v_cnop) if rt is not None else (None, None)
    rnd = inputs.paper_seed_batch(cfg.with_(batch=1), [random_seed])[0, 1]
    out = np.zeros((4, 2, cfg.ny, cfg.nx))
    for k, v in enumerate((v_cnop, rnd, five_mode_seed(v_cnop, E_row=E_row), power_reconstruction(v_cnop, E2=E2))):
        out[k, 1] = v
    return out


def comparison_runs(rt: Context, seeds, eps: float, T: float, n_snap: int) -> dict:
    """March every member (one batched launch per step) from its seed scaled
    to C = eps (Eq. 9) to T, with n_snap uniformly spaced diagnostics:
    total kinetic energy and mixing-layer width (Eqs. 13-14).  Each interval
    ends exactly on its snapshot time (its last CFL step clipped)."""
    u, _ = rt.project_to_constraint(rt.as_dev(seeds), eps, NORM_RHO_KE, SET_SPHERE)
    U = rt.init_state(u)
    t = [0.0]
    ke = [rt.kinetic_energy(U).cpu().numpy().tolist()]
    hm = [rt.mix_width(U).cpu().numpy().tolist()]
    steps = np.zeros(rt.cfg.batch, dtype=np.int64)
    for k in range(1, n_snap + 1):
        U, _, n, _ = rt.integrate(U, T / n_snap)
        steps += n.cpu().numpy()
        t.append(k * T / n_snap)
        ke.append(rt.kinetic_energy(U).cpu().numpy().tolist())
        hm.append(rt.mix_width(U).cpu().numpy().tolist())
    return {"t": t, "ke": ke, "h_mix": hm, "steps": steps.tolist()}
