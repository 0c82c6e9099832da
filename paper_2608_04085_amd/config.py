"""Problem description of the 2-D compressible Rayleigh-Taylor CNOP hot path.

Plain numbers only.  Defaults are the workload the benchmarks use: an ideal
gas with gamma = 1.4 on [0, 0.5] x [0, 1], heavy fluid (rho = 2) above a tanh
interface of width 0.01 at y = 0.5 and light fluid (rho = 1) below, gravity
-0.1 along y, pressure 2.5 at the interface, CFL number 0.4.  The paper's own
setup (Sec. 2.1-2.2 and the fixed-parameter table of Sec. 3.5: gamma = 5/3,
g = 1, unit square, smoothing length 0.02, p(L) = rho_h g L) is available as
the ``paper`` preset.
"""
from __future__ import annotations

import math
from dataclasses import asdict, dataclass, replace

# Perturbed velocity components (bit mask).
COMP_U = 1
COMP_V = 2
COMP_UV = 3

# Norms and sets of the constraint projection (Eq. 11 generalised).
NORM_L2 = 0      # (sum (u^2+v^2) dx dy)^(1/2)
NORM_RMS = 1     # (mean over cells of u^2+v^2)^(1/2)
NORM_RHO_KE = 2  # C = sum rho0 (u^2+v^2)/2 dx dy   (Eq. 9)
SET_SPHERE = 0
SET_BALL = 1

# Reconstructions.
RECON_PRIMITIVE = 0
RECON_BALANCED = 1

# Checkpoint policies of the gradient.
CKPT_STORE_ALL = 0
CKPT_UNIFORM = 1
CKPT_REVOLVE = 2


@dataclass(frozen=True)
class RTConfig:
    nx: int = 64
    ny: int = 128
    batch: int = 1
    lx: float = 0.5
    ly: float = 1.0
    gamma: float = 1.4
    g_y: float = -0.1
    rho_h: float = 2.0
    rho_l: float = 1.0
    y0: float = 0.5
    h: float = 0.01
    p_int: float = 2.5
    cfl: float = 0.4
    comp_mask: int = COMP_UV
    # 0: primitive MC reconstruction on the closed-form background (the
    # workloads); 1: the well-balanced variant (row-balanced background and
    # hydrostatic pressure slopes), which keeps the unperturbed state to
    # round-off instead of relying on a subtracted baseline run
    recon: int = RECON_PRIMITIVE

    @property
    def dx(self) -> float:
        return self.lx / self.nx

    @property
    def dy(self) -> float:
        return self.ly / self.ny

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def with_(self, **kw) -> "RTConfig":
        return replace(self, **kw)

    def as_dict(self) -> dict:
        return asdict(self)


def paper_preset(n: int = 128, batch: int = 1) -> RTConfig:
    """The paper's parameters: unit square, gamma = 5/3, g = 1, h_s = 0.02,
    rho_h = 2, rho_l = 1, p(y = L) = rho_h g L, u_y-only perturbation."""
    L, g, rho_h, rho_l, hs, y0 = 1.0, 1.0, 2.0, 1.0, 0.02, 0.5
    # p(L) = rho_h g L; the interface pressure follows from the hydrostatic
    # integral of Eq. 5 between y0 and L.
    rbar, drho = 0.5 * (rho_h + rho_l), 0.5 * (rho_h - rho_l)
    z = (L - y0) / hs
    lncosh = abs(z) + math.log1p(math.exp(-2 * abs(z))) - math.log(2.0)
    p_int = rho_h * g * L + g * (rbar * (L - y0) + drho * hs * lncosh)
    return RTConfig(nx=n, ny=n, batch=batch, lx=L, ly=L, gamma=5.0 / 3.0, g_y=-g, rho_h=rho_h,
                    rho_l=rho_l, y0=y0, h=hs, p_int=p_int, cfl=0.4, comp_mask=COMP_V)


# The five benchmark workloads.
WORKLOADS = {
    # forward only, 64x128, T = 2, seed RMS 1e-3
    "fwd_64x128": dict(cfg=RTConfig(nx=64, ny=128), T=2.0),
    # forward + adjoint gradient, 256x512, T = 2, checkpoint every 32 steps
    "grad_256x512": dict(cfg=RTConfig(nx=256, ny=512), T=2.0),
    # batched ensemble of 64 at 128x256, T = 2
    "ensemble_64x128x256": dict(cfg=RTConfig(nx=128, ny=256, batch=64), T=2.0),
    # CNOP loop, 8 restarts at 512x1024, T in {1, 4}
    "cnop_8x512x1024": dict(cfg=RTConfig(nx=512, ny=1024, batch=8), T=1.0),
    # high resolution forward + adjoint, 1024x2048, T = 3
    "grad_1024x2048": dict(cfg=RTConfig(nx=1024, ny=2048), T=3.0),
}
