"""Seeded synthetic inputs: initial velocity perturbations (u0, v0).

This module only draws and shapes input fields; it holds none of the scheme's
arithmetic, and both the GPU path and the CPU oracle receive the same arrays
from it.  All fields are float64 numpy arrays laid out [B][2][ny][nx] with
component order (u, v) and x fastest.

* Gaussian seed: i.i.d. standard normal per cell and component (numpy's
  PCG64 generator, ``default_rng(seed)``) times the interface envelope
  exp(-((y - y0)/0.05)^2) at the cell centres.  The paper's initial guess is a
  zero-mean Gaussian random field localised near the density interface
  (Sec. 3.4); the envelope width 0.05 is that of the benchmark workload.
* Fourier seed: v0 = cos(2 pi kx x / Lx + phi) times the same envelope, u0 = 0
  (single horizontal modes, as in the batched ensemble).

The amplitude scalings below (to an RMS value or a velocity L2 norm) define
the size of the input, not a step of the method.
"""
from __future__ import annotations

import numpy as np

from .config import RTConfig

ENVELOPE_WIDTH = 0.05


def cell_centres(cfg: RTConfig):
    x = (np.arange(cfg.nx) + 0.5) * cfg.dx
    y = (np.arange(cfg.ny) + 0.5) * cfg.dy
    return x, y


def envelope(cfg: RTConfig, width: float = ENVELOPE_WIDTH) -> np.ndarray:
    _, y = cell_centres(cfg)
    return np.exp(-(((y - cfg.y0) / width) ** 2))


def gaussian_seed(cfg: RTConfig, seed: int, width: float = ENVELOPE_WIDTH) -> np.ndarray:
    """(2, ny, nx) envelope-masked i.i.d. Gaussian field, unscaled."""
    xi = np.random.default_rng(seed).standard_normal((2, cfg.ny, cfg.nx))
    return xi * envelope(cfg, width)[None, :, None]


def fourier_seed(cfg: RTConfig, kx: int, phase: float) -> np.ndarray:
    """(2, ny, nx) single horizontal mode in v, zero u, unscaled."""
    x, _ = cell_centres(cfg)
    out = np.zeros((2, cfg.ny, cfg.nx))
    out[1] = np.cos(2.0 * np.pi * kx * x / cfg.lx + phase)[None, :] * envelope(cfg)[:, None]
    return out


def scale_rms(uv: np.ndarray, rms: float) -> np.ndarray:
    """Scale so that sqrt(mean over cells of u^2 + v^2) = rms."""
    m = np.sqrt(np.mean(np.sum(uv * uv, axis=0)))
    return uv * (rms / m)


def scale_l2(uv: np.ndarray, cfg: RTConfig, delta: float) -> np.ndarray:
    """Scale so that (sum (u^2 + v^2) dx dy)^(1/2) = delta."""
    m = np.sqrt(np.sum(uv * uv) * cfg.dx * cfg.dy)
    return uv * (delta / m)


def mask_components(uv: np.ndarray, comp_mask: int) -> np.ndarray:
    out = uv.copy()
    if not comp_mask & 1:
        out[..., 0, :, :] = 0.0
    if not comp_mask & 2:
        out[..., 1, :, :] = 0.0
    return out


def seed_batch(cfg: RTConfig, seeds, rms: float | None = 1e-3, l2: float | None = None) -> np.ndarray:
    """[B][2][ny][nx] Gaussian seeds, one per entry of `seeds`."""
    out = []
    for s in seeds:
        uv = mask_components(gaussian_seed(cfg, int(s)), cfg.comp_mask)
        if l2 is not None:
            uv = scale_l2(uv, cfg, l2)
        elif rms is not None:
            uv = scale_rms(uv, rms)
        out.append(uv)
    return np.ascontiguousarray(np.stack(out))


def ensemble_batch(cfg: RTConfig, delta: float = 1e-3) -> np.ndarray:
    """The 64-member ensemble: members 0-31 Gaussian (seeds 0-31), members
    32-63 Fourier modes kx = 1..16 with phase 0 and pi/2, all at velocity L2
    norm delta.  For other batch sizes the same pattern is truncated or
    repeated."""
    members = []
    for b in range(cfg.batch):
        k = b % 64
        if k < 32:
            uv = gaussian_seed(cfg, k)
        else:
            m = k - 32
            uv = fourier_seed(cfg, 1 + m // 2, 0.0 if m % 2 == 0 else 0.5 * np.pi)
        members.append(scale_l2(mask_components(uv, cfg.comp_mask), cfg, delta))
    return np.ascontiguousarray(np.stack(members))


def direction_batch(cfg: RTConfig, seeds, delta: float) -> np.ndarray:
    """Envelope-masked Gaussian directions at L2 norm delta (for finite
    differences of the objective along random directions)."""
    return seed_batch(cfg, seeds, rms=None, l2=delta)


def paper_seed_batch(cfg: RTConfig, seeds, width_frac: float = 0.1) -> np.ndarray:
    """[B][2][ny][nx] initial guesses of the paper's search (Sec. 3.4): a
    Gaussian field localised near the interface with envelope width
    width_frac * Ly, in the components of cfg.comp_mask (v only for the
    paper's setup), unscaled; the caller scales it onto the constraint."""
    return np.ascontiguousarray(np.stack([mask_components(gaussian_seed(cfg, int(s), width_frac * cfg.ly),
                                                          cfg.comp_mask) for s in seeds]))
