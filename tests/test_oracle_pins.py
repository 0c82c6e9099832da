"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks it against a
textbook solution, a closed form, an exact invariant of the discrete scheme,
a symmetry, or an independent derivative (finite differences, forward- vs
reverse-mode AD).
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import exact_riemann
from oracle import rto
from oracle.rto import Oracle, OracleError, hllc, wall_pressure
from paper_2608_04085_amd import inputs
from paper_2608_04085_amd.config import (NORM_L2, NORM_RHO_KE, NORM_RMS, RECON_BALANCED, RECON_PRIMITIVE,
                                         SET_BALL, SET_SPHERE, RTConfig, paper_preset)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *v = line.split()
            out[k] = [float(x) for x in v] if len(v) > 1 else float(v[0])
    return out


def _state(cfg, rho, u, v, p):
    """Conserved state [1][4][ny][nx] from primitive fields."""
    g = cfg.gamma
    U = np.empty((1, 4, cfg.ny, cfg.nx))
    U[0, 0] = rho
    U[0, 1] = rho * u
    U[0, 2] = rho * v
    U[0, 3] = p / (g - 1) + 0.5 * rho * (u * u + v * v)
    return U


def _prims(cfg, U):
    r = U[0, 0]
    u = U[0, 1] / r
    v = U[0, 2] / r
    p = (cfg.gamma - 1) * (U[0, 3] - 0.5 * r * (u * u + v * v))
    return r, u, v, p


# ------------------------------------------------------------ exact Riemann
def test_exact_riemann_sod_star_state_matches_textbook():
    g = _golden("sod_star_state.txt")
    p, u = exact_riemann.star_state(g["left"], g["right"], g["gamma"])
    assert abs(p - g["p_star"]) < 1e-5
    assert abs(u - g["u_star"]) < 1e-5
    w = exact_riemann.sample(g["left"], g["right"], np.array([u - 1e-9, u + 1e-9]), g["gamma"])
    assert abs(w[0, 0] - g["rho_star_left"]) < 1e-5
    assert abs(w[1, 0] - g["rho_star_right"]) < 1e-5


# ------------------------------------------------------------ HLLC
def test_hllc_stationary_contact_is_exact():
    # Density and tangential-velocity jump, uniform pressure, no normal flow:
    # the HLLC flux is exactly (0, p, 0, 0).
    f = hllc(1.4, [1.0, 0.0, 0.3, 2.5], [0.125, 0.0, -0.7, 2.5])
    assert f.tolist() == [0.0, 2.5, 0.0, 0.0]


@pytest.mark.parametrize("state", [[1.0, 0.3, -0.2, 1.0], [0.5, -2.0, 0.1, 0.4], [2.0, 3.0, 1.0, 0.5]])
def test_hllc_consistency_with_physical_flux(state):
    r, n, t, p = state
    E = p / 0.4 + 0.5 * r * (n * n + t * t)
    exact = np.array([r * n, r * n * n + p, r * n * t, n * (E + p)])
    f = hllc(1.4, state, state)
    np.testing.assert_allclose(f, exact, rtol=1e-14, atol=1e-14)


def test_hllc_supersonic_upwinding():
    # All waves move right: the flux is the left physical flux.
    L = [1.0, 5.0, 0.2, 1.0]
    f = hllc(1.4, L, [0.8, 4.5, -0.1, 0.7])
    np.testing.assert_allclose(f, hllc(1.4, L, L), rtol=0, atol=0)


@pytest.mark.parametrize("w", [[1.3, 0.02, -0.1, 2.4], [1.0, -0.3, 0.5, 0.9], [2.0, 0.0, 0.0, 1.0]])
def test_wall_pressure_equals_mirror_riemann_problem(w):
    # Top wall: interior on the left, mirror on the right (normal velocity
    # negated).  The HLLC normal-momentum flux of that problem is p*.
    mirror = [w[0], -w[1], w[2], w[3]]
    f = hllc(1.4, w, mirror)
    assert abs(f[0]) < 1e-14 and abs(f[3]) < 1e-13
    np.testing.assert_allclose(wall_pressure(1.4, w, True), f[1], rtol=1e-14)
    g = hllc(1.4, mirror, w)
    np.testing.assert_allclose(wall_pressure(1.4, w, False), g[1], rtol=1e-14)


# ------------------------------------------------------------ background
def test_background_is_hydrostatic_by_quadrature():
    cfg = RTConfig()
    o = Oracle.from_config(cfg)
    rho0, p0 = o.background()
    y = (np.arange(cfg.ny) + 0.5) * cfg.dy
    # Eq. 5 directly.
    np.testing.assert_allclose(rho0, 1.5 + 0.5 * np.tanh((y - 0.5) / 0.01), rtol=1e-15)
    # p0(y) = p_int + g int_{y0}^{y} rho0 by adaptive quadrature.
    for j in [0, 10, 63, 64, 70, 127]:
        q, _ = integrate.quad(lambda s: 1.5 + 0.5 * math.tanh((s - 0.5) / 0.01), 0.5, y[j],
                              epsabs=1e-13, epsrel=1e-13, limit=400)
        assert abs(p0[j] - (2.5 - 0.1 * q)) < 1e-12


def test_cfl_step_count_of_the_64x128_workload():
    # The forward workload quotes about 1.2k steps to T = 2 at CFL 0.4; the
    # largest signal speed sits at the bottom wall: c = sqrt(1.4 p / rho).
    cfg = RTConfig()
    o = Oracle.from_config(cfg)
    U0 = o.init_state(inputs.seed_batch(cfg, [0]))
    dt0 = o.cfl_dt(U0)[0]
    r, u, v, p = _prims(cfg, U0)
    c = np.sqrt(1.4 * p / r)
    expect = 0.4 / np.max(np.maximum((np.abs(u) + c) / cfg.dx, (np.abs(v) + c) / cfg.dy))
    assert dt0 == pytest.approx(expect, rel=1e-15)
    assert dt0 == pytest.approx(1.654e-3, rel=2e-3)
    _, t, n, _ = o.integrate(U0, 2.0)
    assert t[0] == 2.0 and 1150 <= n[0] <= 1250


def test_stored_long_march_gradient_is_the_oracles():
    # The stored 64x128 gradient fixture (written by make_oracle_gradients.py
    # from the oracle) belongs to the oracle as it stands: same step count
    # and R from a plain forward run; its inner products are those of the
    # stored sample with each direction's entries there bounded by |g| |d|.
    ref = _golden("oracle_gradient_64x128_T2.txt")
    cfg = RTConfig(nx=int(ref["nx"]), ny=int(ref["ny"]))
    o = Oracle.from_config(cfg)
    uv = inputs.seed_batch(cfg, [0], rms=1e-3)
    U0 = o.init_state(uv)
    UT, t, n, _ = o.integrate(U0, ref["T"])
    assert int(n[0]) == int(ref["nsteps"])
    assert (o.kinetic_energy(UT) / o.kinetic_energy(U0))[0] == ref["R"]
    assert len(ref["gd"]) == len(ref["dir_seeds"]) == 8 and len(ref["idx"]) == len(ref["gval"]) == 64
    assert np.max(np.abs(ref["gval"])) == ref["gmax"]
    assert ref["gmax"] <= ref["gnorm"]


# ------------------------------------------------------------ whole-step pins
def test_stationary_contact_and_shear_preserved_exactly():
    cfg = RTConfig(nx=16, ny=16, g_y=0.0)
    o = Oracle.from_config(cfg)
    x = (np.arange(16) + 0.5) * cfg.dx
    rho = np.where(x[None, :] < 0.25, 1.0, 0.125) * np.ones((16, 1))
    v = np.where(x[None, :] < 0.25, 0.3, -0.4) * np.ones((16, 1))  # shear along the contact
    U = _state(cfg, rho, 0.0 * rho, 0.0 * rho, 1.0 + 0.0 * rho)
    U2 = _state(cfg, rho, 0.0 * rho, 0.0 * rho + 0.0, 1.0 + 0.0 * rho)
    for _ in range(50):
        U = o.step(U, 1e-3)
    np.testing.assert_array_equal(U, U2)
    # pure shear: tangential velocity jump at uniform rho, p (y walls see v = 0)
    cfg2 = RTConfig(nx=16, ny=16, g_y=0.0)
    o2 = Oracle.from_config(cfg2)
    Us = _state(cfg2, 1.0 + 0 * rho, 0 * rho, v, 1.0 + 0 * rho)
    Us2 = Us.copy()
    # v is normal to the y walls, so put the shear in u along y instead
    y = (np.arange(16) + 0.5) * cfg2.dy
    u = np.where(y[:, None] < 0.5, 0.3, -0.4) * np.ones((1, 16))
    Us = _state(cfg2, 1.0 + 0 * rho, u, 0 * rho, 1.0 + 0 * rho)
    Us2 = Us.copy()
    for _ in range(50):
        Us = o2.step(Us, 1e-3)
    np.testing.assert_allclose(Us, Us2, rtol=0, atol=1e-15)


def _sod_y(ny, nx=4):
    cfg = RTConfig(nx=nx, ny=ny, lx=nx / ny, ly=1.0, g_y=0.0, cfl=0.4)
    y = (np.arange(ny) + 0.5) / ny
    low = (y < 0.5)[:, None] * np.ones((1, nx))
    U = _state(cfg, np.where(low, 1.0, 0.125), 0 * low, 0 * low, np.where(low, 1.0, 0.1))
    return cfg, U


@pytest.mark.parametrize("dummy", [0])
def test_sod_along_y_converges_to_exact_solution(dummy):
    errs = []
    for ny in (64, 128, 256):
        cfg, U = _sod_y(ny)
        o = Oracle.from_config(cfg)
        U, t, n, _ = o.integrate(U, 0.2)
        r = U[0, 0].mean(axis=1)
        # x-uniform to round-off
        assert np.max(np.abs(U[0, 0] - r[:, None])) == 0.0
        edges = np.arange(ny + 1) / ny
        ex = exact_riemann.cell_averages((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 0.5, 0.2, edges)
        errs.append(np.mean(np.abs(r - ex[:, 0])))
        # mass conserved with walls
        assert abs(U[0, 0].mean() - (0.5 + 0.0625)) < 1e-13
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 5e-3
    assert min(orders) >= 0.6, (errs, orders)


def test_sod_along_x_matches_sod_along_y():
    ny = 128
    cfg, U = _sod_y(ny)
    o = Oracle.from_config(cfg)
    Uy, _, _, _ = o.integrate(U, 0.2)
    # periodic x: [0, 2] with the left state in [0, 0.5) and (1.5, 2], right
    # state between; the two tubes do not interact before t = 0.2.
    nx = 2 * ny
    cfgx = RTConfig(nx=nx, ny=4, lx=2.0, ly=4.0 / ny, g_y=0.0)
    x = (np.arange(nx) + 0.5) / ny
    hi = ((x < 0.5) | (x > 1.5))[None, :] * np.ones((4, 1))
    Ux = _state(cfgx, np.where(hi, 1.0, 0.125), 0 * hi, 0 * hi, np.where(hi, 1.0, 0.1))
    ox = Oracle.from_config(cfgx)
    Ux, _, _, _ = ox.integrate(Ux, 0.2)
    ry = Uy[0, 0, :, 0]
    rx = Ux[0, 0, 0, :ny]
    np.testing.assert_allclose(rx, ry, rtol=0, atol=1e-12)
    np.testing.assert_allclose(Ux[0, 1, 0, :ny], Uy[0, 2, :, 0], rtol=0, atol=1e-12)


def test_conservation_with_walls_and_gravity():
    cfg = RTConfig(nx=32, ny=64)
    o = Oracle.from_config(cfg)
    uv = inputs.seed_batch(cfg, [3], rms=3e-2)
    U = o.init_state(uv)
    y = (np.arange(cfg.ny) + 0.5) * cfg.dy
    phi = (-cfg.g_y * y)[:, None]

    def invariants(U):
        return np.array([U[0, 0].sum(), U[0, 1].sum(), (U[0, 3] + U[0, 0] * phi).sum()])

    I0 = invariants(U)
    for _ in range(300):
        U = o.step(U, o.cfl_dt(U))
    I1 = invariants(U)
    assert abs(I1[0] - I0[0]) / abs(I0[0]) < 1e-13
    assert abs(I1[1] - I0[1]) < 1e-13 * abs(I0[0])  # m_x starts near 0; scale by mass
    assert abs(I1[2] - I0[2]) / abs(I0[2]) < 1e-13


def test_hydrostatic_uniform_density_is_preserved():
    # Atwood number zero: uniform rho, linear p.  MC picks the central slope,
    # so the pressure gradient and the gravity source cancel exactly.
    cfg = RTConfig(nx=16, ny=64, rho_h=1.5, rho_l=1.5)
    o = Oracle.from_config(cfg)
    U0 = o.init_state(np.zeros((1, 2, cfg.ny, cfg.nx)))
    U, _, n, _ = o.integrate(U0, 0.5)
    assert n[0] > 50
    np.testing.assert_allclose(U[0, 0], U0[0, 0], rtol=1e-12, atol=0)
    np.testing.assert_allclose(U[0, 3], U0[0, 3], rtol=1e-12, atol=0)
    assert np.max(np.abs(U[0, 1:3])) < 1e-12


def test_unperturbed_two_layer_state_stays_x_uniform_bitwise():
    cfg = RTConfig(nx=16, ny=64)
    o = Oracle.from_config(cfg)
    U, _, _, _ = o.integrate(o.init_state(np.zeros((1, 2, cfg.ny, cfg.nx))), 0.3)
    assert np.all(U[0, 1] == 0.0)
    for k in range(4):
        assert np.all(U[0, k] == U[0, k][:, :1])


@pytest.mark.slow
def test_hydrostatic_residual_shrinks_under_refinement():
    # The scheme is not well balanced; the paper notes the residual numerical
    # response of the smoothed atmosphere (Sec. 3.2).  It must converge away.
    res = []
    for nx, ny in ((32, 64), (64, 128)):
        cfg = RTConfig(nx=nx, ny=ny)
        o = Oracle.from_config(cfg)
        U, _, _, _ = o.integrate(o.init_state(np.zeros((1, 2, ny, nx))), 0.25)
        res.append(o.kinetic_energy(U)[0])
    assert res[1] < 0.5 * res[0], res


# ------------------------------------------- well-balanced variant (recon = 1)
def test_balanced_variant_keeps_the_unperturbed_state_to_round_off():
    # the primitive reconstruction leaves a residual flow (above); the
    # balanced one keeps the two-layer state at rest to round-off, on the
    # workload physics and on the paper preset
    for cfg in (RTConfig(nx=32, ny=128, recon=RECON_BALANCED), paper_preset(32).with_(recon=RECON_BALANCED)):
        o = Oracle.from_config(cfg)
        U0 = o.init_state(np.zeros((1, 2, cfg.ny, cfg.nx)))
        U, _, n, _ = o.integrate(U0, 1.0)
        assert n[0] > 100
        assert np.max(np.abs(U[0, 1:3] / U[0, 0])) <= 1e-13
        for k in (0, 3):  # density and energy, normwise
            assert np.max(np.abs(U[0, k] - U0[0, k])) <= 1e-13 * np.max(np.abs(U0[0, k]))
        Up, _, _, _ = Oracle.from_config(cfg.with_(recon=RECON_PRIMITIVE)).integrate(U0, 1.0)
        assert np.max(np.abs(Up[0, 2] / Up[0, 0])) > 1e-8  # the primitive variant does move


def test_balanced_background_is_row_balanced_and_converges_to_the_closed_form():
    errs = []
    for ny in (256, 512, 1024):  # dy below the interface width h = 0.01
        cfg = RTConfig(nx=4, ny=ny, recon=RECON_BALANCED)
        rho, p = Oracle.from_config(cfg).background()
        np.testing.assert_allclose(np.diff(p), cfg.g_y * cfg.dy * 0.5 * (rho[1:] + rho[:-1]), rtol=0, atol=1e-13)
        _, pc = Oracle.from_config(cfg.with_(recon=RECON_PRIMITIVE)).background()
        assert p[0] == pc[0]
        errs.append(np.max(np.abs(p - pc)))
    # second order: the trapezoid rule's error of the hydrostatic integral
    assert errs[1] < 0.3 * errs[0] and errs[2] < 0.3 * errs[1], errs


def test_balanced_variant_without_gravity_is_the_primitive_scheme_bitwise():
    cfg = RTConfig(nx=16, ny=24, g_y=0.0)
    o0, o1 = Oracle.from_config(cfg), Oracle.from_config(cfg.with_(recon=RECON_BALANCED))
    uv = inputs.seed_batch(cfg, [5], rms=3e-2)
    U0 = o0.init_state(uv)
    np.testing.assert_array_equal(o1.init_state(uv), U0)
    np.testing.assert_array_equal(o1.integrate(U0, 0.2)[0], o0.integrate(U0, 0.2)[0])


def test_balanced_variant_tangent_adjoint_and_gradient_pins():
    cfg = RTConfig(nx=8, ny=16, recon=RECON_BALANCED)
    o, U = _random_state(cfg, 14)
    rng = np.random.default_rng(4)
    dU = rng.standard_normal(U.shape)
    w = rng.standard_normal(U.shape)
    dt = o.cfl_dt(U)
    _, jv = o.step_jvp(U, dU, dt)
    vj = o.step_vjp(U, dt, w)
    a, b = np.sum(jv * w), np.sum(dU * vj)
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))
    # the gradient of R against central differences of the frozen-schedule
    # march.  The limiter here acts on the small departures from balance, so
    # its case boundaries lie closer together than in the primitive variant
    # and the differences need smaller steps (h <= 1e-7 of the seed).
    uv = inputs.seed_batch(cfg, [0], rms=1e-3)
    R, g, n, log = o.grad_u0(uv, 0.3, cap=4096)
    delta = np.sqrt(np.sum(uv * uv) * cfg.dx * cfg.dy)
    for s in range(1000, 1004):
        d = inputs.direction_batch(cfg, [s], delta)
        an = np.sum(g * d)
        errs = []
        for h in (1e-6, 1e-7, 1e-8):
            fp = o.ke_ratio_frozen(uv + h * d, log, n)[0]
            fm = o.ke_ratio_frozen(uv - h * d, log, n)[0]
            errs.append(abs((fp - fm) / (2 * h) - an) / abs(an))
        assert min(errs) <= 2e-6, (s, errs)


def test_periodic_shift_equivariance_bitwise():
    cfg = RTConfig(nx=24, ny=32)
    o = Oracle.from_config(cfg)
    uv = inputs.seed_batch(cfg, [5], rms=1e-2)
    U = o.init_state(uv)
    Us = np.roll(U, 7, axis=3)
    for _ in range(20):
        dt = o.cfl_dt(U)
        assert o.cfl_dt(Us)[0] == dt[0]
        U, Us = o.step(U, dt), o.step(Us, dt)
    np.testing.assert_array_equal(np.roll(U, 7, axis=3), Us)


def test_x_mirror_symmetry():
    cfg = RTConfig(nx=24, ny=32)
    o = Oracle.from_config(cfg)
    U = o.init_state(inputs.seed_batch(cfg, [6], rms=1e-2))
    Um = U[:, :, :, ::-1].copy()
    Um[:, 1] *= -1
    for _ in range(20):
        dt = o.cfl_dt(U)
        U, Um = o.step(U, dt), o.step(Um, dt)
    back = Um[:, :, :, ::-1].copy()
    back[:, 1] *= -1
    scale = np.max(np.abs(U), axis=(0, 2, 3))
    for k in range(4):
        assert np.max(np.abs(back[0, k] - U[0, k])) <= 1e-13 * max(scale[k], 1e-3)


# ------------------------------------------------------------ derivatives
def _random_state(cfg, seed, amp=3e-2):
    o = Oracle.from_config(cfg)
    U = o.init_state(inputs.seed_batch(cfg, [seed], rms=amp))
    for _ in range(3):  # develop non-trivial slopes
        U = o.step(U, o.cfl_dt(U))
    return o, U


@pytest.mark.parametrize("nx,ny", [(8, 16), (16, 32)])
def test_step_dot_product_tangent_vs_adjoint(nx, ny):
    cfg = RTConfig(nx=nx, ny=ny)
    o, U = _random_state(cfg, 11)
    rng = np.random.default_rng(0)
    dU = rng.standard_normal(U.shape)
    w = rng.standard_normal(U.shape)
    dt = o.cfl_dt(U)
    _, jv = o.step_jvp(U, dU, dt)
    vj = o.step_vjp(U, dt, w)
    a, b = np.sum(jv * w), np.sum(dU * vj)
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def test_fifty_step_dot_product_tangent_vs_adjoint():
    cfg = RTConfig(nx=8, ny=16)
    o, U = _random_state(cfg, 12)
    rng = np.random.default_rng(1)
    dU0 = rng.standard_normal(U.shape)
    w = rng.standard_normal(U.shape)
    states, dts = [], []
    X, dX = U.copy(), dU0.copy()
    for _ in range(50):
        dt = o.cfl_dt(X)
        states.append(X)
        dts.append(dt)
        X, dX = o.step_jvp(X, dX, dt)
    lam = w.copy()
    for s in range(49, -1, -1):
        lam = o.step_vjp(states[s], dts[s], lam)
    a, b = np.sum(dX * w), np.sum(dU0 * lam)
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def test_step_jacobian_matches_central_differences():
    cfg = RTConfig(nx=8, ny=16)
    o, U = _random_state(cfg, 13)
    # Noise in every cell so that no limited slope sits exactly at a kink
    # (the background is exactly x-uniform, where MC is not differentiable).
    rng = np.random.default_rng(2)
    U = U * (1.0 + 1e-3 * rng.standard_normal(U.shape))
    dt = o.cfl_dt(U)
    d = rng.standard_normal(U.shape) * np.abs(U) * 1e-2
    _, jv = o.step_jvp(U, d, dt)
    h = 1e-6
    fd = (o.step(U + h * d, dt) - o.step(U - h * d, dt)) / (2 * h)
    assert np.max(np.abs(fd - jv)) <= 1e-6 * np.max(np.abs(jv))


def test_step_adjoint_reaches_two_cells_and_is_local():
    # Each face's predicted states use the MC slopes of the two cells beside
    # it, whose stencils reach one cell further, and a cell's update sees its
    # four faces: the step depends on the box of cells within two of a cell,
    # walls included (the ghost rows mirror interior rows).  So a cotangent
    # on a window gives an adjoint supported on the window grown by exactly
    # two cells, and on a block of the grid with the same spacing the
    # block's own adjoint equals the grid's around the window.
    cfg = RTConfig(nx=48, ny=64)
    o, U = _random_state(cfg, 14)
    dt = o.cfl_dt(U)
    size, w = 32, 8
    x0 = (size - w) // 2
    for j0, wy0, shift in ((0, 0, 16), (16, 12, -5), (cfg.ny - size, size - w, 3)):
        Ur = np.ascontiguousarray(np.roll(U, shift, axis=3))
        lam_next = np.zeros_like(Ur)
        lam_next[:, :, j0 + wy0 : j0 + wy0 + w, x0 : x0 + w] = np.random.default_rng(j0).standard_normal((1, 4, w, w))
        lam = o.step_vjp(Ur, dt, lam_next)

        def outside(r):
            m = np.ones(lam.shape[2:], dtype=bool)
            m[max(j0 + wy0 - r, 0) : j0 + wy0 + w + r, x0 - r : x0 + w + r] = False
            return m

        assert np.count_nonzero(lam[:, :, outside(2)]) == 0
        assert np.count_nonzero(lam[:, :, outside(1)]) > 0
        sub = cfg.with_(nx=size, ny=size, lx=size * cfg.dx, ly=size * cfg.dy)
        ref = Oracle.from_config(sub).step_vjp(np.ascontiguousarray(Ur[:, :, j0 : j0 + size, :size]), dt,
                                               np.ascontiguousarray(lam_next[:, :, j0 : j0 + size, :size]))
        ya, yb = max(wy0 - 4, 0), min(wy0 + w + 4, size)
        np.testing.assert_array_equal(lam[:, :, j0 + ya : j0 + yb, x0 - 4 : x0 + w + 4],
                                      ref[:, :, ya:yb, x0 - 4 : x0 + w + 4])


@pytest.mark.parametrize("nx,ny,T", [(8, 16, 0.3), (16, 32, 0.15)])
def test_gradient_matches_central_differences(nx, ny, T):
    cfg = RTConfig(nx=nx, ny=ny)
    o = Oracle.from_config(cfg)
    uv = inputs.seed_batch(cfg, [0], rms=1e-3)
    R, g, n, log = o.grad_u0(uv, T, cap=4096)
    delta = np.sqrt(np.sum(uv * uv) * cfg.dx * cfg.dy)
    # The frozen-schedule map is piecewise smooth (limiter and Riemann-solver
    # cases); a finite difference straddling a kink is off by O(h).  Two step
    # sizes: at least one must resolve the derivative.
    for s in range(1000, 1004):
        d = inputs.direction_batch(cfg, [s], delta)
        an = np.sum(g * d)
        errs = []
        for h in (1e-5, 1e-6):
            fp = o.ke_ratio_frozen(uv + h * d, log, n)[0]
            fm = o.ke_ratio_frozen(uv - h * d, log, n)[0]
            errs.append(abs((fp - fm) / (2 * h) - an) / abs(an))
        assert min(errs) <= 1e-6, (s, errs)
    # the frozen-schedule map reproduces the adaptive run
    assert o.ke_ratio_frozen(uv, log, n)[0] == R[0]


def test_gradient_terminal_and_initial_closed_forms():
    # With zero steps' worth of dynamics removed analytically: dR/dU^N equals
    # (1/KE0) (-|m|^2/(2 rho^2), m_x/rho, m_y/rho, 0) dV, and the initial
    # chain gives rho0 (lam_m + u0 lam_E) - (R/KE0) rho0 u0 dV.  Check both on
    # a one-step march by assembling the gradient from the step adjoint.
    cfg = RTConfig(nx=8, ny=16)
    o = Oracle.from_config(cfg)
    uv = inputs.seed_batch(cfg, [4], rms=1e-3)
    U0 = o.init_state(uv)
    T = 0.5 * o.cfl_dt(U0)[0]  # a single clipped step
    R, g, n, _ = o.grad_u0(uv, T, cap=8)
    assert n[0] == 1
    U1 = o.step(U0, T)
    ke0 = o.kinetic_energy(U0)[0]
    dV = cfg.dx * cfg.dy
    r, mx, my = U1[0, 0], U1[0, 1], U1[0, 2]
    lamN = np.stack([-(mx * mx + my * my) / (2 * r * r), mx / r, my / r, 0 * r])[None] * dV / ke0
    lam0 = o.step_vjp(U0, T, lamN)
    rho0 = U0[0, 0]
    gu = rho0 * (lam0[0, 1] + uv[0, 0] * lam0[0, 3]) - R[0] / ke0 * rho0 * uv[0, 0] * dV
    gv = rho0 * (lam0[0, 2] + uv[0, 1] * lam0[0, 3]) - R[0] / ke0 * rho0 * uv[0, 1] * dV
    scale = np.max(np.abs(g))
    assert np.max(np.abs(gu - g[0, 0])) <= 1e-13 * scale
    assert np.max(np.abs(gv - g[0, 1])) <= 1e-13 * scale


def test_gradient_v_only_mask_zeroes_u():
    cfg = RTConfig(nx=8, ny=16, comp_mask=2)
    o = Oracle.from_config(cfg)
    uv = inputs.seed_batch(cfg, [0], rms=1e-3)
    assert np.all(uv[0, 0] == 0)
    _, g, _, _ = o.grad_u0(uv, 0.1)
    assert np.all(g[0, 0] == 0) and np.any(g[0, 1] != 0)


# ------------------------------------------------------------ objective of Eq. 8
def test_ek_field_is_half_rho_speed_squared():
    # Eq. 7 from primitive fields built independently of the conserved state
    cfg = RTConfig(nx=8, ny=16)
    o = Oracle.from_config(cfg)
    rng = np.random.default_rng(11)
    rho = 1.0 + rng.random((cfg.ny, cfg.nx))
    u, v = rng.standard_normal((2, cfg.ny, cfg.nx))
    U = _state(cfg, rho, u, v, 1.0 + rng.random((cfg.ny, cfg.nx)))
    np.testing.assert_allclose(o.ek_field(U)[0], 0.5 * rho * (u * u + v * v), rtol=1e-14)


def test_ek_anomaly_vanishes_at_the_baseline_with_zero_gradient():
    # the unperturbed run reproduces the baseline field: J = 0, and J is
    # quadratic in the anomaly, so its gradient there is exactly zero
    cfg = paper_preset(16, batch=1).with_(nx=8, ny=16)
    o = Oracle.from_config(cfg)
    T = 0.2
    ekb = o.baseline_ek(T)
    J, g, n, _ = o.grad_ek_anomaly(np.zeros(o.shape_uv), T, ekb)
    assert J[0] == 0.0 and n[0] > 0
    assert np.all(g == 0.0)


def test_ek_anomaly_one_tiny_step_approaches_closed_form():
    # After one step of length tau -> 0, U(tau) -> U(0), so J -> sum over
    # cells of (rho0 |u0|^2 / 2 - e_k,base)^2 dV with e_k,base -> 0; the
    # difference is O(tau).
    cfg = RTConfig(nx=8, ny=16)
    o = Oracle.from_config(cfg)
    uv = inputs.seed_batch(cfg, [2], rms=1e-1)
    rho0 = o.background()[0][:, None]
    closed = np.sum((0.5 * rho0 * (uv[0, 0] ** 2 + uv[0, 1] ** 2)) ** 2) * cfg.dx * cfg.dy
    errs = []
    for tau in (1e-6, 1e-8):
        J, _, n, _ = o.grad_ek_anomaly(uv, tau, o.baseline_ek(tau))
        assert n[0] == 1
        errs.append(abs(J[0] - closed) / closed)
    assert errs[1] <= 1e-6 and errs[1] < errs[0]


@pytest.mark.parametrize("nx,ny,T", [(8, 16, 0.3), (16, 16, 0.15)])
def test_ek_anomaly_gradient_matches_central_differences(nx, ny, T):
    cfg = paper_preset(16).with_(nx=nx, ny=ny)
    o = Oracle.from_config(cfg)
    uv = inputs.seed_batch(cfg, [0], rms=1e-2)
    assert np.all(uv[0, 0] == 0)  # u_y-only perturbation of the paper
    ekb = o.baseline_ek(T)
    J, g, n, log = o.grad_ek_anomaly(uv, T, ekb, cap=4096)
    assert np.all(g[0, 0] == 0)
    delta = np.sqrt(np.sum(uv * uv) * cfg.dx * cfg.dy)
    for s in range(1000, 1004):
        d = inputs.direction_batch(cfg, [s], delta)
        an = np.sum(g * d)
        errs = []
        for h in (1e-5, 1e-6):
            fp = o.ek_anomaly_frozen(uv + h * d, log, n, ekb)[0]
            fm = o.ek_anomaly_frozen(uv - h * d, log, n, ekb)[0]
            errs.append(abs((fp - fm) / (2 * h) - an) / abs(an))
        assert min(errs) <= 1e-6, (s, errs)
    assert o.ek_anomaly_frozen(uv, log, n, ekb)[0] == J[0]


def test_ek_anomaly_terminal_adjoint_closed_form():
    # one clipped step: dJ/dU^N = 2 (e_k - e_k,base) (-|m|^2/(2 rho^2), m_x/rho,
    # m_y/rho, 0) dV, then the step adjoint and the initial chain
    # rho0 (lam_m + u0 lam_E)
    cfg = RTConfig(nx=8, ny=16)
    o = Oracle.from_config(cfg)
    uv = inputs.seed_batch(cfg, [4], rms=1e-2)
    U0 = o.init_state(uv)
    T = 0.5 * o.cfl_dt(U0)[0]
    rng = np.random.default_rng(3)
    ekb = 1e-6 * rng.random((1, cfg.ny, cfg.nx))
    J, g, n, _ = o.grad_ek_anomaly(uv, T, ekb, cap=8)
    assert n[0] == 1
    U1 = o.step(U0, T)
    dV = cfg.dx * cfg.dy
    r, mx, my = U1[0, 0], U1[0, 1], U1[0, 2]
    ek = 0.5 * (mx * mx + my * my) / r
    np.testing.assert_allclose(J[0], np.sum((ek - ekb[0]) ** 2) * dV, rtol=1e-12)
    w = 2 * (ek - ekb[0]) * dV
    lamN = np.stack([-w * (mx * mx + my * my) / (2 * r * r), w * mx / r, w * my / r, 0 * r])[None]
    lam0 = o.step_vjp(U0, T, lamN)
    rho0 = U0[0, 0]
    gu = rho0 * (lam0[0, 1] + uv[0, 0] * lam0[0, 3])
    gv = rho0 * (lam0[0, 2] + uv[0, 1] * lam0[0, 3])
    scale = np.max(np.abs(g))
    assert np.max(np.abs(gu - g[0, 0])) <= 1e-12 * scale
    assert np.max(np.abs(gv - g[0, 1])) <= 1e-12 * scale


# ------------------------------------------- gradient through the adaptive march
def _adaptive_case(cfg, seed, amp):
    """A white-noise velocity field (so that one cell clearly holds the
    largest signal speed) and an end time half-way through the second-last
    CFL step of a 0.3-long run (so that the step count does not change under
    a small perturbation)."""
    o = Oracle.from_config(cfg)
    rng = np.random.default_rng(seed)
    uv = amp * rng.standard_normal((1, 2, cfg.ny, cfg.nx))
    uv = uv * np.array([1.0 if cfg.comp_mask & 1 else 0.0, 1.0 if cfg.comp_mask & 2 else 0.0])[None, :, None, None]
    _, _, n, log = o.integrate(o.init_state(uv), 0.3, cap=4096)
    dts = log[0, : n[0]]
    T = float(np.sum(dts[:-2]) + 0.5 * dts[-2])
    return o, uv, T, rng


@pytest.mark.parametrize("objective", ["R", "J"])
def test_adaptive_gradient_matches_central_differences_of_the_adaptive_map(objective):
    # the full derivative (CFL steps depend on the state, the last step on
    # the earlier ones) against finite differences of the adaptive march
    # itself; the frozen-schedule gradient misses those terms and fails the
    # same bound by orders of magnitude, so the check sees them
    if objective == "R":
        cfg = RTConfig(nx=8, ny=16)
        o, uv, T, rng = _adaptive_case(cfg, 5, 0.05)
        ekb = None
        _, gf, _, _ = o.grad_u0(uv, T)
    else:
        cfg = paper_preset(16).with_(nx=8, ny=16)
        o, uv, T, rng = _adaptive_case(cfg, 6, 0.05)
        ekb = o.baseline_ek(T)
        _, gf, _, _ = o.grad_ek_anomaly(uv, T, ekb)
    v, g, n = o.grad_adaptive(uv, T, ekb)
    v2, n2 = o.objective_adaptive(uv, T, ekb)
    assert v2[0] == v[0] and n2[0] == n[0] > 2
    assert np.linalg.norm(g - gf) > 1e-5 * np.linalg.norm(g)
    for s in range(4):
        d = np.abs(uv).mean() * rng.standard_normal(uv.shape) * (uv != 0)
        an, anf = np.sum(g * d), np.sum(gf * d)
        errs = []
        for h in (1e-5, 1e-6):
            fp = o.objective_adaptive(uv + h * d, T, ekb)[0][0]
            fm = o.objective_adaptive(uv - h * d, T, ekb)[0][0]
            fd = (fp - fm) / (2 * h)
            errs.append(abs(fd - an) / abs(an))
        assert min(errs) <= 1e-7, (s, errs)
        assert abs(fd - anf) / abs(anf) > 1e-5


def test_adaptive_gradient_of_a_single_clipped_step_is_the_frozen_one():
    # one step of length T: dt does not depend on the state, so both
    # derivatives are the same map's
    cfg = RTConfig(nx=8, ny=16)
    o, uv, _, _ = _adaptive_case(cfg, 7, 0.05)
    T = 0.5 * o.cfl_dt(o.init_state(uv))[0]
    v, g, n = o.grad_adaptive(uv, T)
    vf, gf, nf, _ = o.grad_u0(uv, T)
    assert n[0] == nf[0] == 1 and v[0] == vf[0]
    np.testing.assert_allclose(g, gf, rtol=0, atol=1e-13 * np.max(np.abs(gf)))


def test_adaptive_march_is_the_frozen_march_of_its_own_schedule():
    # the primal of the adaptive map equals the frozen map at the logged steps
    cfg = RTConfig(nx=8, ny=16)
    o, uv, T, _ = _adaptive_case(cfg, 8, 0.05)
    v, n = o.objective_adaptive(uv, T)
    R, _, nf, log = o.grad_u0(uv, T, cap=4096)
    assert v[0] == R[0] and n[0] == nf[0]
    assert o.ke_ratio_frozen(uv, log, nf)[0] == v[0]


# ------------------------------------------------------------ mixing width (Eqs. 13-14)
def test_mix_width_special_profiles():
    cfg = RTConfig(nx=6, ny=40)
    o = Oracle.from_config(cfg)
    one = np.ones((cfg.ny, cfg.nx))
    mid = 0.5 * (cfg.rho_h + cfg.rho_l)
    # fully mixed: f = 1/2 everywhere, 4 f (1 - f) = 1, width = Ly
    assert abs(o.mix_width(_state(cfg, mid * one, 0 * one, 0 * one, one))[0] - cfg.ly) <= 1e-14
    # sharp two-layer state and densities outside [rho_l, rho_h]: no mixed layer
    y = (np.arange(cfg.ny) + 0.5) * cfg.dy
    sharp = np.where(y[:, None] > cfg.y0, cfg.rho_h, cfg.rho_l) * one
    assert o.mix_width(_state(cfg, sharp, 0 * one, 0 * one, one))[0] == 0.0
    out = np.where(y[:, None] > cfg.y0, 3.0, 0.5) * one
    assert o.mix_width(_state(cfg, out, 0 * one, 0 * one, one))[0] == 0.0
    # only row means matter: shuffling cells within rows changes nothing
    rng = np.random.default_rng(0)
    r = cfg.rho_l + (cfg.rho_h - cfg.rho_l) * rng.random((cfg.ny, cfg.nx))
    a = o.mix_width(_state(cfg, r, 0 * one, 0 * one, one))[0]
    b = o.mix_width(_state(cfg, rng.permuted(r, axis=1), 0 * one, 0 * one, one))[0]
    assert abs(a - b) <= 1e-14 * a


def test_mix_width_of_the_tanh_background():
    # f = (1 + tanh z)/2, 4 f (1 - f) = sech^2 z: the width is
    # h (tanh((Ly - y0)/h) + tanh(y0/h)), close to 2h, up to the midpoint rule
    cfg = RTConfig(nx=4, ny=4096)
    o = Oracle.from_config(cfg)
    U = o.init_state(np.zeros(o.shape_uv))
    exact = cfg.h * (math.tanh((cfg.ly - cfg.y0) / cfg.h) + math.tanh(cfg.y0 / cfg.h))
    assert abs(o.mix_width(U)[0] - exact) <= 1e-6 * exact


# ------------------------------------------------------------ projection
def test_projection_sphere_ball_and_energy_norm():
    cfg = RTConfig(nx=16, ny=32, batch=2)
    o = Oracle.from_config(cfg)
    uv = inputs.seed_batch(cfg, [1, 2], rms=1.0)
    dV = cfg.dx * cfg.dy
    out, m = o.project_to_constraint(uv, 1e-3, NORM_L2, SET_SPHERE)
    np.testing.assert_allclose(m, np.sqrt(np.sum(uv ** 2, axis=(1, 2, 3)) * dV), rtol=1e-14)
    np.testing.assert_allclose(np.sqrt(np.sum(out ** 2, axis=(1, 2, 3)) * dV), 1e-3, rtol=1e-14)
    out, m = o.project_to_constraint(uv, 1e-3, NORM_RMS, SET_SPHERE)
    np.testing.assert_allclose(np.sqrt(np.mean(np.sum(out ** 2, axis=1), axis=(1, 2))), 1e-3, rtol=1e-14)
    # ball: a point inside is left untouched (Eq. 11, first case)
    small = uv * 1e-9
    out, _ = o.project_to_constraint(small, 1e-3, NORM_L2, SET_BALL)
    np.testing.assert_array_equal(out, small)
    # energy constraint of Eq. 9: C = int rho0 |u|^2 / 2 dV saturated at eps
    y = (np.arange(cfg.ny) + 0.5) * cfg.dy
    rho0 = 1.5 + 0.5 * np.tanh((y - 0.5) / 0.01)
    out, C = o.project_to_constraint(uv, 1e-6, NORM_RHO_KE, SET_BALL)
    C_exp = np.sum(0.5 * rho0[None, None, :, None] * uv ** 2, axis=(1, 2, 3)) * dV
    np.testing.assert_allclose(C, C_exp, rtol=1e-13)
    C_after = np.sum(0.5 * rho0[None, None, :, None] * out ** 2, axis=(1, 2, 3)) * dV
    np.testing.assert_allclose(C_after, 1e-6, rtol=1e-13)


def test_projection_rejects_zero_field_on_sphere():
    cfg = RTConfig(nx=8, ny=16)
    o = Oracle.from_config(cfg)
    with pytest.raises(OracleError):
        o.project_to_constraint(np.zeros((1, 2, 16, 8)), 1e-3, NORM_L2, SET_SPHERE)


def test_paper_preset_pressure_anchor():
    cfg = paper_preset(64)
    o = Oracle.from_config(cfg)
    # p(y = L) = rho_h g L (Sec. 2.2), via the closed-form hydrostatic profile
    y_top = cfg.ly
    rbar, drho = 1.5, 0.5
    z = (y_top - 0.5) / 0.02
    p_top = cfg.p_int + cfg.g_y * (rbar * (y_top - 0.5) + drho * 0.02 * (abs(z) + math.log1p(math.exp(-2 * abs(z))) - math.log(2)))
    assert abs(p_top - 2.0) < 1e-14
    rho0, p0 = o.background()
    assert p0[-1] > 2.0 and p0[0] > p0[-1]


def _sigma_linear(cfg, kx, n=4000):
    """Growth rate s of the most unstable incompressible mode w(y) exp(i k x + s t)
    of the tanh density profile between the walls (linear theory of a
    continuously stratified fluid): -(rho0 w')' + k^2 rho0 w = (g k^2 / s^2)
    rho0' w with w(0) = w(Ly) = 0, by second-order finite differences (rho0'
    as the jump of rho0 across each cell, so that a thin interface is exact).
    Its thin-interface limit is Eq. 6's sqrt(A g k)."""
    import scipy.sparse as sp
    from scipy.sparse.linalg import eigsh

    k = 2 * math.pi * kx / cfg.lx
    dy = cfg.ly / (n + 1)
    y = dy * np.arange(1, n + 1)
    rbar, drho = 0.5 * (cfg.rho_h + cfg.rho_l), 0.5 * (cfg.rho_h - cfg.rho_l)

    def rho(yy):
        return rbar + drho * np.tanh((yy - cfg.y0) / cfg.h)

    rp, rm = rho(y + dy / 2), rho(y - dy / 2)
    A = sp.diags([(rp + rm) / dy**2 + k * k * rho(y), -rp[:-1] / dy**2, -rp[:-1] / dy**2], [0, 1, -1], format="csc")
    M = sp.diags((rp - rm) / dy, 0, format="csc")
    nu = eigsh(M, k=1, M=A, which="LA", return_eigenvectors=False)[0]  # s^2 / (g k^2)
    return math.sqrt(nu * (-cfg.g_y) * k * k)


def _fitted_growth(cfg, kx, T=3.0, dt_out=0.1):
    """Growth rate of a single horizontal mode kx seeded in v at amplitude
    1e-5 (the v-perturbation against the unperturbed run), from a fit of
    a e^{s t} + b e^{-s t} to its amplitude over t in [1, T]: a velocity
    seed starts the unstable mode as a mix of both exponentials."""
    from scipy.optimize import curve_fit

    o = Oracle.from_config(cfg)
    uv = inputs.fourier_seed(cfg, kx, 0.0)[None] * 1e-5
    U, Ub = o.init_state(uv), o.init_state(0 * uv)
    ts, amps = [], []
    for m in range(int(round(T / dt_out))):
        U, _, _, _ = o.integrate(U, dt_out)
        Ub, _, _, _ = o.integrate(Ub, dt_out)
        v = U[0, 2] / U[0, 0] - Ub[0, 2] / Ub[0, 0]
        ts.append(dt_out * (m + 1))
        amps.append(np.sqrt(np.sum(np.abs(np.fft.rfft(v, axis=1)[:, kx]) ** 2)))
    ts, amps = np.array(ts), np.array(amps)
    sel = ts >= 1.0 - 1e-9

    def model(t, a, b, s):
        return np.log(a * np.exp(s * t) + b * np.exp(-s * t))

    p, _ = curve_fit(model, ts[sel], np.log(amps[sel]), p0=[amps[sel][0] / 2, amps[sel][0] / 2, 0.5], maxfev=20000)
    return p[2]


def test_linear_rt_growth_rate_against_sqrt_agk():
    # Eq. 6: sigma = sqrt(A g k) for a thin interface; the paper's reference
    # mode (n_k = 2, g = 1, L = 1, A = 1/3) has tau = 1/sigma = 0.49.
    assert abs(1.0 / math.sqrt((1.0 / 3.0) * 1.0 * (2 * math.pi * 2)) - 0.49) < 0.005
    cfg = RTConfig()
    A = (cfg.rho_h - cfg.rho_l) / (cfg.rho_h + cfg.rho_l)

    def sharp(kx):
        return math.sqrt(A * (-cfg.g_y) * 2 * math.pi * kx / cfg.lx)

    # the linear-theory rate of the workload's tanh interface (h = 0.01)
    # tends to Eq. 6 as the interface thins (walls 0.5 away: k H >= 6)
    for kx in (1, 2):
        assert abs(_sigma_linear(cfg.with_(h=1e-5), kx) / sharp(kx) - 1) < 5e-3
    s1, s2 = _sigma_linear(cfg, 1), _sigma_linear(cfg, 2)
    assert 0.94 < s1 / sharp(1) < 0.95 and 0.895 < s2 / sharp(2) < 0.905  # k h = 0.126, 0.251
    # The march grows single modes at that rate: kx = 1 (64 cells per
    # wavelength, 1.3 cells across h at 32 x 128) within 4 % of it
    # (measured +2.4 %); for kx = 2 refinement moves the rate to it
    # (32 x 128: -8.3 %, 64 x 256: -3.8 %).
    f1 = _fitted_growth(RTConfig(nx=32, ny=128), 1)
    assert abs(f1 / s1 - 1) < 0.04, (f1, s1)
    f2c = _fitted_growth(RTConfig(nx=32, ny=128), 2)
    f2f = _fitted_growth(RTConfig(nx=64, ny=256), 2)
    assert abs(f2f / s2 - 1) < abs(f2c / s2 - 1) and abs(f2f / s2 - 1) < 0.06, (f2c, f2f, s2)


# ------------------------------------------------------------ spectrum (Eq. 12)
def test_row_spectrum_against_rfft_single_mode_and_parseval():
    cfg = RTConfig(nx=48, ny=20, batch=2)
    o = Oracle.from_config(cfg)
    rng = np.random.default_rng(4)
    f = rng.standard_normal((2, cfg.ny, cfg.nx))
    E = o.row_spectrum(f)
    # the library FFT: sum over rows of |rfft|^2
    np.testing.assert_allclose(E, np.sum(np.abs(np.fft.rfft(f, axis=2)) ** 2, axis=1), rtol=1e-12, atol=1e-9)
    # Parseval (nx even: the n = 0 and Nyquist bins once, the others twice)
    w = np.full(cfg.nx // 2 + 1, 2.0)
    w[0] = w[-1] = 1.0
    np.testing.assert_allclose(E @ w, cfg.nx * np.sum(f * f, axis=(1, 2)), rtol=1e-12)
    # one selected row
    np.testing.assert_allclose(o.row_spectrum(f, row=7)[1], np.abs(np.fft.rfft(f[1, 7])) ** 2, rtol=1e-12,
                               atol=1e-10)
    # a single horizontal mode k puts (nx/2)^2 sum_j env_j^2 into bin k alone
    i = np.arange(cfg.nx)
    env = np.exp(-((np.arange(cfg.ny) - 9.5) / 4.0) ** 2)
    g = np.broadcast_to(np.cos(2 * np.pi * 5 * i / cfg.nx + 0.3)[None, None, :] * env[None, :, None],
                        (2, cfg.ny, cfg.nx))
    Eg = o.row_spectrum(g)
    assert Eg[0, 5] == pytest.approx((cfg.nx / 2) ** 2 * np.sum(env**2), rel=1e-13)
    assert np.max(np.delete(Eg[0], 5)) <= 1e-24 * Eg[0, 5]


# ------------------------------------------------------------ limiter, slopes, predictor
# The monotonized-central limiter (R-4) case by case, with values computed by
# hand: zero at an extremum or a zero difference, the central difference
# (a+b)/2 while it is within 2|a| and 2|b| (also where it equals one of them),
# else 2a if |a| <= |b|, else 2b.  The derivatives are the weights of the
# selected case (the adjoint's reading).  Minmod, superbee or van Leer give
# other values on several rows.
MC_TABLE = [
    # a, b, tol, slope, d/da, d/db
    (1.0, -1.0, 0.0, 0.0, 0.0, 0.0),     # extremum
    (-2.0, 3.0, 0.0, 0.0, 0.0, 0.0),     # extremum
    (0.0, 2.0, 0.0, 0.0, 0.0, 0.0),      # a = 0
    (2.0, 0.0, 0.0, 0.0, 0.0, 0.0),      # b = 0
    (1.0, 1.0, 0.0, 1.0, 0.5, 0.5),      # central
    (2.0, 3.0, 0.0, 2.5, 0.5, 0.5),      # central
    (1.0, 3.0, 0.0, 2.0, 0.5, 0.5),      # central = 2a: central is taken
    (3.0, 1.0, 0.0, 2.0, 0.5, 0.5),      # central = 2b: central is taken
    (1.0, 4.0, 0.0, 2.0, 2.0, 0.0),      # 2a
    (4.0, 1.0, 0.0, 2.0, 0.0, 2.0),      # 2b
    (-1.0, -4.0, 0.0, -2.0, 2.0, 0.0),   # 2a, negative
    (-5.0, -0.5, 0.0, -1.0, 0.0, 2.0),   # 2b, negative
    (-3.0, -1.0, 0.0, -2.0, 0.5, 0.5),   # central = 2b, negative
    (0.25, 8.0, 0.0, 0.5, 2.0, 0.0),     # 2a far from central
    (1e-12, 1.0, 1e-11, 0.0, 0.0, 0.0),  # a below the tolerance
    (1.0, -1e-12, 1e-11, 0.0, 0.0, 0.0), # b below the tolerance (and of the other sign)
    (1e-10, 1.0, 1e-11, 2e-10, 2.0, 0.0),  # a above the tolerance
]


@pytest.mark.parametrize("a,b,tol,s,da,db", MC_TABLE)
def test_mc_limiter_case_table(a, b, tol, s, da, db):
    got = rto.mc_slope(a, b, tol)
    assert got == (s, da, db)


def test_slopes_scale_the_tie_tolerance_by_density_pressure_and_sound_speed():
    # A difference counts as zero below tie_tol times the cell's density
    # (density), pressure (pressure) or sound speed (velocities).  With
    # rho = 2, p = 1.4, gamma = 1.4: c = sqrt(0.98) = 0.98995 and tie_tol =
    # 1e-10 give thresholds 2e-10, 1.4e-10 and 0.98995e-10.
    cfg = RTConfig(nx=4, ny=4, g_y=0.0)
    o = Oracle.from_config(cfg, tie_tol=1e-10)
    w = np.array([2.0, 0.3, -0.2, 1.4])
    for k, thr in ((0, 2e-10), (1, 0.98995e-10), (2, 0.98995e-10), (3, 1.4e-10)):
        for d, zero in ((0.9 * thr, True), (1.1 * thr, False)):
            wm = w.copy()
            wm[k] -= d
            wp = w.copy()
            wp[k] += 1.0
            s = rto.slopes(o, wm, w, wp)
            expect = 0.0 if zero else 2.0 * (w[k] - wm[k])  # 2a, a as rounded
            assert s[k] == expect, (k, d)
            assert all(s[j] == 0.0 for j in range(4) if j != k)
    # with tie_tol = 0 the same differences give the plain MC slopes
    o0 = Oracle.from_config(cfg, tie_tol=0.0)
    wm = w - np.array([1e-12, 1e-12, 1e-12, 1e-12])
    wp = w + np.array([1.0, 1.0, 1.0, 1.0])
    np.testing.assert_allclose(rto.slopes(o0, wm, w, wp), 2e-12, rtol=1e-3)
    # the balanced y slope of the pressure: rho g_y dy plus MC of the departures
    cfgb = RTConfig(nx=4, ny=4, g_y=-0.5, ly=1.0)
    ob = Oracle.from_config(cfgb, tie_tol=0.0)
    h = 2.0 * (-0.5) * 0.25
    wm = w.copy(); wm[3] = w[3] - h - 0.01
    wp = w.copy(); wp[3] = w[3] + h + 0.03
    assert rto.slopes(ob, wm, w, wp, balanced=True)[3] == pytest.approx(h + 0.02, rel=1e-13)


def _euler_flux(U, axis, gamma):
    """Physical flux of the conservative Euler equations (Eqs. 1-4) along x
    (axis 0) or y (axis 1); U = (rho, m_x, m_y, E), complex allowed."""
    r, mx, my, E = U
    u, v = mx / r, my / r
    p = (gamma - 1) * (E - 0.5 * r * (u * u + v * v))
    n = u if axis == 0 else v
    return np.array([r * n, mx * n + (p if axis == 0 else 0), my * n + (p if axis == 1 else 0), n * (E + p)])


def _cons(W, gamma):
    r, u, v, p = W
    return np.array([r, r * u, r * v, p / (gamma - 1) + 0.5 * r * (u * u + v * v)])


def _prim(U, gamma):
    r, mx, my, E = U
    u, v = mx / r, my / r
    return np.array([r, u, v, (gamma - 1) * (E - 0.5 * r * (u * u + v * v))])


def _quasilinear(W, dW, axis, gamma, h=1e-30):
    """A(W) dW of the primitive form W_t + A_x W_x + A_y W_y = 0, derived from
    the conservative flux: A = (dW/dU)(dF/dU)(dU/dW), each product by a
    complex-step derivative (exact to round-off)."""
    dF = np.imag(_euler_flux(_cons(W + 1j * h * dW, gamma), axis, gamma)) / h
    return np.imag(_prim(_cons(W, gamma) + 1j * h * dF, gamma)) / h


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_predictor_is_the_quasilinear_half_step(seed):
    # R-5: W^{n+1/2} = W - dt/(2 dx) A_x(W) s_x - dt/(2 dy) A_y(W) s_y
    # + (dt/2)(0, 0, g_y, 0), with A_x, A_y taken here from the conservative
    # flux, not from the primitive equations the oracle writes out.
    rng = np.random.default_rng(seed)
    cfg = RTConfig(nx=8, ny=16, lx=0.5, ly=1.0, gamma=1.4, g_y=-0.3)
    o = Oracle.from_config(cfg)
    W = np.array([1.0 + rng.random(), rng.normal(), rng.normal(), 1.0 + rng.random()])
    sx, sy = rng.normal(size=4) * 0.1, rng.normal(size=4) * 0.1
    dt = 1e-3 * (1 + rng.random())
    expect = (W - 0.5 * dt / cfg.dx * _quasilinear(W, sx, 0, cfg.gamma)
              - 0.5 * dt / cfg.dy * _quasilinear(W, sy, 1, cfg.gamma) + np.array([0, 0, 0.5 * dt * cfg.g_y, 0]))
    got = rto.predict(o, W, sx, sy, dt)
    np.testing.assert_allclose(got, expect, rtol=0, atol=1e-14 * np.max(np.abs(W)))
    # and each term matters: the predictor moves every component by more
    # than the tolerance
    assert np.min(np.abs(got - W)) > 1e-8


# ------------------------------------------------------------ smooth solutions: second order
def _smooth_state(cfg, rho, u, v, p):
    return _state(cfg, rho, u, v, p)


def _entropy_wave_error(nx):
    # density wave carried at u = 1 with uniform pressure (g = 0): the exact
    # solution is the translated profile; after one period it is the initial
    # one, compared as exact cell averages
    cfg = RTConfig(nx=nx, ny=2, lx=1.0, ly=2.0 / nx, g_y=0.0)
    x = (np.arange(nx) + 0.5) / nx
    rho = (1 + 0.2 * np.sin(2 * np.pi * x))[None, :] * np.ones((2, 1))
    U = _smooth_state(cfg, rho, 1.0 + 0 * rho, 0 * rho, 1.0 + 0 * rho)
    U, _, _, _ = Oracle.from_config(cfg).integrate(U, 1.0)
    xe = np.arange(nx + 1) / nx
    avg = 1 + 0.2 * nx * (np.cos(2 * np.pi * xe[:-1]) - np.cos(2 * np.pi * xe[1:])) / (2 * np.pi)
    assert np.max(np.abs(U[0, 2])) == 0.0
    return np.mean(np.abs(U[0, 0, 0] - avg))


def test_smooth_entropy_wave_converges_at_second_order():
    # The MUSCL-Hancock scheme with MC slopes is second order on smooth flow
    # (first order only at the O(dx)-wide extrema, which the L1 norm weights
    # by dx).  Dropping the half-step predictor gives order 1; minmod slopes
    # give errors 5x larger at 256 cells.
    ns = (32, 64, 128, 256)
    errs = [_entropy_wave_error(n) for n in ns]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert orders[0] >= 1.7 and min(orders[1:]) >= 1.9, (errs, orders)
    assert errs[-1] <= 6e-5, errs


def _acoustic(n, axis, T=0.3, eps=0.01):
    """Small-amplitude isentropic acoustic wave along x (periodic, a sine
    travelling right) or y (between the walls, a cosine standing wave with
    zero normal velocity at the walls); g = 0.  Returns [4][n] along the
    wave's axis."""
    if axis == 0:
        cfg = RTConfig(nx=n, ny=2, lx=1.0, ly=2.0 / n, g_y=0.0)
        s = (np.arange(n) + 0.5) / n
        f = np.sin(2 * np.pi * s)[None, :] * np.ones((2, 1))
        c = math.sqrt(cfg.gamma)
        U = _smooth_state(cfg, 1 + eps * f, c * eps * f, 0 * f, 1 + cfg.gamma * eps * f)
    else:
        cfg = RTConfig(nx=3, ny=n, lx=3.0 / n, ly=1.0, g_y=0.0)
        s = (np.arange(n) + 0.5) / n
        f = np.cos(np.pi * s)[:, None] * np.ones((1, 3))
        U = _smooth_state(cfg, 1 + eps * f / cfg.gamma, 0 * f, 0 * f, 1 + eps * f)
    U, _, _, _ = Oracle.from_config(cfg).integrate(U, T)
    return U[0, :, 0, :] if axis == 0 else U[0, :, :, 0]


@pytest.mark.parametrize("axis", [0, 1])
def test_smooth_acoustic_wave_self_convergence_is_second_order(axis):
    # Self-convergence: the L1 difference between the solutions on n and 2n
    # cells (the fine one averaged onto the coarse cells) falls by ~4 per
    # refinement.  The wave exercises the predictor's r du, gamma p du and
    # dp/r terms along its axis (a dropped term gives order ~1) and, along y,
    # the wall ghosts.
    ns = (32, 64, 128, 256, 512)
    sol = [_acoustic(n, axis) for n in ns]
    diff = [np.mean(np.abs(a - 0.5 * (b[:, 0::2] + b[:, 1::2])), axis=1) for a, b in zip(sol[:-1], sol[1:])]
    normal = 1 + axis  # the momentum along the wave
    for k in (0, normal, 3):
        orders = [math.log2(diff[i][k] / diff[i + 1][k]) for i in range(len(diff) - 1)]
        assert min(orders) >= 1.9, (k, orders)
    # the momentum across the wave stays zero to round-off (HLLC's star
    # density rho (S_L - n)/(S_L - S*) of two equal states is rho only to an ulp)
    assert np.max(np.abs(sol[-1][2 - axis])) <= 1e-14


# ------------------------------------------------------------ tie tolerance (R-12)
def test_tie_tolerance_moves_the_64x128_march_by_a_bounded_amount():
    # The tolerance below which the oracle (and the kernels) take a near-tie
    # in a discrete decision as a tie is a reading (R-12), not part of the
    # scheme of Sec. 2.3.  Against the plain decisions (tie_tol = 0) over the
    # 1210-step march of the 64x128 workload to T = 2, measured: the same step
    # count, R within 8.2e-12 relative, density and energy within 6.8e-11 and
    # 1.3e-11 of their largest values, the momenta (the perturbation, ~1e-3)
    # within 1.0e-8 and 4.4e-9 of theirs, and the step sizes within 3.8e-9.
    cfg = RTConfig(nx=64, ny=128)
    uv = inputs.seed_batch(cfg, [0], rms=1e-3)
    out = []
    for tol in (rto.TIE_TOL, 0.0):
        o = Oracle.from_config(cfg, tie_tol=tol)
        U0 = o.init_state(uv)
        UT, _, n, log = o.integrate(U0, 2.0, cap=1300)
        out.append((UT, int(n[0]), float(o.kinetic_energy(UT)[0] / o.kinetic_energy(U0)[0]), log[0, : int(n[0])]))
    (Ua, na, Ra, la), (Ub, nb, Rb, lb) = out
    assert na == nb == 1210
    assert abs(Ra - Rb) / Rb <= 5e-11
    rel = [np.max(np.abs(Ua[0, k] - Ub[0, k])) / np.max(np.abs(Ub[0, k])) for k in range(4)]
    assert rel[0] <= 5e-10 and rel[3] <= 5e-10, rel
    assert rel[1] <= 1e-7 and rel[2] <= 1e-7, rel
    assert np.max(np.abs(la - lb) / lb) <= 3e-8


# ------------------------------------------------------------ measurement aids
def test_algorithmic_flops_per_cell_of_the_benchmark():
    # The roofline of the benchmark compares the kernels' FP64 rate with the
    # algorithmic work of the scheme: every operation on state-dependent
    # values as the oracle writes it (rto_count.hpp), per cell, on the
    # workload's state half-way through a march: the step plus the signal
    # speed of the new state (forward), and for the adjoint the step again
    # plus one multiply-add per edge of the step's graph.
    import bench
    cfg = RTConfig(nx=128, ny=256)
    o = Oracle.from_config(cfg)
    U, _, _, _ = o.integrate(o.init_state(inputs.seed_batch(cfg, [0], rms=1e-3)), 1.0)
    c = rto.count_flops(o, U, o.cfl_dt(U))
    assert c["add"] + c["mul"] + c["div"] + c["sqrt"] == pytest.approx(c["step"])
    fwd = c["step"] + c["cfl"]
    adj = c["step"] + 2.0 * c["edges"]
    assert abs(fwd - bench.FWD_FLOPS_PER_CELL) <= 0.03 * fwd, fwd
    assert abs(adj - bench.ADJ_FLOPS_PER_CELL) <= 0.03 * adj, adj
    # the signal speed: c^2 = gamma p / rho (after the primitives), |u| + c,
    # |v| + c, each over its cell width: a fixed count per cell
    assert c["cfl"] == 16.0


def test_threaded_oracle_steps_are_bitwise_the_single_threaded_ones():
    cfg = RTConfig(nx=64, ny=128)
    o = Oracle.from_config(cfg)
    U = o.init_state(inputs.seed_batch(cfg, [2], rms=3e-2))
    dt = o.cfl_dt(U)
    one = o.step(U, dt)
    used = rto.set_threads(4)
    try:
        many = o.step(U, dt)
    finally:
        rto.set_threads(1)
    assert used in (1, 4)
    np.testing.assert_array_equal(one, many)


@pytest.mark.parametrize("nx,ny,band", [(48, 64, 16), (20, 33, 8), (16, 12, 3)])
def test_banded_step_adjoint_is_the_whole_grids_to_the_bit(nx, ny, band):
    # the helper behind the long-march GPU check: each step's adjoint on row
    # bands (each band's block grown by four rows, walls where the grid has
    # them) equals the whole grid's adjoint exactly
    from oracle import chain as oracle_chain
    cfg = RTConfig(nx=nx, ny=ny)
    o, U = _random_state(cfg, 21)
    dt = o.cfl_dt(U)
    lam_next = np.random.default_rng(5).standard_normal(U.shape)
    whole = o.step_vjp(U, dt, lam_next)
    np.testing.assert_array_equal(oracle_chain.banded_vjp(o, U, float(dt[0]), lam_next, band=band), whole)
    # and the closed-form terminal and initial adjoints are the oracle's own
    uv = inputs.seed_batch(cfg, [3], rms=1e-3)
    U0 = o.init_state(uv)
    UT, _, n, log = o.integrate(U0, 0.05, cap=256)
    ke0 = float(o.kinetic_energy(U0)[0])
    R = float(o.kinetic_energy(UT)[0]) / ke0
    states, V = [], U0
    for k in range(int(n[0])):
        states.append(V)
        V = o.step(V, log[0, k])
    lam0 = oracle_chain.adjoint_chain(o, lambda k: states[k], log[0, : int(n[0])],
                                      oracle_chain.terminal_adjoint_R(o, UT, ke0), workers=3, band=band)
    g = oracle_chain.initial_adjoint_R(o, uv, lam0, R, ke0)
    Ro, go, _, _ = o.grad_u0(uv, 0.05)
    assert abs(R - Ro[0]) <= 1e-15 * abs(Ro[0])
    assert np.max(np.abs(g - go)) <= 1e-12 * np.max(np.abs(go))


@pytest.mark.parametrize("nx,ny", [(16, 12), (15, 9), (8, 32)])
def test_power_spectrum_2d_against_rfft2_parseval_and_a_single_mode(nx, ny):
    # App. B's 2-D reconstruction keeps the strongest 2-D Fourier modes; the
    # oracle's spectrum is |2-D DFT|^2 on the half plane k = 0 .. nx/2
    cfg = RTConfig(nx=nx, ny=ny, batch=2)
    o = Oracle.from_config(cfg)
    f = np.random.default_rng(nx * ny).standard_normal((2, ny, nx))
    E = o.power_spectrum_2d(f)
    ref = np.abs(np.fft.rfft2(f)) ** 2  # numpy: full transform along y, half along x
    np.testing.assert_allclose(E, ref, rtol=1e-12, atol=1e-12 * ref.max())
    # Parseval: the full plane (the half plane with its mirror) holds
    # nx ny sum f^2
    w = np.full(nx // 2 + 1, 2.0)
    w[0] = 1.0
    if nx % 2 == 0:
        w[-1] = 1.0
    np.testing.assert_allclose((E * w).sum(axis=(1, 2)), nx * ny * (f * f).sum(axis=(1, 2)), rtol=1e-12)
    # a single 2-D mode cos(2 pi (3 x / nx + 2 y / ny)) lands in one bin of
    # the half plane with |F| = nx ny / 2
    x, y = np.arange(nx), np.arange(ny)
    m = np.cos(2 * np.pi * (3 * x[None, :] / nx + 2 * y[:, None] / ny))
    E1 = Oracle.from_config(cfg.with_(batch=1)).power_spectrum_2d(m[None])[0]
    assert E1[2, 3] == pytest.approx((nx * ny / 2) ** 2, rel=1e-12)
    E1[2, 3] = 0.0
    assert np.max(E1) <= 1e-20 * (nx * ny) ** 2
