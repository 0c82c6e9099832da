/*
 * rtcnop.h - C ABI of the MI355X (gfx950) hot path of the CNOP search for
 * the most dangerous initial velocity perturbation in 2-D compressible
 * Rayleigh-Taylor instability (Ji & Shi, "The Most Dangerous Seed").
 *
 * What the library computes
 *   - The forward map F_t of Sec. 3.1: the 2-D compressible Euler equations
 *     with uniform gravity (Sec. 2.1, Eqs. 1-4) on a uniform grid, by a
 *     finite-volume Godunov-type scheme with an HLLC Riemann solver and a
 *     gravity source (Sec. 2.3).  The paper leaves reconstruction and time
 *     integrator open; this is unsplit MUSCL-Hancock with monotonized-central
 *     limited slopes of (rho, u, v, p), plain HLLC with Davis wave speeds,
 *     and a gravity source that conserves total energy including the
 *     potential energy.  x is periodic; the y boundaries are reflecting walls
 *     whose ghost pressure is extrapolated hydrostatically (dp/dy = rho g,
 *     Sec. 2.1), with the wall flux equal to the wall pressure of the
 *     mirrored Riemann problem.  dt = CFL / max over cells of
 *     max((|u|+c)/dx, (|v|+c)/dy), the last step clipped to end at T.
 *   - The initial state: the two-layer tanh atmosphere of Eq. 5 in
 *     hydrostatic balance (Sec. 2.2), plus a velocity perturbation (u0, v0).
 *   - The kinetic energy KE = sum (m_x^2 + m_y^2)/(2 rho) dx dy (Eq. 7
 *     integrated) and the growth ratio R = KE(U(T)) / KE(U(0)).
 *   - The exact gradient of R with respect to the initial velocity field by a
 *     hand-written discrete adjoint of the step (the paper uses reverse-mode
 *     AD of the discrete march, Sec. 2.3 and 3.4), with the time steps of the
 *     forward run held fixed, and checkpointing to bound memory (Sec. 3.4).
 *   - The constraint projection of Eq. 11 (sphere or ball, in the velocity L2
 *     norm, the RMS norm or the energy norm C of Eq. 9).
 *
 * Conventions
 *   - Arrays are FP64, contiguous, in DEVICE memory owned by the caller
 *     (unless stated), 8-byte aligned at least; 256-byte alignment is best.
 *     State U is [B][4][ny][nx] with variables (rho, m_x, m_y, E), x fastest.
 *     Velocity fields (perturbation, gradient) are [B][2][ny][nx], (u, v).
 *   - The library never allocates device memory: all scratch lives in the
 *     workspace the caller hands to rt_set_workspace, and the checkpoint pool
 *     is handed in with each gradient call.
 *   - Calls are asynchronous on the context's stream (a hipStream_t passed
 *     as void*; NULL = the default stream) unless stated.  rt_integrate and
 *     rt_grad_u0 synchronise that stream (they read device step counters).
 *   - Kernels are launched on the calling thread's current HIP device; the
 *     context's stream, workspace and pool and every array passed in must
 *     belong to that device (the one current at rt_create).
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - Return value: 0 on success or a negative rt_status; rt_last_error()
 *     gives a message for the calling thread's last failure.
 */
#ifndef RTCNOP_H
#define RTCNOP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rt_status {
  RT_OK = 0,
  RT_EINVAL = -1,   /* bad shape, null pointer, T <= 0, zero KE(0), ...     */
  RT_EHIP = -2,     /* a HIP runtime call failed                             */
  RT_ENOMEM = -3,   /* workspace, step-log or checkpoint pool too small      */
  RT_EUNPHYS = -4,  /* rho <= 0, p <= 0 or a non-finite value was produced   */
  RT_ESTATE = -5    /* call order violated (e.g. no workspace set)           */
} rt_status;

/* Grid: nx x ny cells on [0, lx] x [0, ly]; batch independent members. */
typedef struct rt_grid {
  int32_t nx, ny, batch, reserved;
  double lx, ly;
} rt_grid;

/* Physics.  g_y < 0 points down.  The background is
 * rho0(y) = (rho_h + rho_l)/2 + (rho_h - rho_l)/2 tanh((y - y0)/h) (Eq. 5)
 * with p0 from dp0/dy = rho0 g_y and p0(y0) = p_int.  comp_mask: bit 0 = u
 * is perturbed, bit 1 = v (the paper perturbs v only, Sec. 3.1).
 * recon: RT_RECON_PRIMITIVE (MC slopes of the primitives, the background
 * in closed form at the cell centres: the scheme the workloads use), or
 * RT_RECON_BALANCED, a well-balanced variant beyond the paper's method:
 * the background pressure is built row by row, p_{j+1} = p_j + g_y dy
 * (rho0_j + rho0_{j+1})/2 from the closed form at the bottom row, and the y
 * slope of the pressure is rho g_y dy plus the MC slope of the departures
 * from that hydrostatic slope.  The unperturbed state then stays at rest to
 * round-off (the paper instead subtracts an unperturbed run, Sec. 3.2). */
typedef struct rt_phys {
  double gamma, g_y, rho_h, rho_l, y0, h, p_int, cfl;
  int32_t comp_mask, recon;
} rt_phys;

enum { RT_RECON_PRIMITIVE = 0, RT_RECON_BALANCED = 1 };

typedef struct rt_ctx rt_ctx;

/* Checkpoint policy of rt_grad_u0 (Sec. 3.4: checkpoints re-computed from a
 * sparse set of saved states).  kind: 0 store every state, 1 a snapshot every
 * `interval` steps with re-computation inside each interval, 2 binomial
 * (revolve) checkpointing using as many snapshots as `pool_bytes` holds, in
 * two levels (see rt_revolve_plan_stats; `interval` is not read).  The pool
 * is caller-owned device memory. */
typedef struct rt_ckpt_policy {
  int32_t kind, interval;
  void* pool;
  size_t pool_bytes;
} rt_ckpt_policy;

enum { RT_CKPT_STORE_ALL = 0, RT_CKPT_UNIFORM = 1, RT_CKPT_REVOLVE = 2 };
enum { RT_NORM_L2 = 0, RT_NORM_RMS = 1, RT_NORM_RHO_KE = 2 };
enum { RT_SET_SPHERE = 0, RT_SET_BALL = 1 };

/* Create a context for one grid / physics / stream.  Validates the numbers
 * (nx >= 3, ny >= 2, nx * ny < 2^28, batch >= 1, positive lengths,
 * gamma > 1, h > 0, cfl > 0, comp_mask 1..3, recon one of RT_RECON_*).  No
 * device work. */
int rt_create(const rt_grid* grid, const rt_phys* phys, void* stream, rt_ctx** out);
int rt_destroy(rt_ctx* ctx);
int rt_set_stream(rt_ctx* ctx, void* stream);

/* Bytes of device workspace needed for marches of up to max_steps steps per
 * member (the step log of the gradient needs one double per step). */
int rt_workspace_bytes(const rt_ctx* ctx, int32_t max_steps, size_t* bytes);
/* Hand the context its workspace (device, >= rt_workspace_bytes, 256-byte
 * aligned).  The context uses it until the next rt_set_workspace or
 * rt_destroy; the caller frees it afterwards. */
int rt_set_workspace(rt_ctx* ctx, void* dev, size_t bytes, int32_t max_steps);

/* Initial state (Sec. 2.2 and 3.1): U = background + velocity perturbation
 * uv0 ([B][2][ny][nx]) at cell centres; masked components are taken as 0.
 * With RT_RECON_BALANCED the background pressure is the row-balanced one
 * (see rt_phys). */
int rt_init_state(rt_ctx* ctx, const double* uv0, double* U);

/* CFL time step of each member's state (unclipped): dt[B] on the device. */
int rt_cfl_dt(rt_ctx* ctx, const double* U, double* dt);

/* One step U_out = Phi_dt(U_in) with the per-member step dt[B] (device).
 * U_in and U_out must not overlap.  If dt_next is not NULL it receives the
 * unclipped CFL step of U_out.  Unphysical states are reported on the next
 * rt_check_error or synchronising call. */
int rt_step(rt_ctx* ctx, const double* U_in, double* U_out, const double* dt, double* dt_next);

/* March every member from its state U (in/out) to exactly time T with its
 * own CFL step, all members advancing in one batched launch per step.
 * t_out[B], nsteps[B] (int32) receive the end time and step count; dt_log,
 * if not NULL, receives each member's steps, [B][dt_log_cap] (device).
 * Synchronises the stream.  RT_EUNPHYS if any member became unphysical,
 * RT_ENOMEM if a member needs more steps than the workspace allows. */
int rt_integrate(rt_ctx* ctx, double* U, double T, double* t_out, int32_t* nsteps, double* dt_log,
                 int32_t dt_log_cap);

/* Kinetic energy of each member, ke[B] (device). */
int rt_kinetic_energy(rt_ctx* ctx, const double* U, double* ke);

/* Growth ratio of the kinetic energy (the objective of Eq. 10 in the
 * workloads' form): R[b] = KE(UT_b) / KE(U0_b) for the states U0 and UT
 * ([B][4][ny][nx], device; typically the initial state and the state the
 * march reached at T).  R[B] is device memory.  A member with KE(U0) = 0
 * gets inf or NaN; the call does not check it (rt_grad_u0 does). */
int rt_ke_ratio(rt_ctx* ctx, const double* U0, const double* UT, double* R);

/* rt_ke_ratio for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and the same result to the bit, with their scratch (the
 * reductions' partial sums and the two kinetic energies) in a static device
 * array of the library, 512 KiB per GPU, held until the process ends, in
 * place of the context's workspace; no workspace needs to be set.  The call
 * allocates nothing; its first call on a device looks up that device's copy
 * of the array (make that first call before any graph capture).  Limit:
 * (red_blocks + 2) * batch <= 65536 doubles, where red_blocks = min(256,
 * max(1, nx * ny / 2048)): at most 254 members for grids of 2^19 cells or
 * more; beyond it RT_ENOMEM, decided on the host before any device work.
 * All calls on one GPU share the array: calls that overlap on one GPU
 * (other streams, other threads, other contexts) race, so the caller
 * serialises them.  Nothing in the array has to start at zero (every
 * partial is written before it is read).  Asynchronous on the context's
 * stream; U0, UT and R as rt_ke_ratio. */
int rt_ke_ratio_noalloc(rt_ctx* ctx, const double* U0, const double* UT, double* R);

/* Adjoint of one step: lam = (d Phi_dt / dU)(U)^T lam_next with dt[B]
 * (device) held fixed.  Arrays are states [B][4][ny][nx]; lam must not
 * overlap lam_next. */
int rt_step_adjoint(rt_ctx* ctx, const double* U, const double* dt, const double* lam_next, double* lam);

/* R[B] = KE(U(T))/KE(U(0)) for the initial perturbation uv0, and its
 * gradient dR/d(u0, v0) ([B][2][ny][nx], Euclidean, with respect to the
 * array entries) by the discrete adjoint with the forward run's time steps
 * held fixed (or differentiated: rt_set_dt_mode).  nsteps[B] (device, may
 * be NULL) receives the step counts.
 * Synchronises the stream.  RT_ENOMEM if the pool cannot hold the policy's
 * snapshots; RT_EINVAL if KE(0) = 0. */
int rt_grad_u0(rt_ctx* ctx, const double* uv0, double T, const rt_ckpt_policy* policy, double* R,
               double* grad, int32_t* nsteps);

/* Kinetic-energy density of Eq. 7, e_k = |m|^2 / (2 rho), of every cell:
 * U [B][4][ny][nx] -> ek [B][ny][nx] (device). */
int rt_ek_field(rt_ctx* ctx, const double* U, double* ek);

/* Mixing-layer width of Eqs. 13-14 for each member: h[B] = sum over rows
 * of 4 f (1 - f) dy, f = clip((<rho>_x - rho_l) / (rho_h - rho_l), 0, 1),
 * <rho>_x the mean density of the row (device arrays; U [B][4][ny][nx]). */
int rt_mix_width(rt_ctx* ctx, const double* U, double* h);

/* Horizontal power spectrum (Sec. 4.2, Eq. 12 before its normalisation) of
 * one scalar field per member: E[b][n] = sum over the selected rows j of
 * |sum_i f_b(i, j) exp(-2 pi i n i / nx)|^2 for n = 0 .. nx/2, E laid out
 * [B][nx/2 + 1] (device).  f (device) holds member b's field, ny rows of nx
 * doubles, from f + b * member_stride: pass member_stride = nx * ny for a
 * plain field, or f + nx * ny with member_stride = 2 * nx * ny for the v
 * component of a velocity field [B][2][ny][nx]; the caller's buffer must
 * hold (B - 1) * member_stride + nx * ny doubles from f.  row = -1 sums over
 * all rows, 0 <= row < ny takes one.  Eq. 12's E_n is E[b][n] over
 * sum_{m >= 1} E[b][m].  nx <= 4096.  Deterministic (a fixed-order sum). */
int rt_row_spectrum(rt_ctx* ctx, const double* f, int64_t member_stride, int32_t row, double* E);

/* 2-D power spectrum of one scalar field per member, the quantity whose
 * strongest modes, up to 90 % of the spectral energy, make the 2-D
 * reconstruction of App. B: E[b][q][k] = |F_b(q, k)|^2 with F_b(q, k) =
 * sum over cells of f_b(y, x) exp(-2 pi i (k x / nx + q y / ny)), for
 * q = 0 .. ny - 1 and k = 0 .. nx/2 (a real field's spectrum is symmetric,
 * E(q, k) = E(-q mod ny, nx - k), so this half plane holds all of it), E
 * laid out [B][ny][nx/2 + 1] (device).  f and member_stride as in
 * rt_row_spectrum.  nx, ny <= 4096.  Deterministic (fixed-order sums: the
 * transform of every row, then of every column).  Uses the workspace as
 * scratch. */
int rt_power_spectrum_2d(rt_ctx* ctx, const double* f, int64_t member_stride, double* E);

/* Objective of Eq. 8 on the grid: J[B] = sum over cells of
 * (e_k(U) - ek_base)^2 dx dy, with ek_base [B][ny][nx] the e_k field of the
 * unperturbed run at the same time (device arrays). */
int rt_ek_anomaly(rt_ctx* ctx, const double* U, const double* ek_base, double* J);

/* J[B] of Eq. 8 for the perturbation uv0 marched to time T, and its
 * gradient dJ/d(u0, v0) ([B][2][ny][nx]) by the discrete adjoint with the
 * forward run's time steps held fixed (Sec. 3.4; or differentiated:
 * rt_set_dt_mode), under the same checkpoint policies and with the same
 * kernels as rt_grad_u0.  ek_base is the
 * baseline field (rt_ek_field of the unperturbed march to T).  A zero
 * perturbation is allowed (J and the gradient are then those at the
 * baseline).  Synchronises the stream; errors as rt_grad_u0. */
int rt_grad_ek_anomaly(rt_ctx* ctx, const double* uv0, double T, const rt_ckpt_policy* policy,
                       const double* ek_base, double* J, double* grad, int32_t* nsteps);

/* Bytes of checkpoint pool that `kind`/`interval` needs for marches of
 * nsteps_max steps (RT_CKPT_UNIFORM: ceil(nsteps_max / interval) snapshots
 * plus two segment buffers of interval - 1 states, one fewer buffer being
 * the minimum; RT_CKPT_REVOLVE: the minimum, two snapshots). */
int rt_pool_bytes(const rt_ctx* ctx, int32_t kind, int32_t interval, int32_t nsteps_max, size_t* bytes);

/* Eq. 11: scale each member of uv ([B][2][ny][nx], in place) onto the
 * constraint set of radius delta in norm `norm`; set = sphere (always) or
 * ball (only when outside).  For RT_NORM_RHO_KE the bound is the energy
 * epsilon of Eq. 9 and the scale is (epsilon / C)^(1/2).  Masked components
 * are zeroed.  norm_out[B] (device, may be NULL) receives the norm (or C)
 * before scaling. */
int rt_project_to_constraint(rt_ctx* ctx, double* uv, double delta, int32_t norm, int32_t set,
                             double* norm_out);

/* Per-member inner products of velocity fields: out[B] = sum_cells a . b
 * (device).  Used by the spectral projected-gradient step. */
int rt_dot(rt_ctx* ctx, const double* a, const double* b, double* out);

/* Per-member largest magnitude of a velocity field: out[B] = max |a|
 * (device); the infinity norm of the stationarity measure of the search. */
int rt_max_abs(rt_ctx* ctx, const double* a, double* out);

/* out = x + alpha[b] * y per member (alpha device [B]); out may alias x. */
int rt_axpy(rt_ctx* ctx, const double* x, const double* alpha, const double* y, double* out);

/* Kernel variants.  The fused step and adjoint kernels come in tile shapes
 * 16x16, 32x8, 64x4 (256 threads), 16x16, 32x8 (576 threads, one pass per
 * phase), 16x8 (128), 8x8 (64), 16x8 (320, one pass), 8x8 (192, one
 * pass), 32x16 (512), 16x15 and 15x16 (256, every face loop in one pass);
 * ids 0..11 in that order.  Every variant gives bitwise-identical
 * results.  rt_set_tile selects one variant for both kernels;
 * rt_autotune times every variant on the state U (device) with `reps`
 * launches each on the context's stream (steps at a given dt and with the
 * CFL reduction; adjoint steps folded and as two kernels), keeps the
 * fastest step variant and the fastest adjoint variant and mode (see
 * rt_set_fold; variants returned in step_tile / adj_tile, may be NULL) and
 * synchronises the stream.  The workspace buffers serve as scratch. */
int rt_set_tile(rt_ctx* ctx, int32_t tile);
/* Select the step and adjoint variants separately. */
int rt_set_tiles(rt_ctx* ctx, int32_t step_tile, int32_t adj_tile);
/* The adaptive march replays captured HIP graphs of 48 steps (on = 1, the
 * default) or launches step by step (on = 0); results are identical. */
int rt_set_graphs(rt_ctx* ctx, int32_t on);
/* Second stream of the reverse sweep (default priority, created on first
 * use on the current device), on = 1 (the default) or 0.  RT_CKPT_UNIFORM
 * re-computes segment k-1 on it while the adjoint of segment k runs on the
 * context's stream, if the pool holds two segment buffers beside the
 * snapshots (the size rt_pool_bytes returns); with room for one, the sweep
 * runs on one stream.  RT_CKPT_REVOLVE with two or more members runs the
 * binomial plan for members [0, B/2) on the context's stream and for
 * [B/2, B) on the second one, one action later, each on its own slice of
 * every buffer.  Results are identical either way; on = 0 runs everything
 * on the context's stream. */
int rt_set_overlap(rt_ctx* ctx, int32_t on);
int rt_get_tiles(const rt_ctx* ctx, int32_t* step_tile, int32_t* adj_tile);
/* The step kernel's variant (as rt_get_tiles' step_tile). */
int rt_get_tile(const rt_ctx* ctx, int32_t* tile);
int rt_autotune(rt_ctx* ctx, const double* U, int32_t reps, int32_t* step_tile, int32_t* adj_tile);
/* The reverse sweep of RT_CKPT_STORE_ALL / RT_CKPT_UNIFORM runs one kernel
 * per adjoint step, which also completes the previous step's limiter gather
 * (on = 1), or the two kernels of rt_step_adjoint per step (on = 0); results
 * are identical.  rt_autotune folds when the folded step is more than 10%
 * faster than the two-kernel step on their own (the folded kernel shares
 * the CUs less well with the concurrent re-computation); before it, grids
 * of fewer than 2^16 cells in all fold (and use 8x8 single-pass tiles),
 * larger ones run two adjoint kernels, with 32x16 step and 32x8 adjoint
 * tiles up to three 32x8 blocks per CU and 16x15 tiles for both beyond.  Binomial checkpointing,
 * differentiated time steps (rt_set_dt_mode) and the well-balanced variant
 * (RT_RECON_BALANCED) always run two kernels per step. */
int rt_set_fold(rt_ctx* ctx, int32_t on);
int rt_get_fold(const rt_ctx* ctx, int32_t* on);

/* Time steps in the gradients of rt_grad_u0 and rt_grad_ek_anomaly.
 * RT_DT_FROZEN (the default): the steps of the forward run are held fixed,
 * so the gradient is that of the march with that schedule.
 * RT_DT_DIFFERENTIATED: the gradient of the adaptive march itself, in which
 * every step but the last is dt_n = cfl / S(U^n) (S the largest signal
 * speed, Sec. 2.3) and the last one is T - t_n.  The reverse sweep then also
 * forms mu_n = <lambda^{n+1}, dU^{n+1}/d dt_n> and, on every step before the
 * member's last, adds (mu_n - mu_last) d dt_n / dU^n at the cell holding the
 * largest speed (the first such cell in storage order on a tie, the y speed
 * on a tie between x and y).  The number of steps is taken as locally
 * constant.  This mode always runs two kernels per adjoint step plus one
 * small kernel; it is deterministic for a given adjoint tile, and tiles
 * differ only in the rounding of mu's sum. */
enum { RT_DT_FROZEN = 0, RT_DT_DIFFERENTIATED = 1 };
int rt_set_dt_mode(rt_ctx* ctx, int32_t mode);
int rt_get_dt_mode(const rt_ctx* ctx, int32_t* mode);
/* Measurement hook: per-launch times in microseconds of the selected
 * variants, from HIP events on the context's stream around `reps`
 * back-to-back launches each, with U (device) as every step's state:
 * out[0] a step at a given dt (as re-computed in the reverse sweep), out[1]
 * a step with the CFL reduction (as in the march), out[2] one folded
 * adjoint step (one kernel that also completes the previous step's limiter
 * gather), out[3] one rt_step_adjoint (two kernels), out[4] the adjoint step
 * in the sweep's current mode (out[2] or out[3]).  The well-balanced variant
 * has no folded form: there out[2] repeats out[3].  out holds 5 doubles.
 * Synchronises the stream; the workspace serves as scratch. */
int rt_kernel_times(rt_ctx* ctx, const double* U, int32_t reps, double* out);

/* Host-only check of the binomial checkpointing schedule (Sec. 3.4) that
 * RT_CKPT_REVOLVE runs: builds it for nsteps steps and `slots` state slots
 * (slot 0 holding the initial state), replays it on step indices, and fails
 * with RT_EINVAL unless every step is reversed exactly once, in decreasing
 * order, from the right state, using only the given slots.  forward receives
 * the schedule's count of forward steps, optimum the smallest count any
 * schedule with that many slots can reach.  No context, no device work. */
int rt_revolve_stats(int32_t nsteps, int32_t slots, int64_t* forward, int64_t* optimum);

/* Host-only check of the plan RT_CKPT_REVOLVE runs (Sec. 3.4's binomial
 * checkpointing, in two levels): the forward march that evaluates the
 * objective also leaves a snapshot every `interval` steps, an interval the
 * library picks from the step count n_est that the initial CFL step
 * suggests (so that 1.25 n_est steps fit in slots - 1 slots, at the least
 * re-computation); the reverse sweep then reverses each segment, last
 * first, with the binomial schedule on the slots left free.  If the march
 * needs more snapshots than fit, or one binomial schedule over the whole
 * march from U^0 re-computes less, that schedule runs instead.  For a march
 * of nsteps steps with `slots` slots: forward receives all forward steps of
 * the gradient (the objective's march included), interval the level-1
 * interval, two_level 1 if the two-level plan runs.  Replays the plan as
 * rt_revolve_stats does (RT_EINVAL if inconsistent).  nsteps >= 1,
 * slots >= 2, n_est >= 1.  No context, no device work. */
int rt_revolve_plan_stats(int32_t nsteps, int32_t slots, int32_t n_est, int64_t* forward, int32_t* interval,
                          int32_t* two_level);

/* Synchronise the stream and report a device-side error flag (RT_EUNPHYS)
 * raised by earlier asynchronous calls; clears the flag. */
int rt_check_error(rt_ctx* ctx);

const char* rt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RTCNOP_H */
