// C ABI of the MI355X hot path (declared in include/rtcnop.h): context and
// workspace management, the batched CFL march, and the checkpointed discrete
// adjoint driver.  All device memory is the caller's; this file only carves
// the workspace and launches kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rtcnop.h"
#include "rt_diag.h"
#include "rt_kernels.h"
#include "rt_revolve.h"

using rtk::Ctl;
using rtk::Flags;
using rtk::Params;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define RT_HIP(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return fail(RT_EHIP, "%s: %s", #call, hipGetErrorString(e_));    \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// Member groups of the split binomial sweep: at most this many streams.
constexpr int kMaxGroups = 4;
// Groups the sweep uses (fewer if the batch has fewer members).
constexpr int kSplitGroups = 2;

struct rt_ctx {
  Params P;
  hipStream_t stream;
  int tile;      // tile variant of the step kernel
  int tile_adj;  // tile variant of the adjoint kernel
  int red_blocks;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int32_t max_steps = 0;
  double *S0 = nullptr, *S1 = nullptr, *L0 = nullptr, *L1 = nullptr, *Z = nullptr, *Z2 = nullptr;
  int32_t *codes = nullptr, *codes2 = nullptr;
  double* partial = nullptr;
  double* rowmean = nullptr;  // [B][ny] horizontal density means
  uint64_t* acc = nullptr;  // [3][B][kAccRow] signal-speed slots of the march, then [B] for rt_step
  Ctl* ctl = nullptr;       // [2][B] march control, double buffered
  long last_launch = 0;     // launches of the last march (final ctl in ctl[last_launch & 1])
  // Graph of a chunk of kGraphChunk march steps (captured once per set of
  // kernel arguments, replayed on the caller's stream).
  bool use_graphs = true;
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t chunk_exec = nullptr;
  const double* chunk_pool = nullptr;
  int chunk_interval = 0, chunk_slots = 0, chunk_tile = -1;
  // Second stream of the reverse sweep: re-computes the next segment's
  // states while the adjoint of the current one runs (default priority).
  hipStream_t aux_stream = nullptr;
  hipEvent_t seg_ready[2] = {nullptr, nullptr}, seg_free[2] = {nullptr, nullptr}, aux_done = nullptr;
  // Streams of member groups 2.. of the split binomial sweep (group 0 runs
  // on the context's stream, group 1 on aux_stream; entries 0 and 1 stay
  // null) and the events that stagger and join the groups.
  hipStream_t group_stream[kMaxGroups] = {};
  hipEvent_t group_ev[kMaxGroups] = {};
  bool overlap = true;
  // Reverse sweep with the limiter gather folded into the next step's kernel
  // (one kernel per step) or as its own kernel (two per step).
  bool fold = true;
  // Step sizes in the gradient: held at the forward run's values
  // (RT_DT_FROZEN) or differentiated (RT_DT_DIFFERENTIATED).
  int dt_mode = RT_DT_FROZEN;
  double *dtd_mu = nullptr, *dtd_smax = nullptr, *dtd_mu_last = nullptr;
  int32_t* dtd_imax = nullptr;
  int32_t dtd_stride = 0;
  double* bg_p = nullptr;  // [ny] background pressure rows of the well-balanced variant
  // the last binomial-checkpointing gradient: two-level plan, level-1 interval
  bool rev_last_two_level = false;
  int rev_last_interval = 0;
  ~rt_ctx() {
    if (chunk_exec) (void)hipGraphExecDestroy(chunk_exec);
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    for (hipEvent_t e : {seg_ready[0], seg_ready[1], seg_free[0], seg_free[1], aux_done})
      if (e) (void)hipEventDestroy(e);
    for (int k = 0; k < kMaxGroups; ++k) {
      if (group_ev[k]) (void)hipEventDestroy(group_ev[k]);
      if (group_stream[k]) (void)hipStreamDestroy(group_stream[k]);
    }
    if (aux_stream) (void)hipStreamDestroy(aux_stream);
  }
  Flags* flags = nullptr;
  double* dt_log = nullptr;
  int32_t* nsteps = nullptr;
  double* scal = nullptr;  // [8][B]: 0 max speed, 1 ke0, 2 keN, 3 dt, 4 norm, 5 dot, 6-7 rt_ke_ratio
  size_t cells() const { return (size_t)P.nx * P.ny; }
  size_t state_elems() const { return 4 * cells() * P.nb; }
  double* sc(int k) const { return scal + (size_t)k * P.nb; }
};

namespace {

struct Layout {
  size_t S0, S1, L0, L1, Z, Z2, codes, codes2, partial, rowmean, acc, ctl, flags, dt_log, nsteps, scal;
  size_t dtd_mu, dtd_smax, dtd_imax, dtd_mu_last, bg_p, total;
  int32_t dtd_stride;
};

Layout layout(const rt_ctx* c, int32_t max_steps) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  const size_t se = c->state_elems() * sizeof(double);
  int maxblk = c->red_blocks;
  for (int t = 0; t < rtk::TILE_COUNT; ++t) maxblk = std::max(maxblk, rtk::step_blocks(c->P, t));
  L.S0 = take(se);
  L.S1 = take(se);
  L.L0 = take(se);
  L.L1 = take(se);
  L.Z = take(3 * se);
  L.Z2 = take(3 * se);
  L.codes = take(c->cells() * c->P.nb * sizeof(int32_t));
  L.codes2 = take(c->cells() * c->P.nb * sizeof(int32_t));
  L.partial = take((size_t)maxblk * c->P.nb * sizeof(double));
  L.rowmean = take((size_t)c->P.ny * c->P.nb * sizeof(double));
  L.acc = take(((size_t)3 * rtk::kAccRow + 1) * c->P.nb * sizeof(uint64_t));
  L.ctl = take((size_t)2 * c->P.nb * sizeof(Ctl));
  L.flags = take(sizeof(Flags));
  L.dt_log = take((size_t)c->P.nb * std::max<int32_t>(max_steps, 1) * sizeof(double));
  L.nsteps = take((size_t)c->P.nb * sizeof(int32_t));
  L.scal = take((size_t)8 * c->P.nb * sizeof(double));
  // per-block partials of the step-size derivative, for any adjoint tile
  int adjblk = 1;
  for (int t = 0; t < rtk::TILE_COUNT; ++t) adjblk = std::max(adjblk, rtk::step_blocks(c->P, t));
  L.dtd_stride = adjblk;
  L.dtd_mu = take((size_t)adjblk * c->P.nb * sizeof(double));
  L.dtd_smax = take((size_t)adjblk * c->P.nb * sizeof(double));
  L.dtd_imax = take((size_t)adjblk * c->P.nb * sizeof(int32_t));
  L.dtd_mu_last = take((size_t)c->P.nb * sizeof(double));
  L.bg_p = take((size_t)c->P.ny * sizeof(double));
  L.total = off;
  return L;
}

// The row pressures of the well-balanced background, or null (closed form).
const double* background_rows(const rt_ctx* c) {
  return c->P.recon == RT_RECON_BALANCED ? c->bg_p : nullptr;
}

int need_ws(const rt_ctx* c) {
  if (!c) return fail(RT_EINVAL, "null context");
  if (!c->ws) return fail(RT_ESTATE, "no workspace set (call rt_set_workspace)");
  return 0;
}

// Read the device flags (synchronising) and turn them into a status.
int read_flags(rt_ctx* c, Flags* host, bool clear) {
  RT_HIP(hipMemcpyAsync(host, c->flags, sizeof(Flags), hipMemcpyDeviceToHost, c->stream));
  RT_HIP(hipStreamSynchronize(c->stream));
  if (clear && (host->err_unphys || host->err_overflow)) {
    RT_HIP(rtk::launch_fill_i32(reinterpret_cast<int32_t*>(c->flags), 0, 2, c->stream));
  }
  if (clear && host->snap_overflow) RT_HIP(rtk::launch_fill_i32(&c->flags->snap_overflow, 0, 1, c->stream));
  return 0;
}

int flags_status(const Flags& f) {
  if (f.err_unphys) return fail(RT_EUNPHYS, "unphysical state (rho <= 0, p <= 0 or non-finite)");
  if (f.err_overflow) return fail(RT_ENOMEM, "step log or checkpoint pool overflow");
  return 0;
}

rtk::StepArgs adaptive_args(rt_ctx* c, const double* src, double* dst, long launch, double* pool, int interval,
                            int slots) {
  rtk::StepArgs a{};
  a.U = src;
  a.Un = dst;
  a.ctl = c->ctl;
  a.acc = c->acc;
  a.launch = (int32_t)launch;
  a.dt_log = c->dt_log;
  a.dt_log_cap = c->max_steps;
  a.pool = pool;
  a.snap_interval = interval > 0 ? interval : 1;
  a.snap_slots = slots;
  a.flags = c->flags;
  return a;
}

// Control records after the last march.
const Ctl* final_ctl(const rt_ctx* c) { return c->ctl + (size_t)(c->last_launch & 1) * c->P.nb; }

// Level-1 snapshots of the binomial checkpointing cover this multiple of the
// step count the initial CFL step suggests.
constexpr double kRevolveMargin = 1.25;

// Steps per captured graph: a multiple of 6 so that the launch index enters
// the kernels only through L mod 2 and L mod 3.
constexpr long kGraphChunk = 48;

// (Re)capture the graph of kGraphChunk adaptive steps starting at an even
// launch index (S0 -> S1 -> S0 ...).
int ensure_chunk_graph(rt_ctx* c, double* pool, int interval, int slots) {
  if (c->chunk_exec && c->chunk_pool == pool && c->chunk_interval == interval && c->chunk_slots == slots &&
      c->chunk_tile == c->tile)
    return 0;
  if (c->chunk_exec) {
    RT_HIP(hipGraphExecDestroy(c->chunk_exec));
    c->chunk_exec = nullptr;
  }
  if (!c->capture_stream) RT_HIP(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  RT_HIP(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (long k = 0; k < kGraphChunk && e == hipSuccess; ++k) {
    const double* src = (k & 1) ? c->S1 : c->S0;
    double* dst = (k & 1) ? c->S0 : c->S1;
    rtk::StepArgs a = adaptive_args(c, src, dst, k, pool, interval, slots);
    e = rtk::launch_step(c->P, c->tile, a, c->capture_stream);
  }
  const hipError_t e2 = hipStreamEndCapture(c->capture_stream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(RT_EHIP, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  }
  e = hipGraphInstantiate(&c->chunk_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->chunk_exec = nullptr;
    return fail(RT_EHIP, "graph instantiate failed: %s", hipGetErrorString(e));
  }
  c->chunk_pool = pool;
  c->chunk_interval = interval;
  c->chunk_slots = slots;
  c->chunk_tile = c->tile;
  return 0;
}

// Adaptive march of all members from S0 to T, one launch per step for the
// whole batch (captured in graphs of kGraphChunk steps).  Members that are
// done skip their blocks; the host checks the number of active members once
// per round of launches.  On return (stream synced) final_ctl(c) holds the
// per-member step counts; the final state of member b is in S0 if its step
// count is even, else in S1.  Snapshots of U^n go to `pool` every `interval`
// steps when pool is not null.
int march(rt_ctx* c, double T, double* pool, int interval, int slots) {
  Params& P = c->P;
  RT_HIP(rtk::launch_reduce(P, 0, c->S0, nullptr, c->partial, c->red_blocks, c->sc(0), c->stream));
  RT_HIP(rtk::launch_march_begin(P, c->sc(0), T, c->ctl, c->acc, c->flags, c->stream));
  std::vector<double> ms(P.nb);
  RT_HIP(hipMemcpyAsync(ms.data(), c->sc(0), sizeof(double) * P.nb, hipMemcpyDeviceToHost, c->stream));
  RT_HIP(hipStreamSynchronize(c->stream));
  double msmax = 0.0;
  for (double m : ms) msmax = std::max(msmax, m);
  const double dtmin = P.cfl / msmax;
  if (!(dtmin > 0.0) || !std::isfinite(dtmin)) return fail(RT_EUNPHYS, "initial CFL step is %g", dtmin);
  const double est = std::ceil(T / dtmin);
  const long nest = est > 1e9 ? 1000000000L : (long)est;
  const bool graphs = c->use_graphs;
  if (graphs) {
    if (int rc = ensure_chunk_graph(c, pool, interval, slots)) return rc;
  }
  long launched = 0;
  // the first round stops where the step log would overflow, so that a T
  // beyond max_steps is refused after at most one round past the limit
  long target = std::min<long>(nest, (long)c->max_steps + kGraphChunk + 2);
  Flags f{};
  for (;;) {
    while (launched < target) {
      if (graphs) {
        RT_HIP(hipGraphLaunch(c->chunk_exec, c->stream));
        launched += kGraphChunk;
        continue;
      }
      const double* src = (launched & 1) ? c->S1 : c->S0;
      double* dst = (launched & 1) ? c->S0 : c->S1;
      rtk::StepArgs a = adaptive_args(c, src, dst, launched, pool, interval, slots);
      RT_HIP(rtk::launch_step(P, c->tile, a, c->stream));
      ++launched;
    }
    c->last_launch = launched;
    if (int rc = read_flags(c, &f, false)) return rc;
    if (f.n_active == 0 || f.err_unphys || f.err_overflow) break;
    if (launched > (long)c->max_steps + kGraphChunk + 2) {
      return fail(RT_ENOMEM, "march needs more than %d steps (workspace max_steps)", c->max_steps);
    }
    target = launched + std::max<long>(8, nest / 32);
  }
  return 0;
}

}  // namespace

extern "C" {

const char* rt_last_error(void) { return g_err.c_str(); }

int rt_create(const rt_grid* grid, const rt_phys* phys, void* stream, rt_ctx** out) {
  if (!grid || !phys || !out) return fail(RT_EINVAL, "null argument");
  if (grid->nx < 3 || grid->ny < 2 || grid->batch < 1) return fail(RT_EINVAL, "grid must be at least 3 x 2 with batch >= 1");
  // the kernels address a plane of a state with 32-bit byte offsets
  if ((size_t)grid->nx * grid->ny >= (size_t)1 << 28) return fail(RT_EINVAL, "grid too large (nx * ny >= 2^28)");
  if (!(grid->lx > 0) || !(grid->ly > 0)) return fail(RT_EINVAL, "domain lengths must be positive");
  if (!(phys->gamma > 1.0) || !(phys->h > 0) || !(phys->cfl > 0) || !(phys->rho_h > 0) || !(phys->rho_l > 0))
    return fail(RT_EINVAL, "need gamma > 1, h > 0, cfl > 0, positive densities");
  if (phys->comp_mask < 1 || phys->comp_mask > 3) return fail(RT_EINVAL, "comp_mask must be 1, 2 or 3");
  if (phys->recon != RT_RECON_PRIMITIVE && phys->recon != RT_RECON_BALANCED)
    return fail(RT_EINVAL, "recon must be RT_RECON_PRIMITIVE or RT_RECON_BALANCED");
  rt_ctx* c = new rt_ctx();
  Params& P = c->P;
  P.nx = grid->nx;
  P.ny = grid->ny;
  P.nb = grid->batch;
  P.comp_mask = phys->comp_mask;
  P.recon = phys->recon;
  P.dx = grid->lx / grid->nx;
  P.dy = grid->ly / grid->ny;
  P.inv_dx = 1.0 / P.dx;
  P.inv_dy = 1.0 / P.dy;
  P.gamma = phys->gamma;
  P.gm1 = phys->gamma - 1.0;
  P.inv_gm1 = 1.0 / P.gm1;
  P.g_y = phys->g_y;
  P.cfl = phys->cfl;
  P.rho_h = phys->rho_h;
  P.rho_l = phys->rho_l;
  P.y0 = phys->y0;
  P.h = phys->h;
  P.p_int = phys->p_int;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  // Defaults from measurements on MI355X.  Tiny grids (one partial round of
  // blocks) are bound by one block's critical path: single-pass 8x8 tiles
  // and the folded adjoint (one kernel per step) win.  From 2^16 cells on
  // the adjoint runs two kernels.  While 32x8 tiles fill at most one round
  // of three blocks per CU, each launch lasts about one block's critical
  // path: the step takes 32x16 tiles of 512 threads (the least halo work
  // per cell) and the adjoint 32x8 tiles.  Beyond that both take 16x15 tiles
  // of 256 threads: every face loop is one pass of the block (255 and 256
  // faces of each direction; the step's single face list two), and four
  // small blocks per CU hide one another's barriers better than two large
  // ones.  rt_autotune measures instead.
  const size_t all_cells = (size_t)P.nx * P.ny * P.nb;
  const bool tiny = all_cells < ((size_t)1 << 16);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  const bool one_round = all_cells <= (size_t)3 * cus * 256;
  c->tile = tiny ? rtk::TILE_8x8W : (one_round ? rtk::TILE_32x16 : rtk::TILE_16x15);
  c->tile_adj = tiny ? rtk::TILE_8x8W : (one_round ? rtk::TILE_32x8 : rtk::TILE_16x15);
  c->fold = tiny;
  const size_t n = c->cells();
  c->red_blocks = (int)std::min<size_t>(256, std::max<size_t>(1, n / 2048));
  *out = c;
  return 0;
}

int rt_destroy(rt_ctx* c) {
  delete c;
  return 0;
}

int rt_set_stream(rt_ctx* c, void* stream) {
  if (!c) return fail(RT_EINVAL, "null context");
  c->stream = reinterpret_cast<hipStream_t>(stream);
  return 0;
}

// Internal tuning hook: choose the tile shape of the step / adjoint kernels.
int rt_set_tile(rt_ctx* c, int32_t tile) {
  if (!c || tile < 0 || tile >= rtk::TILE_COUNT) return fail(RT_EINVAL, "bad tile id");
  c->tile = tile;
  c->tile_adj = tile;
  return 0;
}

int rt_set_tiles(rt_ctx* c, int32_t step_tile, int32_t adj_tile) {
  if (!c || step_tile < 0 || step_tile >= rtk::TILE_COUNT || adj_tile < 0 || adj_tile >= rtk::TILE_COUNT)
    return fail(RT_EINVAL, "bad tile id");
  c->tile = step_tile;
  c->tile_adj = adj_tile;
  return 0;
}

int rt_get_tile(const rt_ctx* c, int32_t* tile) {
  if (!c || !tile) return fail(RT_EINVAL, "null argument");
  *tile = c->tile;
  return 0;
}

// Replay the march in captured graphs (1, default) or launch step by step (0).
int rt_set_graphs(rt_ctx* c, int32_t on) {
  if (!c) return fail(RT_EINVAL, "null context");
  c->use_graphs = on != 0;
  return 0;
}

int rt_set_overlap(rt_ctx* c, int32_t on) {
  if (!c) return fail(RT_EINVAL, "null context");
  c->overlap = on != 0;
  return 0;
}

int rt_set_fold(rt_ctx* c, int32_t on) {
  if (!c) return fail(RT_EINVAL, "null context");
  c->fold = on != 0;
  return 0;
}

int rt_get_fold(const rt_ctx* c, int32_t* on) {
  if (!c || !on) return fail(RT_EINVAL, "null argument");
  *on = c->fold ? 1 : 0;
  return 0;
}

int rt_set_dt_mode(rt_ctx* c, int32_t mode) {
  if (!c) return fail(RT_EINVAL, "null context");
  if (mode != RT_DT_FROZEN && mode != RT_DT_DIFFERENTIATED) return fail(RT_EINVAL, "unknown dt mode %d", mode);
  c->dt_mode = mode;
  return 0;
}

int rt_get_dt_mode(const rt_ctx* c, int32_t* mode) {
  if (!c || !mode) return fail(RT_EINVAL, "null argument");
  *mode = c->dt_mode;
  return 0;
}

int rt_get_tiles(const rt_ctx* c, int32_t* step_tile, int32_t* adj_tile) {
  if (!c || !step_tile || !adj_tile) return fail(RT_EINVAL, "null argument");
  *step_tile = c->tile;
  *adj_tile = c->tile_adj;
  return 0;
}

namespace {
// The second stream and its events, created on first use on the current
// device.
int ensure_aux(rt_ctx* c) {
  if (c->aux_stream) return 0;
  RT_HIP(hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking));
  for (hipEvent_t* e : {&c->seg_ready[0], &c->seg_ready[1], &c->seg_free[0], &c->seg_free[1], &c->aux_done})
    RT_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
  return 0;
}

// Streams and events of member groups 0 .. ng-1 of the split sweep (group 0
// runs on the context's stream, group 1 on aux_stream), created on first use
// on the current device, default priority.
int ensure_groups(rt_ctx* c, int ng) {
  if (int rc = ensure_aux(c)) return rc;
  for (int k = 0; k < ng; ++k) {
    if (k >= 2 && !c->group_stream[k]) RT_HIP(hipStreamCreateWithFlags(&c->group_stream[k], hipStreamNonBlocking));
    if (!c->group_ev[k]) RT_HIP(hipEventCreateWithFlags(&c->group_ev[k], hipEventDisableTiming));
  }
  return 0;
}
}  // namespace

namespace {

// Per-launch times (ms) of the kernels as the library launches them: [0] the
// given-dt step (re-computation), [1] the adaptive step with its CFL
// epilogue (march; never reaches its end time here), [2] one adjoint step
// of the folded sweep (kernel A forming lambda^{n+1} from the previous
// step's outputs), [3] the unfolded adjoint step (kernels A + B).  The
// state U serves as every step's state; the workspace buffers are scratch.
int time_kernels(rt_ctx* c, const double* U, int step_tile, int adj_tile, int reps, hipEvent_t e0, hipEvent_t e1,
                 float out[4]) {
  hipStream_t s = c->stream;
  const size_t se = c->state_elems();
  const Params& P = c->P;
  rtk::StepArgs a{};
  a.U = U;
  a.Un = c->S1;
  a.dt = c->sc(3);
  a.dt_stride = 1;
  a.flags = c->flags;
  rtk::AdjArgs j{};
  j.U = U;
  j.lam_next = c->L0;
  j.lam = c->L1;
  j.Z = c->Z;
  j.codes = c->codes;
  j.dt = c->sc(3);
  j.dt_stride = 1;
  j.flags = c->flags;
  auto timed = [&](auto&& body, float* ms) -> hipError_t {
    hipError_t e = hipEventRecord(e0, s);
    for (int k = 0; k < reps && e == hipSuccess; ++k) e = body(k);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e == hipSuccess) *ms /= (float)reps;
    return e;
  };
  hipError_t e = rtk::launch_step(P, step_tile, a, s);
  if (e == hipSuccess) e = rtk::launch_adjoint(P, adj_tile, j, s, false);  // fills Z, codes for the fold
  if (e == hipSuccess) e = timed([&](int) { return rtk::launch_step(P, step_tile, a, s); }, &out[0]);
  if (e == hipSuccess) e = rtk::launch_copy(U, c->S0, se, s);
  if (e == hipSuccess) e = rtk::launch_reduce(P, 0, c->S0, nullptr, c->partial, c->red_blocks, c->sc(0), s);
  if (e == hipSuccess) e = rtk::launch_march_begin(P, c->sc(0), 1e300, c->ctl, c->acc, c->flags, s);
  if (e == hipSuccess)
    e = timed(
        [&](int k) {
          rtk::StepArgs m = adaptive_args(c, (k & 1) ? c->S1 : c->S0, (k & 1) ? c->S0 : c->S1, k, nullptr, 1, 0);
          m.dt_log = nullptr;
          return rtk::launch_step(P, step_tile, m, s);
        },
        &out[1]);
  // the well-balanced variant has no folded form: out[2] repeats out[3]
  const bool can_fold = P.recon == RT_RECON_PRIMITIVE;
  if (e == hipSuccess && can_fold)
    e = hipMemcpyAsync(c->Z2, c->Z, 3 * se * sizeof(double), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && can_fold)
    e = hipMemcpyAsync(c->codes2, c->codes, c->cells() * P.nb * sizeof(int32_t), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && can_fold)
    e = timed(
        [&](int k) {
          rtk::AdjArgs f = j;
          f.Z = (k & 1) ? c->Z : c->Z2;
          f.codes = (k & 1) ? c->codes : c->codes2;
          f.fold.Z = (k & 1) ? c->Z2 : c->Z;
          f.fold.codes = (k & 1) ? c->codes2 : c->codes;
          f.fold.U = U;
          f.fold.lam_next = c->L0;
          f.fold.lam_out = c->L1;
          f.fold.dt_index = 0;
          return rtk::launch_adjoint(P, adj_tile, f, s, false);
        },
        &out[2]);
  if (e == hipSuccess) e = timed([&](int) { return rtk::launch_adjoint(P, adj_tile, j, s); }, &out[3]);
  if (!can_fold) out[2] = out[3];
  return e == hipSuccess ? 0 : fail(RT_EHIP, "kernel timing: %s", hipGetErrorString(e));
}

}  // namespace

// Autotuner: times every tile variant of the step kernel (given-dt plus
// adaptive launches) and of the adjoint step (folded and two-kernel) on the
// caller's state U (device, [B][4][ny][nx]) with HIP events on the context's
// stream and keeps the fastest step variant and the fastest adjoint variant
// of the chosen form.  All variants give bitwise-identical results, so this
// changes speed only.  Uses the workspace buffers as scratch.  Synchronises
// the stream.
int rt_autotune(rt_ctx* c, const double* U, int32_t reps, int32_t* step_tile, int32_t* adj_tile) {
  if (int rc = need_ws(c)) return rc;
  if (!U || reps < 1) return fail(RT_EINVAL, "bad argument");
  if (int rc = rt_cfl_dt(c, U, c->sc(3))) return rc;
  RT_HIP(rtk::launch_copy(U, c->L0, c->state_elems(), c->stream));  // any finite cotangent will do
  hipEvent_t e0, e1;
  RT_HIP(hipEventCreate(&e0));
  RT_HIP(hipEventCreate(&e1));
  float best_s = 1e30f, best_f = 1e30f, best_u = 1e30f;
  int bs = c->tile, bfold = c->tile_adj, bunf = c->tile_adj;
  int rc = 0;
  for (int t = 0; t < rtk::TILE_COUNT && rc == 0; ++t) {
    float ms[4];
    rc = time_kernels(c, U, t, t, reps, e0, e1, ms);
    if (rc) break;
    if (ms[0] + ms[1] < best_s) { best_s = ms[0] + ms[1]; bs = t; }
    if (ms[2] < best_f) { best_f = ms[2]; bfold = t; }
    if (ms[3] < best_u) { best_u = ms[3]; bunf = t; }
  }
  // Folded or two-kernel adjoint.  In the two-stream sweep the folded
  // kernel (more LDS, no LDS-free gather kernel between adjoint launches)
  // leaves less room on the CUs for the concurrent re-computation, which
  // costs it about 10% there relative to its time alone; so it is taken
  // only when it is more than 10% faster alone.
  const bool fold = c->P.recon == RT_RECON_PRIMITIVE && best_f < 0.9f * best_u;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  RT_HIP(hipGetLastError());
  const int ba = fold ? bfold : bunf;
  c->tile = bs;
  c->tile_adj = ba;
  c->fold = fold;
  if (step_tile) *step_tile = bs;
  if (adj_tile) *adj_tile = ba;
  Flags f{};
  return read_flags(c, &f, true);
}

// Per-launch times (microseconds) of the current variants, as in
// time_kernels: out[0] given-dt step, [1] adaptive step, [2] folded adjoint
// step (one kernel), [3] unfolded adjoint step (two kernels), [4] the
// adjoint step of the reverse sweep's current mode.
int rt_kernel_times(rt_ctx* c, const double* U, int32_t reps, double* out) {
  if (int rc = need_ws(c)) return rc;
  if (!U || reps < 1 || !out) return fail(RT_EINVAL, "bad argument");
  if (int rc = rt_cfl_dt(c, U, c->sc(3))) return rc;
  RT_HIP(rtk::launch_copy(U, c->L0, c->state_elems(), c->stream));
  hipEvent_t e0, e1;
  RT_HIP(hipEventCreate(&e0));
  RT_HIP(hipEventCreate(&e1));
  float ms[4] = {0, 0, 0, 0};
  const int rc = time_kernels(c, U, c->tile, c->tile_adj, reps, e0, e1, ms);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  for (int k = 0; k < 4; ++k) out[k] = 1e3 * ms[k];
  out[4] = (c->fold && c->dt_mode == RT_DT_FROZEN && c->P.recon == RT_RECON_PRIMITIVE) ? out[2] : out[3];
  Flags f{};
  return read_flags(c, &f, true);
}

int rt_workspace_bytes(const rt_ctx* c, int32_t max_steps, size_t* bytes) {
  if (!c || !bytes || max_steps < 1) return fail(RT_EINVAL, "bad argument");
  *bytes = layout(c, max_steps).total;
  return 0;
}

int rt_set_workspace(rt_ctx* c, void* dev, size_t bytes, int32_t max_steps) {
  if (!c || !dev || max_steps < 1) return fail(RT_EINVAL, "bad argument");
  if (reinterpret_cast<uintptr_t>(dev) & 255) return fail(RT_EINVAL, "workspace must be 256-byte aligned");
  const Layout L = layout(c, max_steps);
  if (bytes < L.total) return fail(RT_ENOMEM, "workspace of %zu bytes < %zu needed", bytes, L.total);
  char* w = static_cast<char*>(dev);
  if (c->chunk_exec) {
    RT_HIP(hipGraphExecDestroy(c->chunk_exec));
    c->chunk_exec = nullptr;
  }
  c->ws = w;
  c->ws_bytes = bytes;
  c->max_steps = max_steps;
  c->S0 = reinterpret_cast<double*>(w + L.S0);
  c->S1 = reinterpret_cast<double*>(w + L.S1);
  c->L0 = reinterpret_cast<double*>(w + L.L0);
  c->L1 = reinterpret_cast<double*>(w + L.L1);
  c->Z = reinterpret_cast<double*>(w + L.Z);
  c->Z2 = reinterpret_cast<double*>(w + L.Z2);
  c->codes = reinterpret_cast<int32_t*>(w + L.codes);
  c->codes2 = reinterpret_cast<int32_t*>(w + L.codes2);
  c->partial = reinterpret_cast<double*>(w + L.partial);
  c->rowmean = reinterpret_cast<double*>(w + L.rowmean);
  c->acc = reinterpret_cast<uint64_t*>(w + L.acc);
  c->ctl = reinterpret_cast<Ctl*>(w + L.ctl);
  c->flags = reinterpret_cast<Flags*>(w + L.flags);
  c->dt_log = reinterpret_cast<double*>(w + L.dt_log);
  c->nsteps = reinterpret_cast<int32_t*>(w + L.nsteps);
  c->scal = reinterpret_cast<double*>(w + L.scal);
  c->dtd_mu = reinterpret_cast<double*>(w + L.dtd_mu);
  c->dtd_smax = reinterpret_cast<double*>(w + L.dtd_smax);
  c->dtd_imax = reinterpret_cast<int32_t*>(w + L.dtd_imax);
  c->dtd_mu_last = reinterpret_cast<double*>(w + L.dtd_mu_last);
  c->dtd_stride = L.dtd_stride;
  c->bg_p = reinterpret_cast<double*>(w + L.bg_p);
  if (c->P.recon == RT_RECON_BALANCED) RT_HIP(rtk::launch_background_rows(c->P, c->bg_p, c->stream));
  RT_HIP(rtk::launch_fill_i32(reinterpret_cast<int32_t*>(c->acc), 0, 2 * ((size_t)3 * rtk::kAccRow + 1) * c->P.nb,
                              c->stream));
  RT_HIP(rtk::launch_fill_i32(reinterpret_cast<int32_t*>(c->flags), 0, sizeof(Flags) / 4, c->stream));
  return 0;
}

int rt_init_state(rt_ctx* c, const double* uv0, double* U) {
  if (!c || !uv0 || !U) return fail(RT_EINVAL, "null argument");
  RT_HIP(rtk::launch_init_state(c->P, uv0, U, background_rows(c), c->stream));
  return 0;
}

int rt_cfl_dt(rt_ctx* c, const double* U, double* dt) {
  if (int rc = need_ws(c)) return rc;
  if (!U || !dt) return fail(RT_EINVAL, "null argument");
  RT_HIP(rtk::launch_reduce(c->P, 0, U, nullptr, c->partial, c->red_blocks, c->sc(0), c->stream));
  RT_HIP(rtk::launch_cfl_from_speed(c->P, c->sc(0), dt, c->stream));
  return 0;
}

int rt_step(rt_ctx* c, const double* U_in, double* U_out, const double* dt, double* dt_next) {
  if (int rc = need_ws(c)) return rc;
  if (!U_in || !U_out || U_in == U_out) return fail(RT_EINVAL, "need distinct non-null U_in, U_out");
  if (!dt) {
    if (int rc = rt_cfl_dt(c, U_in, c->sc(3))) return rc;
    dt = c->sc(3);
  }
  rtk::StepArgs a{};
  a.U = U_in;
  a.Un = U_out;
  a.dt = dt;
  a.dt_stride = 1;
  a.dt_index = 0;
  a.flags = c->flags;
  uint64_t* acc_out = c->acc + 3 * (size_t)rtk::kAccRow * c->P.nb;  // after the march's rows
  if (dt_next) {
    RT_HIP(rtk::launch_fill_i32(reinterpret_cast<int32_t*>(acc_out), 0, 2 * c->P.nb, c->stream));
    a.acc_out = acc_out;
  }
  RT_HIP(rtk::launch_step(c->P, c->tile, a, c->stream));
  if (dt_next) RT_HIP(rtk::launch_cfl_from_bits(c->P, acc_out, dt_next, c->stream));
  return 0;
}

int rt_integrate(rt_ctx* c, double* U, double T, double* t_out, int32_t* nsteps, double* dt_log, int32_t cap) {
  if (int rc = need_ws(c)) return rc;
  if (!U || !(T > 0) || !std::isfinite(T)) return fail(RT_EINVAL, "need U and 0 < T < inf");
  if (dt_log && cap < 1) return fail(RT_EINVAL, "dt_log needs cap >= 1");
  RT_HIP(rtk::launch_copy(U, c->S0, c->state_elems(), c->stream));
  if (int rc = march(c, T, nullptr, 1, 0)) return rc;
  RT_HIP(rtk::launch_copy_final(c->P, final_ctl(c), c->S0, c->S1, U, t_out, nsteps, c->dt_log, c->max_steps, dt_log,
                                cap, c->stream));
  Flags f{};
  if (int rc = read_flags(c, &f, true)) return rc;
  if (int rc = flags_status(f)) return rc;
  if (dt_log) {
    std::vector<Ctl> h(c->P.nb);
    RT_HIP(hipMemcpyAsync(h.data(), final_ctl(c), sizeof(Ctl) * c->P.nb, hipMemcpyDeviceToHost, c->stream));
    RT_HIP(hipStreamSynchronize(c->stream));
    for (const Ctl& x : h)
      if (x.nsteps > cap) return fail(RT_ENOMEM, "dt_log capacity %d < %d steps", cap, x.nsteps);
  }
  return 0;
}

int rt_kinetic_energy(rt_ctx* c, const double* U, double* ke) {
  if (int rc = need_ws(c)) return rc;
  if (!U || !ke) return fail(RT_EINVAL, "null argument");
  RT_HIP(rtk::launch_reduce(c->P, 1, U, nullptr, c->partial, c->red_blocks, ke, c->stream));
  return 0;
}

int rt_ke_ratio(rt_ctx* c, const double* U0, const double* UT, double* R) {
  if (int rc = need_ws(c)) return rc;
  if (!U0 || !UT || !R) return fail(RT_EINVAL, "null argument");
  RT_HIP(rtk::launch_reduce(c->P, 1, U0, nullptr, c->partial, c->red_blocks, c->sc(6), c->stream));
  RT_HIP(rtk::launch_reduce(c->P, 1, UT, nullptr, c->partial, c->red_blocks, c->sc(7), c->stream));
  RT_HIP(rtk::launch_ratio(c->P.nb, c->sc(7), c->sc(6), R, c->stream));
  return 0;
}

namespace {
// Scratch of rt_ke_ratio_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code reaches it only through the
// device address hipGetSymbolAddress returns (the array's name is a host-side
// stand-in, not a device address), taken once per device on that entry
// point's first call there.
constexpr size_t kNoAllocScratchDoubles = 65536;  // 512 KiB
__device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, or null (with the
// error recorded) if it cannot be had.
double* scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    fail(RT_EHIP, "no current HIP device (or device id beyond %d)", kMaxDevices - 1);
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      fail(RT_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

int rt_ke_ratio_noalloc(rt_ctx* c, const double* U0, const double* UT, double* R) {
  if (!c) return fail(RT_EINVAL, "null context");
  if (!U0 || !UT || !R) return fail(RT_EINVAL, "null argument");
  // partials of the two reductions (red_blocks per member, reused) and the
  // two kinetic energies of every member
  const size_t need = (size_t)c->red_blocks * c->P.nb + 2 * (size_t)c->P.nb;
  if (need > kNoAllocScratchDoubles)
    return fail(RT_ENOMEM, "rt_ke_ratio_noalloc: batch %d needs %zu doubles of scratch, the static array holds %zu "
                "(at most %zu members)", c->P.nb, need, kNoAllocScratchDoubles,
                kNoAllocScratchDoubles / ((size_t)c->red_blocks + 2));
  double* sp = scratch_on_current_device();
  if (!sp) return RT_EHIP;
  double* partial = sp;
  double* ke0 = sp + (size_t)c->red_blocks * c->P.nb;
  double* keT = ke0 + c->P.nb;
  // every partial and both energies are written before they are read:
  // nothing has to start at zero
  RT_HIP(rtk::launch_reduce(c->P, 1, U0, nullptr, partial, c->red_blocks, ke0, c->stream));
  RT_HIP(rtk::launch_reduce(c->P, 1, UT, nullptr, partial, c->red_blocks, keT, c->stream));
  RT_HIP(rtk::launch_ratio(c->P.nb, keT, ke0, R, c->stream));
  return 0;
}

int rt_step_adjoint(rt_ctx* c, const double* U, const double* dt, const double* lam_next, double* lam) {
  if (int rc = need_ws(c)) return rc;
  if (!U || !dt || !lam_next || !lam || lam == lam_next) return fail(RT_EINVAL, "bad argument");
  rtk::AdjArgs a{};
  a.U = U;
  a.lam_next = lam_next;
  a.lam = lam;
  a.Z = c->Z;
  a.codes = c->codes;
  a.dt = dt;
  a.dt_stride = 1;
  a.dt_index = 0;
  a.flags = c->flags;
  RT_HIP(rtk::launch_adjoint(c->P, c->tile_adj, a, c->stream));
  return 0;
}

int rt_pool_bytes(const rt_ctx* c, int32_t kind, int32_t interval, int32_t nsteps_max, size_t* bytes) {
  if (!c || !bytes || nsteps_max < 1) return fail(RT_EINVAL, "bad argument");
  const size_t se = c->state_elems() * sizeof(double);
  if (kind == RT_CKPT_STORE_ALL) {
    *bytes = se * (size_t)nsteps_max;
  } else if (kind == RT_CKPT_UNIFORM) {
    if (interval < 1) return fail(RT_EINVAL, "interval must be >= 1");
    *bytes = se * ((size_t)(nsteps_max + interval - 1) / interval + 2 * (size_t)(interval - 1));
  } else if (kind == RT_CKPT_REVOLVE) {
    *bytes = se * 2;
  } else {
    return fail(RT_EINVAL, "unknown checkpoint kind %d", kind);
  }
  return 0;
}


namespace {
// Forward march with checkpoints, then the reverse sweep, for the objective
// R = KE(T)/KE(0) (ek_base == nullptr) or J of Eq. 8 against the baseline
// field ek_base; the objective value goes to val[B].
int grad_objective(rt_ctx* c, const double* uv0, double T, const rt_ckpt_policy* pol, const double* ek_base,
                   double* R, double* grad, int32_t* nsteps_out) {
  if (int rc = need_ws(c)) return rc;
  if (!uv0 || !pol || !R || !grad || !(T > 0) || !std::isfinite(T)) return fail(RT_EINVAL, "bad argument");
  if (!pol->pool) return fail(RT_EINVAL, "checkpoint pool is null");
  Params& P = c->P;
  hipStream_t s = c->stream;
  const size_t se = c->state_elems();
  const size_t slots_total = pol->pool_bytes / (se * sizeof(double));
  double* pool = static_cast<double*>(pol->pool);
  auto state_slot = [&](size_t k) { return pool + k * se; };

  // forward: U^0, KE(U^0)
  RT_HIP(rtk::launch_init_state(P, uv0, c->S0, background_rows(c), s));
  RT_HIP(rtk::launch_reduce(P, 1, c->S0, nullptr, c->partial, c->red_blocks, c->sc(1), s));

  int interval = 1;
  size_t snap_slots = 0;
  int rev_slots = 0;
  if (pol->kind == RT_CKPT_STORE_ALL || pol->kind == RT_CKPT_UNIFORM) {
    interval = pol->kind == RT_CKPT_STORE_ALL ? 1 : pol->interval;
    if (interval < 1) return fail(RT_EINVAL, "interval must be >= 1");
    if (slots_total < (size_t)interval) return fail(RT_ENOMEM, "pool holds %zu states, need > %d", slots_total, interval - 1);
    snap_slots = slots_total - (interval - 1);
    if (int rc = march(c, T, pool, interval, (int)std::min<size_t>(snap_slots, 1u << 30))) return rc;
  } else if (pol->kind == RT_CKPT_REVOLVE) {
    if (slots_total < 2) return fail(RT_ENOMEM, "revolve needs a pool of at least 2 states");
    // The objective's forward march also leaves level-1 snapshots, every
    // `interval` steps, in slots 0 .. rev_slots - 2 (slot 0: U^0); the
    // interval comes from the step count the initial CFL step suggests.
    rev_slots = (int)std::min<size_t>(slots_total, 1u << 20);
    RT_HIP(rtk::launch_reduce(P, 0, c->S0, nullptr, c->partial, c->red_blocks, c->sc(0), s));
    std::vector<double> ms(P.nb);
    RT_HIP(hipMemcpyAsync(ms.data(), c->sc(0), sizeof(double) * P.nb, hipMemcpyDeviceToHost, s));
    RT_HIP(hipStreamSynchronize(s));
    const double msmax = *std::max_element(ms.begin(), ms.end());
    const double est = std::ceil(T * msmax / P.cfl);
    const int n_est = !(est < 1e8) ? 100000000 : std::max(1, (int)est);
    interval = rtrev::level1_interval(n_est, rev_slots, kRevolveMargin);
    if (int rc = march(c, T, pool, interval, std::max(1, rev_slots - 1))) return rc;
  } else {
    return fail(RT_EINVAL, "unknown checkpoint kind %d", pol->kind);
  }
  Flags f{};
  if (int rc = read_flags(c, &f, true)) return rc;
  if (int rc = flags_status(f)) return rc;
  // Level-1 snapshots beyond the pool: the uniform policies cannot go on;
  // revolve falls back to one binomial schedule over the whole march from
  // U^0 in slot 0 (the march it just ran then served to count the steps).
  const bool snaps_fit = !f.snap_overflow;
  if (!snaps_fit && pol->kind != RT_CKPT_REVOLVE)
    return fail(RT_ENOMEM, "checkpoint pool of %zu states overflowed", slots_total);

  // step counts and final state
  RT_HIP(rtk::launch_copy_final(P, final_ctl(c), c->S0, c->S1, c->L1, nullptr, c->nsteps, nullptr, 0, nullptr, 0, s));
  if (nsteps_out) RT_HIP(hipMemcpyAsync(nsteps_out, c->nsteps, sizeof(int32_t) * P.nb, hipMemcpyDeviceToDevice, s));
  std::vector<int32_t> hn(P.nb);
  std::vector<double> hke0(P.nb);
  RT_HIP(hipMemcpyAsync(hn.data(), c->nsteps, sizeof(int32_t) * P.nb, hipMemcpyDeviceToHost, s));
  RT_HIP(hipMemcpyAsync(hke0.data(), c->sc(1), sizeof(double) * P.nb, hipMemcpyDeviceToHost, s));
  RT_HIP(hipStreamSynchronize(s));
  if (!ek_base)
    for (double k : hke0)
      if (!(k > 0.0) || !std::isfinite(k)) return fail(RT_EINVAL, "KE(0) = %g: the perturbation is zero or not finite", k);
  const int nmax = *std::max_element(hn.begin(), hn.end());

  // terminal adjoint lambda^N into L0 (from U^N in L1)
  if (ek_base) {
    RT_HIP(rtk::launch_reduce(P, 7, c->L1, ek_base, c->partial, c->red_blocks, R, s));
    RT_HIP(rtk::launch_terminal_adjoint_ek(P, c->L1, ek_base, c->L0, s));
  } else {
    RT_HIP(rtk::launch_reduce(P, 1, c->L1, nullptr, c->partial, c->red_blocks, c->sc(2), s));
    RT_HIP(rtk::launch_terminal_adjoint(P, c->L1, c->sc(1), c->L0, s));
  }
  double* lam = c->L0;
  double* lam_other = c->L1;

  auto step_given = [&](const double* src, double* dst, int n, hipStream_t ss) -> int {
    rtk::StepArgs a{};
    a.U = src;
    a.Un = dst;
    a.dt = c->dt_log;
    a.dt_stride = c->max_steps;
    a.dt_index = n;
    a.nsteps_limit = c->nsteps;
    a.flags = c->flags;
    RT_HIP(rtk::launch_step(P, c->tile, a, ss));
    return 0;
  };
  const bool dtd = c->dt_mode == RT_DT_DIFFERENTIATED;
  // the folded sweep serves the frozen steps of the primitive variant
  const bool use_fold = c->fold && !dtd && P.recon == RT_RECON_PRIMITIVE;
  auto adjoint = [&](const double* Un, int n) -> int {
    rtk::AdjArgs a{};
    a.U = Un;
    a.lam_next = lam;
    a.lam = lam_other;
    a.Z = c->Z;
    a.codes = c->codes;
    a.dt = c->dt_log;
    a.dt_stride = c->max_steps;
    a.dt_index = n;
    a.nsteps_limit = c->nsteps;
    a.flags = c->flags;
    if (dtd) {
      a.dtd.mu = c->dtd_mu;
      a.dtd.smax = c->dtd_smax;
      a.dtd.imax = c->dtd_imax;
      a.dtd.stride = c->dtd_stride;
      a.dtd.count = rtk::step_blocks(P, c->tile_adj);
      a.dtd.mu_last = c->dtd_mu_last;
    }
    RT_HIP(rtk::launch_adjoint(P, c->tile_adj, a, s));
    if (dtd) RT_HIP(rtk::launch_dt_correct(P, a, s));  // updates lambda^n (a.lam) in place
    std::swap(lam, lam_other);
    return 0;
  };
  // Folded sweep: kernel A of step n also forms lambda^{n+1} from step
  // n+1's Z (the gather kernel is not launched), so one kernel per step.
  // Needs U^{n+1} to stay where the previous call found it, which holds for
  // the snapshot/segment sweep; kernel A of step n writes Z and codes into
  // the buffer pair that step n+1 does not read.
  struct Pending {
    int n = -1;
    const double* U = nullptr;
    int buf = 0;
  } pend;
  double* Zb[2] = {c->Z, c->Z2};
  int32_t* Cb[2] = {c->codes, c->codes2};
  auto adjoint_folded = [&](const double* Un, int n) -> int {
    rtk::AdjArgs a{};
    const int buf = pend.n < 0 ? 0 : pend.buf ^ 1;
    a.U = Un;
    a.Z = Zb[buf];
    a.codes = Cb[buf];
    a.dt = c->dt_log;
    a.dt_stride = c->max_steps;
    a.dt_index = n;
    a.nsteps_limit = c->nsteps;
    a.flags = c->flags;
    if (pend.n < 0) {
      a.lam_next = lam;  // lambda^{n+1} as it is
    } else {
      a.fold.Z = Zb[pend.buf];
      a.fold.codes = Cb[pend.buf];
      a.fold.U = pend.U;
      a.fold.lam_next = lam;
      a.fold.lam_out = lam_other;
      a.fold.dt_index = pend.n;
      std::swap(lam, lam_other);
    }
    RT_HIP(rtk::launch_adjoint(P, c->tile_adj, a, s, false));
    pend.n = n;
    pend.U = Un;
    pend.buf = buf;
    return 0;
  };
  auto finish_folded = [&]() -> int {
    if (pend.n < 0) return 0;
    rtk::AdjArgs a{};
    a.U = pend.U;
    a.lam_next = lam;
    a.lam = lam_other;
    a.Z = Zb[pend.buf];
    a.codes = Cb[pend.buf];
    a.dt = c->dt_log;
    a.dt_stride = c->max_steps;
    a.dt_index = pend.n;
    a.nsteps_limit = c->nsteps;
    a.flags = c->flags;
    RT_HIP(rtk::launch_adj_gather(P, a, s));
    std::swap(lam, lam_other);
    pend.n = -1;
    return 0;
  };

  if (pol->kind != RT_CKPT_REVOLVE) {
    const int K = (nmax + interval - 1) / interval;
    // Two segment buffers if the pool has room: segment k-1 is re-computed
    // on the second stream while the adjoint of segment k runs, which fills
    // the GPU better when one kernel alone cannot.  The kernels and their
    // order per buffer are those of the one-stream sweep, so the result is
    // the same to the bit.
    // Segment buffers right after the K snapshots the march wrote (the march
    // leaves room for one: K <= slots_total - (interval - 1)).
    const bool two = c->overlap && interval > 1 && K > 1 && slots_total >= (size_t)K + 2 * (size_t)(interval - 1);
    double* segs[2] = {state_slot((size_t)K), state_slot((size_t)K + (two ? interval - 1 : 0))};
    if (two) {
      if (int rc = ensure_aux(c)) return rc;
      RT_HIP(hipEventRecord(c->seg_free[0], s));
      RT_HIP(hipEventRecord(c->seg_free[1], s));
    }
    auto st = [&](int k, int n) -> double* {
      const int base = k * interval;
      return n == base ? state_slot(k) : segs[two ? (k & 1) : 0] + (size_t)(n - base - 1) * se;
    };
    auto recompute = [&](int k, hipStream_t rs) -> int {
      const int base = k * interval, hi = std::min(base + interval, nmax);
      for (int n = base; n < hi - 1; ++n)
        if (int rc = step_given(st(k, n), st(k, n + 1), n, rs)) return rc;
      return 0;
    };
    if (two) {
      RT_HIP(hipStreamWaitEvent(c->aux_stream, c->seg_free[(K - 1) & 1], 0));
      if (int rc = recompute(K - 1, c->aux_stream)) return rc;
      RT_HIP(hipEventRecord(c->seg_ready[(K - 1) & 1], c->aux_stream));
    }
    for (int k = K - 1; k >= 0; --k) {
      const int base = k * interval, hi = std::min(base + interval, nmax);
      if (two) {
        if (k > 0) {
          RT_HIP(hipStreamWaitEvent(c->aux_stream, c->seg_free[(k - 1) & 1], 0));
          if (int rc = recompute(k - 1, c->aux_stream)) return rc;
          RT_HIP(hipEventRecord(c->seg_ready[(k - 1) & 1], c->aux_stream));
        }
        RT_HIP(hipStreamWaitEvent(s, c->seg_ready[k & 1], 0));
      } else if (int rc = recompute(k, s)) {
        return rc;
      }
      for (int n = hi - 1; n >= base; --n)
        if (int rc = use_fold ? adjoint_folded(st(k, n), n) : adjoint(st(k, n), n)) return rc;
      if (two) RT_HIP(hipEventRecord(c->seg_free[k & 1], s));
    }
    if (int rc = finish_folded()) return rc;
    if (two) {
      RT_HIP(hipEventRecord(c->aux_done, c->aux_stream));
      RT_HIP(hipStreamWaitEvent(s, c->aux_done, 0));
    }
  } else {
    // Binomial checkpointing over slots [0, rev_slots).  Two-level: the
    // segments between the level-1 snapshots, last first (slot k holds
    // U^{k interval}); single level if that is cheaper or the snapshots did
    // not fit (slot 0 holds U^0 either way).
    const bool two = snaps_fit && rtrev::two_level_cost(nmax, interval, rev_slots) <=
                                      rtrev::min_forward_steps(nmax, rev_slots);
    std::vector<rtrev::Action> plan = two ? rtrev::two_level_plan(nmax, interval, rev_slots)
                                          : rtrev::schedule(nmax, rev_slots);
    std::vector<int> slot_step(rev_slots, -1);
    slot_step[0] = 0;
    if (two)
      for (int k = 0; (long)k * interval < nmax; ++k) slot_step[k] = k * interval;
    c->rev_last_two_level = two;
    c->rev_last_interval = interval;
    // The restarts split over streams when the batch has two or more
    // members: group k takes members [k B / ng, (k + 1) B / ng) and runs the
    // whole plan on its own slice of every buffer (states, pool slots,
    // lambda, Z, cases, step logs), group 0 on the caller's stream and the
    // others on streams of their own.  Members are independent, so each gets
    // the same kernels and bits as unsplit; group k starts once group k - 1
    // has launched its first kernels, so that one group's gather (bound by
    // HBM) and steps overlap another's kernel A (bound by VALU issue)
    // instead of running in lockstep with it.
    const bool split = c->overlap && P.nb >= 2;
    const int ng = split ? std::min(P.nb, kSplitGroups) : 1;
    const size_t N = (size_t)P.nx * P.ny, sm = 4 * N;
    struct Group {
      Params P;
      size_t b0;
      hipStream_t st;
      const double* cur;  // holds step cur_step; only ever read
      int cur_step;
      double* lam;
      double* lam_other;
    } g[kMaxGroups];
    if (split)
      if (int rc = ensure_groups(c, ng)) return rc;
    for (int k = 0; k < ng; ++k) {
      Group& G = g[k];
      G.b0 = (size_t)P.nb * k / ng;
      G.P = P;
      G.P.nb = (int)((size_t)P.nb * (k + 1) / ng - G.b0);
      G.st = k == 0 ? s : (k == 1 ? c->aux_stream : c->group_stream[k]);
      G.cur = state_slot(0) + G.b0 * sm;
      G.cur_step = 0;
      G.lam = lam + G.b0 * sm;
      G.lam_other = lam_other + G.b0 * sm;
    }
    if (split) {
      RT_HIP(hipEventRecord(c->group_ev[0], s));  // the march and the terminal adjoint
      for (int k = 1; k < ng; ++k) RT_HIP(hipStreamWaitEvent(g[k].st, c->group_ev[0], 0));
    }
    auto gslot = [&](const Group& G, int slot) { return state_slot((size_t)slot) + G.b0 * sm; };
    auto gstep = [&](const Group& G, const double* src, double* dst, int n) -> int {
      rtk::StepArgs a{};
      a.U = src;
      a.Un = dst;
      a.dt = c->dt_log + G.b0 * (size_t)c->max_steps;
      a.dt_stride = c->max_steps;
      a.dt_index = n;
      a.nsteps_limit = c->nsteps + G.b0;
      a.flags = c->flags;
      RT_HIP(rtk::launch_step(G.P, c->tile, a, G.st));
      return 0;
    };
    auto gadjoint = [&](Group& G, const double* Un, int n) -> int {
      rtk::AdjArgs a{};
      a.U = Un;
      a.lam_next = G.lam;
      a.lam = G.lam_other;
      a.Z = c->Z + G.b0 * 12 * N;
      a.codes = c->codes + G.b0 * N;
      a.dt = c->dt_log + G.b0 * (size_t)c->max_steps;
      a.dt_stride = c->max_steps;
      a.dt_index = n;
      a.nsteps_limit = c->nsteps + G.b0;
      a.flags = c->flags;
      if (dtd) {
        a.dtd.mu = c->dtd_mu + G.b0 * (size_t)c->dtd_stride;
        a.dtd.smax = c->dtd_smax + G.b0 * (size_t)c->dtd_stride;
        a.dtd.imax = c->dtd_imax + G.b0 * (size_t)c->dtd_stride;
        a.dtd.stride = c->dtd_stride;
        a.dtd.count = rtk::step_blocks(G.P, c->tile_adj);
        a.dtd.mu_last = c->dtd_mu_last + G.b0;
      }
      RT_HIP(rtk::launch_adjoint(G.P, c->tile_adj, a, G.st));
      if (dtd) RT_HIP(rtk::launch_dt_correct(G.P, a, G.st));  // updates lambda^n (a.lam) in place
      std::swap(G.lam, G.lam_other);
      return 0;
    };
    // The working state of each group always holds step cur_step and is
    // only ever read: a restore points it at the pool slot, and an advance
    // that a snapshot follows writes its last step straight into that slot,
    // so the schedule needs no state copies (a snapshot of an unadvanced
    // state, if a plan had one, is copied).
    int skew = split ? 1 : ng;  // the next group still to be staggered
    for (size_t ai = 0; ai < plan.size(); ++ai) {
      const rtrev::Action& act = plan[ai];
      for (int k = 0; k < ng; ++k) {
        Group& G = g[k];
        bool launched = false;
        switch (act.kind) {
          case rtrev::Action::TAKESHOT:
            if (G.cur != gslot(G, act.slot)) {
              RT_HIP(rtk::launch_copy(G.cur, gslot(G, act.slot), (size_t)G.P.nb * sm, G.st));
              launched = true;
            }
            if (k == 0) slot_step[act.slot] = G.cur_step;
            G.cur = gslot(G, act.slot);
            break;
          case rtrev::Action::RESTORE:
            G.cur = gslot(G, act.slot);
            G.cur_step = slot_step[act.slot];
            break;
          case rtrev::Action::ADVANCE: {
            double* shot = (ai + 1 < plan.size() && plan[ai + 1].kind == rtrev::Action::TAKESHOT)
                               ? gslot(G, plan[ai + 1].slot)
                               : nullptr;
            double* s0 = c->S0 + G.b0 * sm;
            double* s1 = c->S1 + G.b0 * sm;
            for (int n = G.cur_step; n < act.to; ++n) {
              double* dst = (n == act.to - 1 && shot) ? shot : (G.cur == s0 ? s1 : s0);
              if (int rc = gstep(G, G.cur, dst, n)) return rc;
              G.cur = dst;
              launched = true;
            }
            G.cur_step = act.to;
            break;
          }
          case rtrev::Action::REVERSE:
            if (int rc = gadjoint(G, G.cur, G.cur_step)) return rc;
            launched = true;
            break;
        }
        if (k + 1 == skew && skew < ng && launched) {
          // group k + 1 waits for group k's first kernels
          RT_HIP(hipEventRecord(c->group_ev[skew], G.st));
          RT_HIP(hipStreamWaitEvent(g[skew].st, c->group_ev[skew], 0));
          ++skew;
        }
      }
    }
    for (int k = 1; k < ng; ++k) {
      RT_HIP(hipEventRecord(c->group_ev[k], g[k].st));
      RT_HIP(hipStreamWaitEvent(s, c->group_ev[k], 0));
    }
    // every group reversed the same steps, so its lambda^0 sits in the same
    // buffer of the pair
    lam = g[0].lam;
    lam_other = g[0].lam_other;
  }

  // initial adjoint -> R, gradient
  if (ek_base)
    RT_HIP(rtk::launch_initial_adjoint_plain(P, uv0, lam, grad, s));
  else
    RT_HIP(rtk::launch_initial_adjoint(P, uv0, lam, c->sc(1), c->sc(2), R, grad, s));
  if (int rc = read_flags(c, &f, true)) return rc;
  return flags_status(f);
}
}  // namespace

int rt_grad_u0(rt_ctx* c, const double* uv0, double T, const rt_ckpt_policy* pol, double* R, double* grad,
               int32_t* nsteps_out) {
  return grad_objective(c, uv0, T, pol, nullptr, R, grad, nsteps_out);
}

int rt_grad_ek_anomaly(rt_ctx* c, const double* uv0, double T, const rt_ckpt_policy* pol, const double* ek_base,
                       double* J, double* grad, int32_t* nsteps) {
  if (!ek_base) return fail(RT_EINVAL, "null baseline field");
  return grad_objective(c, uv0, T, pol, ek_base, J, grad, nsteps);
}

int rt_ek_field(rt_ctx* c, const double* U, double* ek) {
  if (int rc = need_ws(c)) return rc;
  if (!U || !ek) return fail(RT_EINVAL, "null argument");
  RT_HIP(rtk::launch_ek_field(c->P, U, ek, c->stream));
  return 0;
}

int rt_mix_width(rt_ctx* c, const double* U, double* h) {
  if (int rc = need_ws(c)) return rc;
  if (!U || !h) return fail(RT_EINVAL, "null argument");
  RT_HIP(rtk::launch_mix_width(c->P, U, c->rowmean, h, c->stream));
  return 0;
}

int rt_row_spectrum(rt_ctx* c, const double* f, int64_t member_stride, int32_t row, double* E) {
  if (!c || !f || !E) return fail(RT_EINVAL, "null argument");
  if (c->P.nx > rtk::kSpecMaxNx) return fail(RT_EINVAL, "nx = %d exceeds %d for the spectrum", c->P.nx, rtk::kSpecMaxNx);
  if (row < -1 || row >= c->P.ny) return fail(RT_EINVAL, "row %d outside -1 .. ny - 1", row);
  if (c->P.nb > 1 && member_stride < (int64_t)c->cells()) return fail(RT_EINVAL, "member_stride below nx * ny");
  RT_HIP(rtk::launch_row_spectrum(c->P.nx, c->P.ny, c->P.nb, f, (long long)member_stride, row, E, c->stream));
  return 0;
}

int rt_power_spectrum_2d(rt_ctx* c, const double* f, int64_t member_stride, double* E) {
  if (int rc = need_ws(c)) return rc;
  if (!f || !E) return fail(RT_EINVAL, "null argument");
  if (c->P.nx > rtk::kSpecMaxNx || c->P.ny > rtk::kSpecMaxNx)
    return fail(RT_EINVAL, "%d x %d exceeds %d x %d for the 2-D spectrum", c->P.nx, c->P.ny, rtk::kSpecMaxNx,
                rtk::kSpecMaxNx);
  if (c->P.nb > 1 && member_stride < (int64_t)c->cells()) return fail(RT_EINVAL, "member_stride below nx * ny");
  // the row transforms, 2 nb ny (nx/2 + 1) <= 12 nb nx ny doubles, in the
  // adjoint's intermediate buffer
  RT_HIP(rtk::launch_power_spectrum_2d(c->P.nx, c->P.ny, c->P.nb, f, (long long)member_stride, c->Z, E, c->stream));
  return 0;
}

int rt_ek_anomaly(rt_ctx* c, const double* U, const double* ek_base, double* J) {
  if (int rc = need_ws(c)) return rc;
  if (!U || !ek_base || !J) return fail(RT_EINVAL, "null argument");
  RT_HIP(rtk::launch_reduce(c->P, 7, U, ek_base, c->partial, c->red_blocks, J, c->stream));
  return 0;
}

int rt_project_to_constraint(rt_ctx* c, double* uv, double delta, int32_t norm, int32_t set, double* norm_out) {
  if (int rc = need_ws(c)) return rc;
  if (!uv || !(delta > 0) || norm < 0 || norm > 2 || set < 0 || set > 1) return fail(RT_EINVAL, "bad argument");
  double* m = norm_out ? norm_out : c->sc(4);
  RT_HIP(rtk::launch_reduce(c->P, 2 + norm, uv, nullptr, c->partial, c->red_blocks, m, c->stream));
  RT_HIP(rtk::launch_scale_project(c->P, uv, m, delta, norm, set, c->stream));
  return 0;
}

int rt_dot(rt_ctx* c, const double* a, const double* b, double* out) {
  if (int rc = need_ws(c)) return rc;
  if (!a || !b || !out) return fail(RT_EINVAL, "null argument");
  RT_HIP(rtk::launch_reduce(c->P, 5, a, b, c->partial, c->red_blocks, out, c->stream));
  return 0;
}

int rt_max_abs(rt_ctx* c, const double* a, double* out) {
  if (int rc = need_ws(c)) return rc;
  if (!a || !out) return fail(RT_EINVAL, "null argument");
  RT_HIP(rtk::launch_reduce(c->P, 6, a, nullptr, c->partial, c->red_blocks, out, c->stream));
  return 0;
}

int rt_axpy(rt_ctx* c, const double* x, const double* alpha, const double* y, double* out) {
  if (!c || !x || !alpha || !y || !out) return fail(RT_EINVAL, "null argument");
  RT_HIP(rtk::launch_axpy(c->P, x, alpha, y, out, c->stream));
  return 0;
}

int rt_check_error(rt_ctx* c) {
  if (int rc = need_ws(c)) return rc;
  Flags f{};
  if (int rc = read_flags(c, &f, true)) return rc;
  return flags_status(f);
}

namespace {
// Replays a reverse-sweep plan on step indices: every step reversed exactly
// once, in decreasing order, from the right state, using only slots
// [0, slots) whose steps slot_step gives at the start.  Adds its forward
// steps to *fw.
int replay_plan(const std::vector<rtrev::Action>& plan, int nsteps, int slots, std::vector<int> slot_step,
                int64_t* fw) {
  int cur = 0, next_rev = nsteps - 1;
  for (const rtrev::Action& a : plan) {
    switch (a.kind) {
      case rtrev::Action::ADVANCE:
        if (a.to < cur) return fail(RT_EINVAL, "schedule advances backwards");
        *fw += a.to - cur;
        cur = a.to;
        break;
      case rtrev::Action::TAKESHOT:
        if (a.slot < 0 || a.slot >= slots) return fail(RT_EINVAL, "slot out of range");
        slot_step[a.slot] = cur;
        break;
      case rtrev::Action::RESTORE:
        if (a.slot < 0 || a.slot >= slots || slot_step[a.slot] < 0) return fail(RT_EINVAL, "restore of empty slot");
        cur = slot_step[a.slot];
        break;
      case rtrev::Action::REVERSE:
        if (a.to != next_rev || cur != a.to) return fail(RT_EINVAL, "reverse out of order at %d", a.to);
        --next_rev;
        break;
    }
  }
  if (next_rev != -1) return fail(RT_EINVAL, "schedule left %d steps unreversed", next_rev + 1);
  return 0;
}
}  // namespace

// Host-only check of the binomial schedule (no GPU): builds the schedule for
// nsteps steps and `slots` slots, replays it on step indices and verifies that
// every step is reversed exactly once, in decreasing order, from the right
// state, using only slots [0, slots).  Returns its forward-step count and
// the closed-form minimum.
int rt_revolve_stats(int32_t nsteps, int32_t slots, int64_t* forward, int64_t* optimum) {
  if (nsteps < 1 || slots < 1 || !forward || !optimum) return fail(RT_EINVAL, "bad argument");
  std::vector<int> slot_step(slots, -1);
  slot_step[0] = 0;
  int64_t fw = 0;
  if (int rc = replay_plan(rtrev::schedule(nsteps, slots), nsteps, slots, slot_step, &fw)) return rc;
  *forward = fw;
  *optimum = rtrev::min_forward_steps(nsteps, slots);
  return 0;
}

// Host-only check of what RT_CKPT_REVOLVE runs for a march of nsteps steps
// with `slots` pool slots when the initial CFL step suggested n_est steps:
// the level-1 interval, then the two-level plan if its snapshots fit in
// slots - 1 slots and it is no dearer than one binomial schedule, else that
// schedule.  Replays and checks the plan as rt_revolve_stats does; forward
// receives every forward step of the gradient (the objective's march
// included), interval and two_level what was chosen.
int rt_revolve_plan_stats(int32_t nsteps, int32_t slots, int32_t n_est, int64_t* forward, int32_t* interval,
                          int32_t* two_level) {
  if (nsteps < 1 || slots < 2 || n_est < 1 || !forward || !interval || !two_level)
    return fail(RT_EINVAL, "bad argument");
  const int I = rtrev::level1_interval(n_est, slots, kRevolveMargin);
  const bool fit = (nsteps + (int64_t)I - 1) / I <= slots - 1;
  const bool two = fit && rtrev::two_level_cost(nsteps, I, slots) <= rtrev::min_forward_steps(nsteps, slots);
  std::vector<int> slot_step(slots, -1);
  slot_step[0] = 0;
  if (two)
    for (int k = 0; (int64_t)k * I < nsteps; ++k) slot_step[k] = k * I;
  int64_t fw = nsteps;  // the objective's forward march
  const std::vector<rtrev::Action> plan = two ? rtrev::two_level_plan(nsteps, I, slots) : rtrev::schedule(nsteps, slots);
  if (int rc = replay_plan(plan, nsteps, slots, slot_step, &fw)) return rc;
  *forward = fw;
  *interval = I;
  *two_level = two ? 1 : 0;
  return 0;
}

}  // extern "C"
