// Internal launch interface between the C ABI (rt_api.hip) and the HIP
// kernels (rt_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "rt_device.h"

namespace rtk {

// Per-member march control, device resident and double buffered: the step
// launched with index L reads ctl[L & 1] and its block (0, 0) writes
// ctl[(L + 1) & 1], so no block can see a half-updated record.
struct Ctl {
  double t;        // time reached
  double T;        // end time
  double dt_last;  // step taken by the launch that wrote this record
  int32_t nsteps;  // steps taken
  int32_t done;    // 1 once t == T
};

// Flags shared by all members (device).
struct Flags {
  int32_t err_unphys;    // a state or face state was unphysical
  int32_t err_overflow;  // step log overflow (stops the march)
  int32_t n_active;      // members not done
  int32_t snap_overflow; // a snapshot fell beyond the pool's slots (the march goes on)
};

// Arguments of the fused step kernel.
constexpr int kAccSlots = 32;   // atomic-max slots per member and row
constexpr int kAccStride = 16;  // uint64 per slot: one 128-byte line each
constexpr int kAccRow = kAccSlots * kAccStride;

struct StepArgs {
  const double* U;     // U^n       [B][4][ny][nx]
  double* Un;          // U^{n+1}
  // Adaptive mode (ctl != nullptr).  The largest signal speed of each
  // member's state is kept as the bit pattern of a non-negative double
  // (ordered like the unsigned integer) in acc[3][B][kAccSlots] (one slot
  // per 128-byte line): launch L reads acc[L % 3] (speeds of U^n, the max
  // over the slots) to form its CFL step, folds the speeds of U^{n+1} into
  // acc[(L + 1) % 3] with one atomic max per block on the block's slot, and
  // clears acc[(L + 2) % 3] for the next launch.  Spreading the blocks'
  // atomics over the slots keeps them from queueing on one address.
  Ctl* ctl;                     // [2][B]
  uint64_t* acc;                // [3][B][kAccSlots * kAccStride]
  int32_t launch;
  double* dt_log;               // step log [B][dt_log_cap]
  int32_t dt_log_cap;
  // snapshots: U^n copied to pool[slot][B][4][ny][nx] when
  // nsteps % snap_interval == 0, slot = nsteps / snap_interval
  double* pool;
  int32_t snap_interval, snap_slots;
  // Given-dt mode: dt = dt[b * dt_stride + dt_index]; members with
  // dt_index >= nsteps_limit[b] are skipped.  acc_out (may be null) receives
  // the largest signal speed of U^{n+1} (bit pattern, must start at 0).
  const double* dt;
  int32_t dt_stride, dt_index;
  const int32_t* nsteps_limit;
  uint64_t* acc_out;
  Flags* flags;
};

struct AdjArgs {
  const double* U;         // U^n
  const double* lam_next;  // lambda^{n+1}
  double* lam;             // lambda^n
  double* Z;               // [B][12][ny][nx] kernel A's output for the gather (direct part, slope cotangents)
  int32_t* codes;          // [B][ny][nx] MC cases
  const double* dt;        // dt[b * dt_stride + dt_index]
  int32_t dt_stride, dt_index;
  const int32_t* nsteps_limit;  // members with dt_index >= limit[b] pass lambda through
  Flags* flags;
  // Folded gather (fold.Z != nullptr): lambda^{n+1} is not read from
  // lam_next but formed on the tile + halo 1 from the previous adjoint
  // kernel's outputs for step n+1 (its Z, codes, state U^{n+1} and
  // lambda^{n+2}); the tile's own cells of lambda^{n+1} go to fold.lam_out.
  struct Fold {
    const double* Z;
    const int32_t* codes;
    const double* U;         // U^{n+1}
    const double* lam_next;  // lambda^{n+2}
    double* lam_out;         // lambda^{n+1}
    int32_t dt_index;        // n + 1
  } fold;
  // Differentiated step size (dtd.mu != nullptr, two-kernel form only):
  // kernel A also writes, per block (tile index ty * tiles_x + tx), its
  // share of mu = <lambda^{n+1}, dU^{n+1}/d dt> (every face once, every own
  // cell once) and the largest signal speed of U^n over its own cells with
  // the smallest index of a cell that holds it; launch_dt_correct then
  // combines them.
  struct Dtd {
    double* mu;       // [B][stride]
    double* smax;     // [B][stride]
    int32_t* imax;    // [B][stride]
    int32_t stride;   // partials per member, >= the adjoint grid's tiles
    int32_t count;    // tiles of the adjoint grid per member
    double* mu_last;  // [B] mu of each member's last (clipped) step
  } dtd;
};

// Tile shapes of the fused step / adjoint kernels: TX x TY cells with 256
// threads, with 576 threads ("W" variants: one pass per phase), 32 x 16
// cells with 512 threads (less halo work per cell), or 16 x 15 and 15 x 16
// cells with 256 threads (every face loop of the adjoint in one pass of the
// block: 255 and 256 faces of each direction).  All variants produce
// bitwise-identical results.
enum TileId {
  TILE_16x16 = 0,
  TILE_32x8 = 1,
  TILE_64x4 = 2,
  TILE_16x16W = 3,
  TILE_32x8W = 4,
  TILE_16x8 = 5,
  TILE_8x8 = 6,
  TILE_16x8W = 7,
  TILE_8x8W = 8,
  TILE_32x16 = 9,
  TILE_16x15 = 10,
  TILE_15x16 = 11,
  TILE_COUNT = 12
};
void tile_dims(int tile, int* tx, int* ty, int* nt);
int step_blocks(const Params& P, int tile);  // blocks per member

// prow: background pressure per row (well-balanced variant) or null.
hipError_t launch_init_state(const Params& P, const double* uv0, double* U, const double* prow, hipStream_t s);
// Background pressure per row of the well-balanced variant into prow[ny].
hipError_t launch_background_rows(const Params& P, double* prow, hipStream_t s);
hipError_t launch_step(const Params& P, int tile, const StepArgs& a, hipStream_t s);
// Adjoint of one step: kernel A (face and predictor adjoints -> Z, codes),
// then kernel B (limiter gather -> lambda^n), or kernel A alone
// (gather = false) when the next kernel A folds the gather in.
hipError_t launch_adjoint(const Params& P, int tile, const AdjArgs& a, hipStream_t s, bool gather = true);
// Kernel B alone: lambda^n from Z, codes, U^n and lambda^{n+1} of step n.
hipError_t launch_adj_gather(const Params& P, const AdjArgs& a, hipStream_t s);
// Differentiated step size, after both adjoint kernels of step n (a.U = U^n,
// a.lam = lambda^n, updated in place, a.dtd filled by kernel A): on the
// member's last step, mu_last = mu; on every earlier step,
// lambda^n += (mu - mu_last) d dt_n / dU^n at the cell of the largest
// signal speed, dt_n = cfl / S(U^n).  One block per member.
hipError_t launch_dt_correct(const Params& P, const AdjArgs& a, hipStream_t s);
// Per-member reductions: kind 0 = max signal speed, 1 = kinetic energy,
// 2.. = weighted |uv|^2 for the projection (norm id = kind - 2), 5 = dot,
// 6 = max |x| of a velocity field, 7 = objective of Eq. 8 (a = U,
// b = baseline e_k field [B][ny][nx]).
hipError_t launch_reduce(const Params& P, int kind, const double* a, const double* b, double* partial,
                         int nblk, double* out, hipStream_t s);
hipError_t launch_march_begin(const Params& P, const double* maxspeed, double T, Ctl* ctl, uint64_t* acc,
                              Flags* flags, hipStream_t s);
hipError_t launch_cfl_from_speed(const Params& P, const double* maxspeed, double* dt, hipStream_t s);
hipError_t launch_cfl_from_bits(const Params& P, const uint64_t* acc, double* dt, hipStream_t s);
hipError_t launch_copy_final(const Params& P, const Ctl* ctl, const double* A, const double* Bbuf, double* U,
                             double* t_out, int32_t* nsteps_out, const double* log_src, int32_t log_src_cap,
                             double* log_dst, int32_t log_dst_cap, hipStream_t s);
hipError_t launch_copy(const double* src, double* dst, size_t n, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, size_t n, hipStream_t s);
hipError_t launch_terminal_adjoint(const Params& P, const double* U, const double* ke0, double* lam,
                                   hipStream_t s);
hipError_t launch_initial_adjoint(const Params& P, const double* uv0, const double* lam0, const double* ke0,
                                  const double* keN, double* R, double* grad, hipStream_t s);
hipError_t launch_terminal_adjoint_ek(const Params& P, const double* U, const double* ek_base, double* lam,
                                      hipStream_t s);
hipError_t launch_initial_adjoint_plain(const Params& P, const double* uv0, const double* lam0, double* grad,
                                       hipStream_t s);
hipError_t launch_ek_field(const Params& P, const double* U, double* ek, hipStream_t s);
// Mixing width of Eqs. 13-14 (rowmean: scratch [B][ny]).
hipError_t launch_mix_width(const Params& P, const double* U, double* rowmean, double* h, hipStream_t s);
hipError_t launch_scale_project(const Params& P, double* uv, const double* m, double delta, int norm,
                                int set, hipStream_t s);
hipError_t launch_axpy(const Params& P, const double* x, const double* alpha, const double* y, double* out,
                       hipStream_t s);
hipError_t launch_ratio(int nb, const double* num, const double* den, double* out, hipStream_t s);

}  // namespace rtk
