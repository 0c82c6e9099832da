// Internal launch interface between the C ABI (rt_api.hip) and the HIP
// kernels (rt_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "rt_device.h"

namespace rtk {

// Per-member march control, device resident.  Written by the step kernel's
// last block (or by march_begin), read by the next step.
struct Ctl {
  double t;        // time reached
  double dt;       // step to take next
  double T;        // end time
  int32_t nsteps;  // steps taken
  int32_t done;    // 1 once t == T
  int32_t last;    // 1 if dt was clipped to end exactly at T
  int32_t pad;
};

// Flags shared by all members (device).
struct Flags {
  int32_t err_unphys;   // a state or face state was unphysical
  int32_t err_overflow; // step log or snapshot pool overflow
  int32_t n_active;     // members not done
  int32_t pad;
};

// Arguments of the fused step kernel.
struct StepArgs {
  const double* U;     // U^n       [B][4][ny][nx]
  double* Un;          // U^{n+1}
  // time step: adaptive (ctl != nullptr) or given (dt[b * dt_stride + dt_index])
  Ctl* ctl;
  const double* dt;
  int32_t dt_stride, dt_index;
  const int32_t* nsteps_limit;  // given-dt mode: members with dt_index >= limit[b] are skipped
  // CFL epilogue: per-block max signal speed of U^{n+1}
  double* partial;              // [B][nblk]
  uint32_t* counter;            // [B] last-block counters (self-resetting)
  double* dt_next;              // given-dt mode: unclipped CFL step of U^{n+1} (may be null)
  double* dt_log;               // adaptive mode: step log [B][dt_log_cap]
  int32_t dt_log_cap;
  // snapshots (adaptive mode): U^n copied to pool[slot][B][4][ny][nx] when
  // nsteps % snap_interval == 0, slot = nsteps / snap_interval
  double* pool;
  int32_t snap_interval, snap_slots;
  Flags* flags;
};

struct AdjArgs {
  const double* U;         // U^n
  const double* lam_next;  // lambda^{n+1}
  double* lam;             // lambda^n
  double* Z;               // [B][12][ny][nx] predictor-adjoint output
  int32_t* codes;          // [B][ny][nx] MC cases
  const double* dt;        // dt[b * dt_stride + dt_index]
  int32_t dt_stride, dt_index;
  const int32_t* nsteps_limit;  // members with dt_index >= limit[b] pass lambda through
  Flags* flags;
};

struct Launch {
  int tile;   // tile shape id
  int red_blocks;
};

// Tile shapes of the fused step / adjoint kernels (TX x TY cells, 256 threads).
enum TileId { TILE_16x16 = 0, TILE_32x8 = 1, TILE_64x4 = 2, TILE_COUNT = 3 };
void tile_dims(int tile, int* tx, int* ty);
int step_blocks(const Params& P, int tile);  // blocks per member

hipError_t launch_init_state(const Params& P, const double* uv0, double* U, hipStream_t s);
hipError_t launch_step(const Params& P, int tile, const StepArgs& a, hipStream_t s);
hipError_t launch_adjoint(const Params& P, int tile, const AdjArgs& a, hipStream_t s);
// Per-member reductions: kind 0 = max signal speed, 1 = kinetic energy,
// 2.. = weighted |uv|^2 for the projection (norm id = kind - 2), 5 = dot.
hipError_t launch_reduce(const Params& P, int kind, const double* a, const double* b, double* partial,
                         int nblk, double* out, hipStream_t s);
hipError_t launch_march_begin(const Params& P, const double* maxspeed, double T, Ctl* ctl, Flags* flags,
                              hipStream_t s);
hipError_t launch_cfl_from_speed(const Params& P, const double* maxspeed, double* dt, hipStream_t s);
hipError_t launch_copy_final(const Params& P, const Ctl* ctl, const double* A, const double* Bbuf, double* U,
                             double* t_out, int32_t* nsteps_out, const double* log_src, int32_t log_src_cap,
                             double* log_dst, int32_t log_dst_cap, hipStream_t s);
hipError_t launch_copy(const double* src, double* dst, size_t n, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, size_t n, hipStream_t s);
hipError_t launch_terminal_adjoint(const Params& P, const double* U, const double* ke0, double* lam,
                                   hipStream_t s);
hipError_t launch_initial_adjoint(const Params& P, const double* uv0, const double* lam0, const double* ke0,
                                  const double* keN, double* R, double* grad, hipStream_t s);
hipError_t launch_scale_project(const Params& P, double* uv, const double* m, double delta, int norm,
                                int set, hipStream_t s);
hipError_t launch_axpy(const Params& P, const double* x, const double* alpha, const double* y, double* out,
                       hipStream_t s);
hipError_t launch_ratio(int nb, const double* num, const double* den, double* out, hipStream_t s);

}  // namespace rtk
