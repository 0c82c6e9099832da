// HIP kernels for gfx950: the fused forward step, the two-kernel discrete
// adjoint of the step, and the small elementwise / reduction kernels around
// them.  All arithmetic is FP64.
//
// Fused step (one launch per time step for all members):
//   block = one tile of TX x TY cells of one member (the tile shapes and
//            thread counts are listed with TileId);
//   phase A  primitives of the tile plus a 2-cell halo into LDS (x periodic,
//            y ghost rows from the wall boundary condition);
//   phase B  MC slopes and the MUSCL-Hancock predictor of the tile plus a
//            1-cell cross-shaped halo into LDS;
//   phase C  HLLC fluxes of every face of the tile, each computed once;
//   phase D  conservative update with the gravity source, store, optional
//            snapshot of U^n, and the largest signal speed of U^{n+1};
//   epilogue the block's largest signal speed goes by an integer atomic max
//            (on the bit pattern) into one of the member's slots, which the
//            next launch reduces into its CFL step (no extra launch, no host
//            sync).
// Adjoint of one step (frozen dt): kernel A recomputes phases A-C, runs the
// HLLC / wall-flux adjoints on every face of the tile and the predictor
// adjoint of every tile cell, and forms each cell's direct part of lambda^n
// (its own primitive cotangent through the primitive-variable adjoint, plus
// the identity and gravity terms); kernel B gathers the limiter adjoints of
// the five slope stencils touching a cell, maps them through the
// primitive-variable adjoint and adds the direct part.
#include <hip/hip_runtime.h>

#include "rt_kernels.h"

namespace rtk {

namespace {

// Periodic column index.  The tile halos reach at most TX + 2 columns past
// the domain, so for every grid wider than that one conditional add or
// subtract does; narrower grids take the loop.
__device__ __forceinline__ int wrapx(int i, int nx) {
  i = i < 0 ? i + nx : (i >= nx ? i - nx : i);
  if ((unsigned)i >= (unsigned)nx) {
    while (i < 0) i += nx;
    while (i >= nx) i -= nx;
  }
  return i;
}

// Element i of an array of doubles (or int32) addressed as a uniform base
// plus a 32-bit byte offset, which maps onto the scalar-base / 32-bit
// vector-offset form of the global memory instructions.  Every plane of a
// state holds fewer than 2^28 cells (checked when a context is created).
__device__ __forceinline__ double ldg(const double* base, uint32_t i) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + i * 8u);
}
__device__ __forceinline__ void stg(double* base, uint32_t i, double v) {
  *reinterpret_cast<double*>(reinterpret_cast<char*>(base) + i * 8u) = v;
}
__device__ __forceinline__ int32_t ldg(const int32_t* base, uint32_t i) {
  return *reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(base) + i * 4u);
}
__device__ __forceinline__ void stg(int32_t* base, uint32_t i, int32_t v) {
  *reinterpret_cast<int32_t*>(reinterpret_cast<char*>(base) + i * 4u) = v;
}

// Wavefront reductions with DPP lane permutations inside each row of 16
// lanes (swap neighbours, swap pairs, mirror half-rows, mirror rows: after
// the four steps every lane holds its row's result, the same in every lane
// because each step combines a lane with its partner in both orders), then
// the four rows' results read from lanes 0, 16, 32, 48 and combined in a
// fixed order.  Called with the whole wavefront active; `id` fills lanes
// whose source is inactive.
template <int CTRL>
__device__ __forceinline__ double dpp_perm(double v, double id) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned long long o = (unsigned long long)__double_as_longlong(id);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)o, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
  const unsigned hi =
      (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(o >> 32), (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

constexpr int kDppQuadSwap1 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadSwap2 = 0x4E;  // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;

__device__ __forceinline__ double wave_max(double v) {
  const double id = -__builtin_inf();
  v = fmax(v, dpp_perm<kDppQuadSwap1>(v, id));
  v = fmax(v, dpp_perm<kDppQuadSwap2>(v, id));
  v = fmax(v, dpp_perm<kDppHalfMirror>(v, id));
  v = fmax(v, dpp_perm<kDppMirror>(v, id));
  return fmax(fmax(read_lane(v, 0), read_lane(v, 16)), fmax(read_lane(v, 32), read_lane(v, 48)));
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_perm<kDppQuadSwap1>(v, 0.0);
  v += dpp_perm<kDppQuadSwap2>(v, 0.0);
  v += dpp_perm<kDppHalfMirror>(v, 0.0);
  v += dpp_perm<kDppMirror>(v, 0.0);
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

template <int NT>
__device__ double block_max(double v, double* red) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double m = red[0];
#pragma unroll
  for (int k = 1; k < NT / 64; ++k) m = fmax(m, red[k]);
  return m;
}

template <int NT>
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int k = 1; k < NT / 64; ++k) s += red[k];
  return s;
}

// Largest s over the block with the smallest i among equal s (a total
// order, so the result does not depend on the order of combination).
__device__ __forceinline__ void argmax_merge(double& s, int& i, double s2, int i2) {
  if (s2 > s || (s2 == s && i2 < i)) {
    s = s2;
    i = i2;
  }
}

template <int NT>
__device__ void block_argmax(double& s, int& i, double* rs, int* ri) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) argmax_merge(s, i, __shfl_xor(s, o, 64), __shfl_xor(i, o, 64));
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) {
    rs[w] = s;
    ri[w] = i;
  }
  __syncthreads();
  s = rs[0];
  i = ri[0];
#pragma unroll
  for (int k = 1; k < NT / 64; ++k) argmax_merge(s, i, rs[k], ri[k]);
}

__device__ __forceinline__ double rho0_at(const Params& P, double y) {
  return 0.5 * (P.rho_h + P.rho_l) + 0.5 * (P.rho_h - P.rho_l) * tanh((y - P.y0) / P.h);
}

__device__ __forceinline__ double p0_at(const Params& P, double y) {
  const double z = (y - P.y0) / P.h;
  const double az = fabs(z);
  const double lc = az + log1p(exp(-2.0 * az)) - 0.69314718055994530942;
  return P.p_int + P.g_y * (0.5 * (P.rho_h + P.rho_l) * (y - P.y0) + 0.5 * (P.rho_h - P.rho_l) * P.h * lc);
}

// ----------------------------------------------------------------- tile of a workgroup
// Workgroups are dispatched round-robin over the 8 XCDs of the chip (linear
// id mod 8), and each XCD has its own L2.  With tiles in raster order,
// horizontally adjacent tiles would sit on different XCDs and each L2 would
// fetch the halo cache lines they share.  Instead, the workgroups of XCD k
// take the k-th contiguous band of tiles (in raster order within the band):
// horizontal neighbours share an L2, and vertical neighbours follow one
// tile row later in the same L2.  A bijection of [0, T) for any T.
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_band(int L, int T) {
  const int per = (T + kXcds - 1) / kXcds;  // items of each of the first `tall` XCDs
  const int tall = T - (per - 1) * kXcds;   // 1..8 XCDs with `per` items, the rest per - 1
  const int xcd = L % kXcds, local = L / kXcds;
  return xcd < tall ? xcd * per + local : tall * per + (xcd - tall) * (per - 1) + local;
}

__device__ __forceinline__ void tile_of_block(int& bx, int& by) {
  const int nbx = (int)gridDim.x;
  const int t = xcd_band((int)blockIdx.x + nbx * (int)blockIdx.y, nbx * (int)gridDim.y);
  bx = t % nbx;
  by = t / nbx;
}

// ----------------------------------------------------------------- LDS tile helpers
// Phase A: primitives of the tile + halo 2.  Returns nonzero on an
// unphysical interior state.  A thread's cells are addressed first and all
// their loads issued before any is used, so the memory latencies of its
// passes overlap instead of adding up; halo rows beyond the wall ghosts load
// a clamped in-range cell that is never used.
template <int TX, int TY, int NT, class LDS>
__device__ int tile_prims(const Params& P, const double* U, size_t N, int x0, int y0, LDS& S) {
  constexpr int AX = TX + 4, AY = TY + 4, IT = (AX * AY + NT - 1) / NT;
  int bad = 0;
  uint32_t c[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int k = (int)threadIdx.x + it * NT;
    const int kk = k < AX * AY ? k : AX * AY - 1;
    const int lx = kk % AX, ly = kk / AX;
    const int gx = wrapx(x0 - 2 + lx, P.nx);
    const int gy = y0 - 2 + ly;
    const int sy = gy < 0 ? 0 : (gy >= P.ny ? P.ny - 1 : gy);
    c[it] = (uint32_t)(sy * P.nx + gx);
  }
  double r[IT], mx[IT], my[IT], E[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    r[it] = ldg(U, c[it]);
    mx[it] = ldg(U + N, c[it]);
    my[it] = ldg(U + 2 * N, c[it]);
    E[it] = ldg(U + 3 * N, c[it]);
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int k = (int)threadIdx.x + it * NT;
    if (k >= AX * AY) break;
    const int lx = k % AX, ly = k / AX;
    const int gy = y0 - 2 + ly;
    W4 w{1.0, 0.0, 0.0, 1.0, 1.0};
    if (gy >= -1 && gy <= P.ny) {
      w = cons_to_prim(P, r[it], mx[it], my[it], E[it]);
      if (gy >= 0 && gy < P.ny) bad |= unphysical(w);
      if (gy < 0) w = ghost_bottom(P, w);
      else if (gy >= P.ny) w = ghost_top(P, w);
    }
    S.W[0][ly][lx] = w.r;
    S.W[1][ly][lx] = w.u;
    S.W[2][ly][lx] = w.v;
    S.W[3][ly][lx] = w.p;
    S.W[4][ly][lx] = w.ri;
  }
  return bad;
}

template <class LDS>
__device__ __forceinline__ W4 ldW(const LDS& S, int x, int y) {
  return W4{S.W[0][y][x], S.W[1][y][x], S.W[2][y][x], S.W[3][y][x], S.W[4][y][x]};
}
template <class LDS>
__device__ __forceinline__ W4 ldQ(const LDS& S, int k, int x, int y) {
  return W4{S.Q[4 * k + 0][y][x], S.Q[4 * k + 1][y][x], S.Q[4 * k + 2][y][x], S.Q[4 * k + 3][y][x], 0.0};
}

// Phase B: slopes and predictor on the cross-shaped halo-1 region.  BAL:
// the well-balanced pressure slopes in y (mc_p_balanced).  CODES: the MC
// cases of the tile cells go to codes_out.
//
// One position k of the halo-1 region, computed without branches: a corner,
// a row outside the domain or an index past the region is computed from
// in-range LDS values (k clamped) and reported as not valid, so the caller
// stores nothing for it.
template <int TX, int TY, bool BAL, bool CODES, class LDS>
__device__ __forceinline__ bool predict_at(const Params& P, const LDS& S, int k, int y0, double hx, double hy,
                                           double hg, W4& q, W4& sx, W4& sy, int& cx, int& cy) {
  constexpr int QX = TX + 2, QY = TY + 2;
  const int kc = k < QX * QY ? k : QX * QY - 1;
  const int lx = kc % QX, ly = kc / QX;
  const int gy = y0 - 1 + ly;
  const bool valid = k < QX * QY && !((lx == 0 || lx == QX - 1) && (ly == 0 || ly == QY - 1)) && gy >= 0 &&
                     gy < P.ny;
  const W4 wc = ldW(S, lx + 1, ly + 1);
  sx = mc4<CODES>(P, ldW(S, lx, ly + 1), wc, ldW(S, lx + 2, ly + 1), cx);
  sy = mc4<CODES>(P, ldW(S, lx + 1, ly), wc, ldW(S, lx + 1, ly + 2), cy);
  if constexpr (BAL) mc_p_balanced<CODES>(P, ldW(S, lx + 1, ly), wc, ldW(S, lx + 1, ly + 2), sy, cy);
  q = predict(P, wc, sx, sy, hx, hy, hg);
  return valid;
}

// Stores one position's predicted state and slopes (and its MC cases for a
// tile cell); returns nonzero if a face state would be unphysical.
template <int TX, int TY, bool CODES, class LDS>
__device__ __forceinline__ int predict_store(const Params& P, LDS& S, int k, int x0, int y0, const W4& q,
                                             const W4& sx, const W4& sy, int cx, int cy, int32_t* codes_out) {
  constexpr int QX = TX + 2;
  const int lx = k % QX, ly = k / QX;
  S.Q[0][ly][lx] = q.r;
  S.Q[1][ly][lx] = q.u;
  S.Q[2][ly][lx] = q.v;
  S.Q[3][ly][lx] = q.p;
  S.Q[4][ly][lx] = sx.r;
  S.Q[5][ly][lx] = sx.u;
  S.Q[6][ly][lx] = sx.v;
  S.Q[7][ly][lx] = sx.p;
  S.Q[8][ly][lx] = sy.r;
  S.Q[9][ly][lx] = sy.u;
  S.Q[10][ly][lx] = sy.v;
  S.Q[11][ly][lx] = sy.p;
  if constexpr (CODES) {
    if (lx >= 1 && lx <= TX && ly >= 1 && ly <= TY) {
      const int gx = x0 - 1 + lx;
      if (gx < P.nx) stg(codes_out, (uint32_t)((y0 - 1 + ly) * P.nx + gx), cx | (cy << 8));
    }
  }
  const double hr = 0.5 * fabs(sx.r), hp = 0.5 * fabs(sx.p), vr = 0.5 * fabs(sy.r), vp = 0.5 * fabs(sy.p);
  return !(q.r - hr > 0.0) || !(q.p - hp > 0.0) || !(q.r - vr > 0.0) || !(q.p - vp > 0.0);
}

// The region has more positions than the block has threads for the 256-
// thread tiles, so some wavefronts take two.  With PAIR those compute both
// positions in one branch-free stretch (their instruction streams
// interleave and hide each other's latency) instead of one after the
// other; whether a wavefront has a second position is uniform across it.
// PAIR costs registers: the step kernel has them to spare, the adjoint
// kernel would drop to two wavefronts per SIMD.
//
// ALIAS: the predicted states overwrite the primitive tile they are computed
// from (one LDS region serves both): every thread computes its positions
// (two at most) into registers, the block waits until all have read the
// primitives, then the results are stored.
template <int TX, int TY, int NT, bool BAL, bool CODES, bool PAIR, bool ALIAS = false, class LDS>
__device__ int tile_predict(const Params& P, double dt, int x0, int y0, LDS& S, int32_t* codes_out) {
  constexpr int QN = (TX + 2) * (TY + 2);
  const double hx = 0.5 * dt * P.inv_dx, hy = 0.5 * dt * P.inv_dy, hg = 0.5 * dt * P.g_y;
  int bad = 0;
  if constexpr (ALIAS) {
    static_assert(PAIR && !CODES && QN <= 2 * NT, "one pass of at most two positions per thread");
    const int k = threadIdx.x;
    const int wave_first = k - (int)(threadIdx.x & 63);
    W4 q, sx, sy, q2 = W4{}, sx2 = W4{}, sy2 = W4{};
    int cx = 0, cy = 0, cx2 = 0, cy2 = 0;
    const bool v1 = predict_at<TX, TY, BAL, CODES>(P, S, k, y0, hx, hy, hg, q, sx, sy, cx, cy);
    bool v2 = false;
    if (wave_first + NT < QN) v2 = predict_at<TX, TY, BAL, CODES>(P, S, k + NT, y0, hx, hy, hg, q2, sx2, sy2, cx2, cy2);
    __syncthreads();  // the primitives are read: their space takes the predicted states
    if (v1) bad |= predict_store<TX, TY, CODES>(P, S, k, x0, y0, q, sx, sy, cx, cy, codes_out);
    if (v2) bad |= predict_store<TX, TY, CODES>(P, S, k + NT, x0, y0, q2, sx2, sy2, cx2, cy2, codes_out);
    return bad;
  }
  for (int k = threadIdx.x; k < QN; k += (PAIR ? 2 : 1) * NT) {
    const int wave_first = k - (int)(threadIdx.x & 63);
    W4 q, sx, sy;
    int cx = 0, cy = 0;
    if (PAIR && wave_first + NT < QN) {
      W4 q2, sx2, sy2;
      int cx2 = 0, cy2 = 0;
      const bool v1 = predict_at<TX, TY, BAL, CODES>(P, S, k, y0, hx, hy, hg, q, sx, sy, cx, cy);
      const bool v2 = predict_at<TX, TY, BAL, CODES>(P, S, k + NT, y0, hx, hy, hg, q2, sx2, sy2, cx2, cy2);
      if (v1) bad |= predict_store<TX, TY, CODES>(P, S, k, x0, y0, q, sx, sy, cx, cy, codes_out);
      if (v2) bad |= predict_store<TX, TY, CODES>(P, S, k + NT, x0, y0, q2, sx2, sy2, cx2, cy2, codes_out);
    } else {
      if (predict_at<TX, TY, BAL, CODES>(P, S, k, y0, hx, hy, hg, q, sx, sy, cx, cy))
        bad |= predict_store<TX, TY, CODES>(P, S, k, x0, y0, q, sx, sy, cx, cy, codes_out);
    }
  }
  return bad;
}

// Face states from the predictor region: x faces in (r, n = u, t = v, p),
// y faces in (r, n = v, t = u, p).
template <class LDS>
__device__ __forceinline__ FS xface_right_of(const LDS& S, int x, int y) {  // state at the cell's right face
  return FS{S.Q[0][y][x] + 0.5 * S.Q[4][y][x], S.Q[1][y][x] + 0.5 * S.Q[5][y][x], S.Q[2][y][x] + 0.5 * S.Q[6][y][x],
            S.Q[3][y][x] + 0.5 * S.Q[7][y][x]};
}
template <class LDS>
__device__ __forceinline__ FS xface_left_of(const LDS& S, int x, int y) {
  return FS{S.Q[0][y][x] - 0.5 * S.Q[4][y][x], S.Q[1][y][x] - 0.5 * S.Q[5][y][x], S.Q[2][y][x] - 0.5 * S.Q[6][y][x],
            S.Q[3][y][x] - 0.5 * S.Q[7][y][x]};
}
template <class LDS>
__device__ __forceinline__ FS yface_top_of(const LDS& S, int x, int y) {
  return FS{S.Q[0][y][x] + 0.5 * S.Q[8][y][x], S.Q[2][y][x] + 0.5 * S.Q[10][y][x], S.Q[1][y][x] + 0.5 * S.Q[9][y][x],
            S.Q[3][y][x] + 0.5 * S.Q[11][y][x]};
}
template <class LDS>
__device__ __forceinline__ FS yface_bottom_of(const LDS& S, int x, int y) {
  return FS{S.Q[0][y][x] - 0.5 * S.Q[8][y][x], S.Q[2][y][x] - 0.5 * S.Q[10][y][x], S.Q[1][y][x] - 0.5 * S.Q[9][y][x],
            S.Q[3][y][x] - 0.5 * S.Q[11][y][x]};
}

// Phase C's face items: k < NXF are the x faces (TX + 1 per tile row, TY
// rows), the next NYF the y faces (TX per face row, TY + 1 rows), with no
// gap, so a wavefront may hold both kinds.  Both kinds run one instruction
// stream: the face's two predicted states are read through per-lane LDS
// offsets (which planes hold the normal and the tangential velocity and
// their slopes, and whether the right state is the next column or the next
// row), and the flux comes back in face-normal order.  Only y faces on a
// wall branch off.
template <int TX, int TY>
struct FaceItems {
  static constexpr int QX = TX + 2, PS = (TX + 2) * (TY + 2);
  static constexpr int NXF = (TX + 1) * TY, NYF = TX * (TY + 1), N = NXF + NYF;
};

// Flux of face item k in face-normal order; returns 1 for an x face, 2 for a
// y face, 0 past the items or for a face outside the domain.  Every lane
// runs the same instructions (an item past the end reads the last item's
// states, a face outside the domain reads whatever its rows hold, and a
// wall face's HLLC result is replaced), so a wavefront never takes two
// paths except for the wall faces of the first and last tile rows.
template <int TX, int TY, class LDS>
__device__ __forceinline__ int step_face_flux(const Params& P, const LDS& S, int k, int y0, double f[4]) {
  using FI = FaceItems<TX, TY>;
  const int kc = k < FI::N ? k : FI::N - 1;
  const bool xf = kc < FI::NXF;
  const int kk = kc - FI::NXF;
  const int fy = xf ? kc / (TX + 1) : kk / TX;
  const int fx = xf ? kc - (kc / (TX + 1)) * (TX + 1) : kk % TX;
  const int j = y0 + fy;
  // left state: the right face of cell (fx, fy + 1) or the top face of
  // cell (fx + 1, fy) of the predictor region; right state one column or
  // one row further
  const int l = xf ? (fy + 1) * FI::QX + fx : fy * FI::QX + fx + 1;
  const int r = l + (xf ? 1 : FI::QX);
  const int pn = xf ? FI::PS : 2 * FI::PS, pt = xf ? 2 * FI::PS : FI::PS;  // velocity planes
  const int sb = xf ? 4 * FI::PS : 8 * FI::PS;                             // slope planes
  const double* q = &S.Q[0][0][0];
  const FS L{q[l] + 0.5 * q[sb + l], q[pn + l] + 0.5 * q[sb + pn + l], q[pt + l] + 0.5 * q[sb + pt + l],
             q[3 * FI::PS + l] + 0.5 * q[sb + 3 * FI::PS + l]};
  const FS R{q[r] - 0.5 * q[sb + r], q[pn + r] - 0.5 * q[sb + pn + r], q[pt + r] - 0.5 * q[sb + pt + r],
             q[3 * FI::PS + r] - 0.5 * q[sb + 3 * FI::PS + r]};
  hllc(P, L, R, f);
  if (!xf && (j == 0 || j == P.ny)) {
    f[1] = j == 0 ? wall_pressure(P, R, false) : wall_pressure(P, L, true);
    f[0] = 0.0;
    f[2] = 0.0;
    f[3] = 0.0;
  }
  const bool inside = k < FI::N && (xf ? j < P.ny : j <= P.ny);
  return inside ? (xf ? 1 : 2) : 0;
}

// Stores the flux of face item k (kind from step_face_flux) into F or G.
template <int TX, int TY, class LDS>
__device__ __forceinline__ void step_face_store(LDS& S, int k, int kind, const double f[4]) {
  using FI = FaceItems<TX, TY>;
  if (kind == 1) {
    const int fx = k % (TX + 1), fy = k / (TX + 1);
    S.fg.F[0][fy][fx] = f[0];
    S.fg.F[1][fy][fx] = f[1];
    S.fg.F[2][fy][fx] = f[2];
    S.fg.F[3][fy][fx] = f[3];
  } else if (kind == 2) {
    const int kk = k - FI::NXF, fx = kk % TX, fy = kk / TX;
    S.fg.G[0][fy][fx] = f[0];
    S.fg.G[1][fy][fx] = f[2];
    S.fg.G[2][fy][fx] = f[1];
    S.fg.G[3][fy][fx] = f[3];
  }
}

// ----------------------------------------------------------------- step
// LDS of the step kernel: the flux arrays reuse the primitive tile, which is
// dead once the predictor has run.
template <int TX, int TY, bool ALIAS = false>
struct StepLDS {
  static constexpr int AX = TX + 4, AY = TY + 4;
  static constexpr int QX = TX + 2, QY = TY + 2;
  union {
    double W[5][AY][AX];  // rho, u, v, p, 1/rho
    struct {
      double F[4][TY][TX + 1];
      double G[4][TY + 1][TX];
    } fg;
  };
  double Q[12][QY][QX];
};
// ALIAS: one region by phase (primitives, then predicted states and slopes,
// then fluxes), for a fourth resident block per CU on large grids.
template <int TX, int TY>
struct StepLDS<TX, TY, true> {
  static constexpr int AX = TX + 4, AY = TY + 4;
  static constexpr int QX = TX + 2, QY = TY + 2;
  union {
    double W[5][AY][AX];
    double Q[12][QY][QX];
    struct {
      double F[4][TY][TX + 1];
      double G[4][TY + 1][TX];
    } fg;
  };
};

template <int TX, int TY, int NT, bool BAL, bool ALIAS = false>
__global__ __launch_bounds__(NT) void k_step(Params P, StepArgs a) {
  static_assert(NT >= TX * TY && NT % 64 == 0, "one thread per tile cell at least");
  __shared__ StepLDS<TX, TY, ALIAS> S;
  __shared__ double sRed[NT / 64];

  const int b = blockIdx.z;
  int tbx, tby;
  tile_of_block(tbx, tby);
  const int x0 = tbx * TX, y0 = tby * TY;
  const int tid = threadIdx.x;
  const int nx = P.nx, ny = P.ny;
  const size_t N = (size_t)nx * ny;
  const double* U = a.U + (size_t)b * 4 * N;
  const bool first_block = blockIdx.x == 0 && blockIdx.y == 0;

  // time step of this member.  In the march the control record and the
  // signal-speed slots are loaded here but used only after phase A, which
  // does not depend on them, so their latency overlaps it.
  double dt = 0.0;
  int nstep = 0;
  bool last = false;
  const Ctl* cin = nullptr;
  Ctl* cout = nullptr;
  int done = 0;
  double t_in = 0.0, T_in = 0.0, ms_lane = 0.0;
  if (a.ctl) {
    const int L = a.launch;
    cin = a.ctl + (size_t)(L & 1) * P.nb + b;
    cout = a.ctl + (size_t)((L + 1) & 1) * P.nb + b;
    done = cin->done;
    t_in = cin->t;
    T_in = cin->T;
    nstep = cin->nsteps;
    // a few slots per lane; the max across the wave is taken after phase A
    const uint64_t* row = a.acc + ((size_t)(L % 3) * P.nb + b) * kAccRow;
    const int lane = tid & 63;
#pragma unroll
    for (int k = lane; k < kAccSlots; k += 64)
      ms_lane = fmax(ms_lane, __longlong_as_double((long long)row[k * kAccStride]));
  } else {
    if (a.nsteps_limit && a.dt_index >= a.nsteps_limit[b]) return;
    dt = a.dt[(size_t)b * a.dt_stride + a.dt_index];
  }

  // prefetch this thread's own cell for the update
  const int tx = tid % TX, ty = tid / TX;
  const int gx = x0 + tx, gy = y0 + ty;
  const bool own = tid < TX * TY && gx < nx && gy < ny;
  const uint32_t c = own ? (uint32_t)(gy * nx + gx) : 0u;
  double u0 = 0.0, u1 = 0.0, u2 = 0.0, u3 = 0.0;
  if (own) {
    u0 = ldg(U, c);
    u1 = ldg(U + N, c);
    u2 = ldg(U + 2 * N, c);
    u3 = ldg(U + 3 * N, c);
  }

  // phase A: primitives of the tile + halo 2
  int bad = tile_prims<TX, TY, NT>(P, U, N, x0, y0, S);
  if (a.ctl) {
    // the same member for the whole block, so the return is uniform
    if (done) {
      if (first_block && tid == 0) *cout = *cin;
      return;
    }
    const double ms = wave_max(ms_lane);
    const double rem = T_in - t_in;
    dt = P.cfl / ms;
    if (dt >= rem) {
      dt = rem;
      last = true;
    }
  }
  __syncthreads();

  // phase B: slopes and predictor on the cross-shaped halo-1 region
  bad |= tile_predict<TX, TY, NT, BAL, false, true, ALIAS>(P, dt, x0, y0, S, nullptr);
  __syncthreads();

  // phase C: every face of the tile once
  constexpr int NF = FaceItems<TX, TY>::N;
  if constexpr (ALIAS) {
    // the fluxes overwrite the predicted states: all faces of this thread
    // first, then the stores once every thread has read its states
    constexpr int FMAX = (NF + NT - 1) / NT;
    double fl[FMAX][4];
    int kind[FMAX];
#pragma unroll
    for (int it = 0; it < FMAX; ++it) {
      kind[it] = 0;
      if ((tid & ~63) + it * NT < NF) kind[it] = step_face_flux<TX, TY>(P, S, tid + it * NT, y0, fl[it]);
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < FMAX; ++it) step_face_store<TX, TY>(S, tid + it * NT, kind[it], fl[it]);
  } else {
    for (int k = tid; (k & ~63) < NF; k += NT) {
      double f[4];
      const int kind = step_face_flux<TX, TY>(P, S, k, y0, f);
      step_face_store<TX, TY>(S, k, kind, f);
    }
  }
  __syncthreads();

  // phase D: update with the gravity source
  const bool need_speed = a.ctl != nullptr || a.acc_out != nullptr;
  double smax = 0.0;
  if (own) {
    const double ax = dt * P.inv_dx, ay = dt * P.inv_dy;
    double n0 = u0 - ax * (S.fg.F[0][ty][tx + 1] - S.fg.F[0][ty][tx]) - ay * (S.fg.G[0][ty + 1][tx] - S.fg.G[0][ty][tx]);
    double n1 = u1 - ax * (S.fg.F[1][ty][tx + 1] - S.fg.F[1][ty][tx]) - ay * (S.fg.G[1][ty + 1][tx] - S.fg.G[1][ty][tx]);
    double n2 = u2 - ax * (S.fg.F[2][ty][tx + 1] - S.fg.F[2][ty][tx]) - ay * (S.fg.G[2][ty + 1][tx] - S.fg.G[2][ty][tx]);
    double n3 = u3 - ax * (S.fg.F[3][ty][tx + 1] - S.fg.F[3][ty][tx]) - ay * (S.fg.G[3][ty + 1][tx] - S.fg.G[3][ty][tx]);
    const double dtg = dt * P.g_y;
    n2 = n2 + dtg * 0.5 * (u0 + n0);
    n3 = n3 + dtg * 0.5 * (S.fg.G[0][ty][tx] + S.fg.G[0][ty + 1][tx]);
    double* Un = a.Un + (size_t)b * 4 * N;
    stg(Un, c, n0);
    stg(Un + N, c, n1);
    stg(Un + 2 * N, c, n2);
    stg(Un + 3 * N, c, n3);
    if (a.pool && (nstep % a.snap_interval) == 0) {
      const int slot = nstep / a.snap_interval;
      if (slot < a.snap_slots) {
        double* sp = a.pool + ((size_t)slot * P.nb + b) * 4 * N;
        stg(sp, c, u0);
        stg(sp + N, c, u1);
        stg(sp + 2 * N, c, u2);
        stg(sp + 3 * N, c, u3);
      } else {
        bad |= 4;  // snapshot beyond the pool, reported below
      }
    }
    if (need_speed) {
      const W4 w = cons_to_prim(P, n0, n1, n2, n3);
      bad |= unphysical(w);
      const double cs = sqrt_fast(P.gamma * w.p * w.ri);
      const double sx = (fabs(w.u) + cs) * P.inv_dx, sy = (fabs(w.v) + cs) * P.inv_dy;
      smax = sx > sy ? sx : sy;
    }
  }
  if (bad & 4) atomicOr(&a.flags->snap_overflow, 1);
  if (bad & 1) atomicOr(&a.flags->err_unphys, 1);
  if (!need_speed) return;

  // epilogue: fold the block's largest signal speed of U^{n+1} into the
  // member's accumulator (non-negative doubles order like their bits)
  const double bm = block_max<NT>(smax, sRed);
  if (a.ctl == nullptr) {
    if (tid == 0) atomicMax((unsigned long long*)(a.acc_out + b), (unsigned long long)__double_as_longlong(bm));
    return;
  }
  const int L = a.launch;
  if (first_block) {
    // clear the slots of launch L + 1's target, one per thread
    uint64_t* clr = a.acc + ((size_t)((L + 2) % 3) * P.nb + b) * kAccRow;
    for (int k = tid; k < kAccSlots; k += NT) clr[k * kAccStride] = 0ull;
  }
  if (tid != 0) return;
  const int slot = (int)((blockIdx.x + (size_t)gridDim.x * blockIdx.y) % kAccSlots);
  atomicMax((unsigned long long*)(a.acc + ((size_t)((L + 1) % 3) * P.nb + b) * kAccRow + slot * kAccStride),
            (unsigned long long)__double_as_longlong(bm));
  if (!first_block) return;
  if (a.dt_log) {
    if (nstep < a.dt_log_cap) a.dt_log[(size_t)b * a.dt_log_cap + nstep] = dt;
    else atomicOr(&a.flags->err_overflow, 1);
  }
  Ctl o;
  o.T = T_in;
  o.t = last ? T_in : t_in + dt;
  o.dt_last = dt;
  o.nsteps = nstep + 1;
  o.done = last ? 1 : 0;
  *cout = o;
  if (last) atomicSub(&a.flags->n_active, 1);
}

// ----------------------------------------------------------------- limiter gather
__device__ __forceinline__ void add_slope_terms(double sb[4], int code, double scale_a, double scale_b, double out[4]) {
  // out += (scale_a * wa + scale_b * wb) * sb, per variable with its own case
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double wa, wb;
    mc_weights((code >> (2 * v)) & 3, wa, wb);
    out[v] += (scale_a * wa + scale_b * wb) * sb[v];
  }
}

// Outputs of kernel A for one step n of one member, read by the gather.
struct GatherSrc {
  const double* Z;        // [12][ny][nx]: planes 0..3 the cell's direct part of lambda^n (conservative),
                          // 4..7 and 8..11 the cotangents of its x and y slopes (primitive)
  const int32_t* codes;   // [ny][nx]
  const double* U;        // U^n, [4][ny][nx]
  const double* lam_next; // lambda^{n+1}, [4][ny][nx] (read for finished members only)
  bool pass;              // member finished before step n: lambda^n = lambda^{n+1}
};

// lambda^n at cell (i, j): the limiter gather of the slope cotangents of
// the cell and its four neighbours through the MC cases and the wall ghost
// terms, mapped by the adjoint of the primitive map at U^n, plus the direct
// part kernel A left in Z (the cell's own primitive cotangent mapped the
// same way, and the identity and gravity-source terms of the update).  BAL:
// the well-balanced pressure slopes' dependence on the cell's density.
template <bool BAL>
__device__ __forceinline__ void lambda_at(const Params& P, const GatherSrc& g, int i, int j, double out[4]) {
  const int nx = P.nx, ny = P.ny;
  const size_t N = (size_t)nx * ny;
  const uint32_t idx = (uint32_t)(j * nx + i);
  const double* Lm = g.lam_next;
  if (g.pass) {
    out[0] = ldg(Lm, idx);
    out[1] = ldg(Lm + N, idx);
    out[2] = ldg(Lm + 2 * N, idx);
    out[3] = ldg(Lm + 3 * N, idx);
    return;
  }
  const double* Z = g.Z;
  const int32_t* codes = g.codes;
  const double* U = g.U;
  double wb[4] = {0.0, 0.0, 0.0, 0.0};
  // x slopes at d = c-1, c, c+1
  {
    const uint32_t cm = (uint32_t)(j * nx + (i == 0 ? nx - 1 : i - 1));
    const uint32_t cp = (uint32_t)(j * nx + (i == nx - 1 ? 0 : i + 1));
    double sm[4] = {ldg(Z + 4 * N, cm), ldg(Z + 5 * N, cm), ldg(Z + 6 * N, cm), ldg(Z + 7 * N, cm)};
    double s0[4] = {ldg(Z + 4 * N, idx), ldg(Z + 5 * N, idx), ldg(Z + 6 * N, idx), ldg(Z + 7 * N, idx)};
    double sp[4] = {ldg(Z + 4 * N, cp), ldg(Z + 5 * N, cp), ldg(Z + 6 * N, cp), ldg(Z + 7 * N, cp)};
    add_slope_terms(sm, ldg(codes, cm) & 0xff, 0.0, 1.0, wb);    // c is d+1: +wb
    add_slope_terms(s0, ldg(codes, idx) & 0xff, 1.0, -1.0, wb);  // c is d: wa - wb
    add_slope_terms(sp, ldg(codes, cp) & 0xff, -1.0, 0.0, wb);   // c is d-1: -wa
  }
  // y slopes
  {
    const int c0 = ldg(codes, idx) >> 8;
    double s0[4] = {ldg(Z + 8 * N, idx), ldg(Z + 9 * N, idx), ldg(Z + 10 * N, idx), ldg(Z + 11 * N, idx)};
    add_slope_terms(s0, c0, 1.0, -1.0, wb);
    if constexpr (BAL) {
      // the balanced pressure slope h + MC(a' , b') also depends on the
      // cell's density through h = rho g_y dy, in h and in a', b'
      double wa, wbb;
      mc_weights((c0 >> 6) & 3, wa, wbb);
      wb[0] += P.g_y * P.dy * (1.0 - wa - wbb) * s0[3];
    }
    if (j > 0) {
      const uint32_t cm = idx - (uint32_t)nx;
      double sm[4] = {ldg(Z + 8 * N, cm), ldg(Z + 9 * N, cm), ldg(Z + 10 * N, cm), ldg(Z + 11 * N, cm)};
      add_slope_terms(sm, ldg(codes, cm) >> 8, 0.0, 1.0, wb);
    }
    if (j < ny - 1) {
      const uint32_t cp = idx + (uint32_t)nx;
      double sp[4] = {ldg(Z + 8 * N, cp), ldg(Z + 9 * N, cp), ldg(Z + 10 * N, cp), ldg(Z + 11 * N, cp)};
      add_slope_terms(sp, ldg(codes, cp) >> 8, -1.0, 0.0, wb);
    }
    // the wall ghost cell is a function of this cell
    if (j == 0 || j == ny - 1) {
      double gb[4] = {0.0, 0.0, 0.0, 0.0};
      if (j == 0) add_slope_terms(s0, c0, -1.0, 0.0, gb);       // ghost below: a = W - Wg
      if (j == ny - 1) add_slope_terms(s0, c0, 0.0, 1.0, gb);   // ghost above: b = Wg - W
      // (for ny == 1 both apply; ny >= 2 is required)
      const double sgn = j == 0 ? -1.0 : 1.0;
      wb[0] += gb[0] + sgn * P.g_y * P.dy * gb[3];
      wb[1] += gb[1];
      wb[2] -= gb[2];
      wb[3] += gb[3];
    }
  }
  const W4 w = cons_to_prim(P, ldg(U, idx), ldg(U + N, idx), ldg(U + 2 * N, idx), ldg(U + 3 * N, idx));
  double ub[4];
  prim_adj(P, w, W4{wb[0], wb[1], wb[2], wb[3]}, ub);
  out[0] = ldg(Z, idx) + ub[0];
  out[1] = ldg(Z + N, idx) + ub[1];
  out[2] = ldg(Z + 2 * N, idx) + ub[2];
  out[3] = ldg(Z + 3 * N, idx) + ub[3];
}

// ----------------------------------------------------------------- adjoint A
// LDS of adjoint kernel A.  The face cotangents reuse the primitive tile,
// which is dead once the predictor has run (the tile cell's own primitives
// are recomputed from registers for the predictor adjoint).  lambda^{n+1}
// on the halo-1 region is staged in LDS only when the kernel forms it by
// the folded gather; otherwise the face loops read it from global memory
// (L2), which keeps the footprint small enough for more resident blocks
// per CU.
//
// Two ways to hand a face's cotangents to its two cells.  OWNF (blocks with
// a spare thread for every boundary face): each tile cell's thread takes
// the face to its right and the face above it and keeps the cotangent of its
// own side in registers; the block's spare threads take the tile's left and
// bottom boundary faces.  Only the far side's cotangent goes through LDS,
// and the x and y faces share one phase (one barrier instead of three).
// Otherwise the x faces and then the y faces are loops over all faces of
// the tile, both sides through LDS.
template <int TX, int TY, bool OWNF>
struct AdjCore {
  static constexpr int AX = TX + 4, AY = TY + 4;
  static constexpr int QX = TX + 2, QY = TY + 2;
  union {
    double W[5][AY][AX];  // rho, u, v, p, 1/rho
    struct {
      double XL[4][TY][TX + 1];  // x faces: cotangent of the left state (r, u, v, p)
      double XR[4][TY][TX + 1];  // x faces: cotangent of the right state
    } fx;
    struct {
      double YB[4][TY + 1][TX];  // y faces: cotangent of the state below
      double YT[4][TY + 1][TX];  // y faces: cotangent of the state above
    } fy;
  };
  double Q[12][QY][QX];
};
template <int TX, int TY>
struct AdjCore<TX, TY, true> {
  static constexpr int AX = TX + 4, AY = TY + 4;
  static constexpr int QX = TX + 2, QY = TY + 2;
  union {
    double W[5][AY][AX];
    struct {
      double XR[4][TY][TX];  // cell (x, y): cotangent of the right state of its left face (r, u, v, p)
      double YT[4][TY][TX];  // cell (x, y): cotangent of the upper state of its bottom face (r, u, v, p)
    } fo;
  };
  double Q[12][QY][QX];
};
template <int TX, int TY, bool FOLD, bool OWNF>
struct AdjLDS : AdjCore<TX, TY, OWNF> {};
template <int TX, int TY, bool OWNF>
struct AdjLDS<TX, TY, true, OWNF> : AdjCore<TX, TY, OWNF> {
  double L[4][AdjCore<TX, TY, OWNF>::QY][AdjCore<TX, TY, OWNF>::QX];  // lambda on the halo-1 region
};

// DTD: also the step-size derivative mu and the signal-speed argmax of U^n
// (AdjArgs::Dtd).  With lambda-tilde l (l_0 = lambda_0 + (dt g/2) lambda_2)
// and the fluxes F of the step, mu sums
//   x faces   (1/dx) [<l_R - l_L, F> + (dt g/2)(l_2R - l_2L) F_0]
//   y faces   (1/dy) [<l_T - l_B, G> + (dt g/2)(l_2T - l_2B) G_0]
//             + (g/2)(l_3B + l_3T) G_0     (walls: +-(1/dy) l_2 p*)
//   cells     g lambda_2 rho - <q-bar, A_x(W) s_x>/(2 dx)
//             - <q-bar, A_y(W) s_y>/(2 dy) + (g/2) q-bar_v
// which is d<lambda^{n+1}, U^{n+1}>/d dt of the update with gravity
// source (the flux terms once from the explicit dt, once from the dt in
// the source's use of rho^{n+1}) and of the MUSCL-Hancock predictor.
template <int TX, int TY, int NT, bool FOLD, bool DTD, bool BAL>
__global__ __launch_bounds__(NT) void k_adj_a(Params P, AdjArgs a) {
  static_assert(NT >= TX * TY && NT % 64 == 0, "one thread per tile cell at least");
  static_assert(!(FOLD && DTD), "the step-size derivative needs the two-kernel form");
  static_assert(!(FOLD && BAL), "the well-balanced variant runs the two-kernel form");
  // a spare thread for each boundary face: the tile's own faces in one phase
  constexpr bool OWNF = NT - TX * TY >= (TX > TY ? TX : TY);
  constexpr int QX = AdjCore<TX, TY, OWNF>::QX, QY = AdjCore<TX, TY, OWNF>::QY;
  __shared__ AdjLDS<TX, TY, FOLD, OWNF> S;

  const int b = blockIdx.z;
  int tbx, tby;
  tile_of_block(tbx, tby);
  const int x0 = tbx * TX, y0 = tby * TY;
  const int tid = threadIdx.x;
  const int nx = P.nx, ny = P.ny;
  const size_t N = (size_t)nx * ny;
  if (a.nsteps_limit && a.dt_index >= a.nsteps_limit[b]) {
    // the member finished before step n; a folded step n+1 >= n has
    // finished too, so lambda^{n+1} = lambda^{n+2} on the tile
    if (FOLD && tid < TX * TY) {
      const int gx = x0 + tid % TX, gy = y0 + tid / TX;
      if (gx < nx && gy < ny) {
        const uint32_t c = (uint32_t)(gy * nx + gx);
        const double* Ln = a.fold.lam_next + (size_t)b * 4 * N;
        double* Lo = a.fold.lam_out + (size_t)b * 4 * N;
        stg(Lo, c, ldg(Ln, c));
        stg(Lo + N, c, ldg(Ln + N, c));
        stg(Lo + 2 * N, c, ldg(Ln + 2 * N, c));
        stg(Lo + 3 * N, c, ldg(Ln + 3 * N, c));
      }
    }
    return;
  }
  const double* U = a.U + (size_t)b * 4 * N;
  const double* Lm = a.lam_next + (size_t)b * 4 * N;
  const double dt = a.dt[(size_t)b * a.dt_stride + a.dt_index];
  const double hdtg = 0.5 * dt * P.g_y;
  const int tx = tid % TX, ty = tid / TX;
  const int gx = x0 + tx, gy = y0 + ty;
  const bool own = tid < TX * TY && gx < nx && gy < ny;
  const uint32_t c = own ? (uint32_t)(gy * nx + gx) : 0u;
  double u0 = 1.0, u1 = 0.0, u2 = 0.0, u3 = 1.0;
  if (own) {
    u0 = ldg(U, c);
    u1 = ldg(U + N, c);
    u2 = ldg(U + 2 * N, c);
    u3 = ldg(U + 3 * N, c);
  }

  int bad = tile_prims<TX, TY, NT>(P, U, N, x0, y0, S);
  if constexpr (FOLD) {
    // lambda^{n+1} on the halo-1 region (corners unused), formed by the
    // folded gather of step n+1; the tile's own cells go to lam_out
    GatherSrc g{};
    g.Z = a.fold.Z + (size_t)b * 12 * N;
    g.codes = a.fold.codes + (size_t)b * N;
    g.U = a.fold.U + (size_t)b * 4 * N;
    g.lam_next = a.fold.lam_next + (size_t)b * 4 * N;
    g.pass = a.nsteps_limit && a.fold.dt_index >= a.nsteps_limit[b];
    double* lam_out = a.fold.lam_out + (size_t)b * 4 * N;
    for (int k = tid; k < QX * QY; k += NT) {
      const int lx = k % QX, ly = k / QX;
      const int qy = y0 - 1 + ly;
      double l[4] = {0.0, 0.0, 0.0, 0.0};
      const bool corner = (lx == 0 || lx == QX - 1) && (ly == 0 || ly == QY - 1);
      if (qy >= 0 && qy < ny && !corner) {
        const int ux = x0 - 1 + lx, qx = wrapx(ux, nx);
        lambda_at<false>(P, g, qx, qy, l);
        if (lx >= 1 && lx <= TX && ly >= 1 && ly <= TY && ux < nx) {
          const uint32_t cc = (uint32_t)(qy * nx + qx);
          stg(lam_out, cc, l[0]);
          stg(lam_out + N, cc, l[1]);
          stg(lam_out + 2 * N, cc, l[2]);
          stg(lam_out + 3 * N, cc, l[3]);
        }
      }
      S.L[0][ly][lx] = l[0];
      S.L[1][ly][lx] = l[1];
      S.L[2][ly][lx] = l[2];
      S.L[3][ly][lx] = l[3];
    }
  }
  __syncthreads();
  bad |= tile_predict<TX, TY, NT, BAL, true, false>(P, dt, x0, y0, S, a.codes + (size_t)b * N);
  __syncthreads();

  // lambda-tilde (rho entry shifted by the momentum source) at halo-1
  // position (lx, ly) of the tile; rows outside the domain are never asked
  auto lam = [&](int lx, int ly, double l[4]) {
    if constexpr (FOLD) {
      l[0] = S.L[0][ly][lx] + hdtg * S.L[2][ly][lx];
      l[1] = S.L[1][ly][lx];
      l[2] = S.L[2][ly][lx];
      l[3] = S.L[3][ly][lx];
    } else {
      const uint32_t cc = (uint32_t)((y0 - 1 + ly) * nx + wrapx(x0 - 1 + lx, nx));
      const double l2 = ldg(Lm + 2 * N, cc);
      l[0] = ldg(Lm, cc) + hdtg * l2;
      l[1] = ldg(Lm + N, cc);
      l[2] = l2;
      l[3] = ldg(Lm + 3 * N, cc);
    }
  };

  const double ax = dt * P.inv_dx, ay = dt * P.inv_dy;
  double mu = 0.0;  // DTD: this thread's share of d<lambda^{n+1}, U^{n+1}>/d dt
  // The adjoint of x face (fx, fy), between halo-1 cells (fx, fy+1) [left]
  // and (fx+1, fy+1) [right], into the cotangents of its two states (x
  // frame: r, n = u, t = v, p).  DTD counts each face once: the right faces
  // of the tile's own cells.
  auto xface = [&](int fx, int fy, FS& Lb, FS& Rb) {
    double lL[4], lR[4];
    lam(fx, fy + 1, lL);
    lam(fx + 1, fy + 1, lR);
    const double Fb[4] = {ax * (lR[0] - lL[0]), ax * (lR[1] - lL[1]), ax * (lR[2] - lL[2]), ax * (lR[3] - lL[3])};
    if constexpr (DTD) {
      double F[4];
      hllc_adj(P, xface_right_of(S, fx, fy + 1), xface_left_of(S, fx + 1, fy + 1), Fb, Lb, Rb, F);
      if (fx >= 1 && x0 + fx - 1 < nx)
        mu += P.inv_dx * ((lR[0] - lL[0]) * F[0] + (lR[1] - lL[1]) * F[1] + (lR[2] - lL[2]) * F[2] +
                          (lR[3] - lL[3]) * F[3] + hdtg * (lR[2] - lL[2]) * F[0]);
    } else {
      hllc_adj(P, xface_right_of(S, fx, fy + 1), xface_left_of(S, fx + 1, fy + 1), Fb, Lb, Rb);
    }
  };
  // y face (fx, fy), between halo-1 cells (fx+1, fy) [below] and (fx+1,
  // fy+1) [above], row j = y0 + fy of faces (walls at 0 and ny, nothing
  // beyond), into the cotangents of its two states (y frame: r, n = v,
  // t = u, p).  DTD counts each face once: the walls and the top faces of
  // the tile's own rows (col: the face's column is in the domain).
  auto yface = [&](int fx, int fy, bool col, FS& Bb, FS& Tb) {
    const int j = y0 + fy;
    if (j == 0) {
      double lT[4];
      lam(fx + 1, fy + 1, lT);
      wall_pressure_adj(P, yface_bottom_of(S, fx + 1, fy + 1), false, ay * lT[2], Tb);
      if constexpr (DTD)
        if (col) mu += P.inv_dy * lT[2] * wall_pressure(P, yface_bottom_of(S, fx + 1, fy + 1), false);
    } else if (j == ny) {
      double lB[4];
      lam(fx + 1, fy, lB);
      wall_pressure_adj(P, yface_top_of(S, fx + 1, fy), true, -ay * lB[2], Bb);
      if constexpr (DTD)
        if (col) mu -= P.inv_dy * lB[2] * wall_pressure(P, yface_top_of(S, fx + 1, fy), true);
    } else if (j < ny) {
      double lB[4], lT[4];
      lam(fx + 1, fy, lB);
      lam(fx + 1, fy + 1, lT);
      const double g0 = ay * (lT[0] - lB[0]) + hdtg * (lT[3] + lB[3]);
      const double g1 = ay * (lT[1] - lB[1]);
      const double g2 = ay * (lT[2] - lB[2]);
      const double g3 = ay * (lT[3] - lB[3]);
      const double Fb[4] = {g0, g2, g1, g3};  // y frame: normal momentum is m_y
      if constexpr (DTD) {
        double F[4];  // y frame: mass, m_y, m_x, energy
        hllc_adj(P, yface_top_of(S, fx + 1, fy), yface_bottom_of(S, fx + 1, fy + 1), Fb, Bb, Tb, F);
        if (fy >= 1 && col)
          mu += P.inv_dy * ((lT[0] - lB[0]) * F[0] + (lT[1] - lB[1]) * F[2] + (lT[2] - lB[2]) * F[1] +
                            (lT[3] - lB[3]) * F[3] + hdtg * (lT[2] - lB[2]) * F[0]) +
                0.5 * P.g_y * (lT[3] + lB[3]) * F[0];
      } else {
        hllc_adj(P, yface_top_of(S, fx + 1, fy), yface_bottom_of(S, fx + 1, fy + 1), Fb, Bb, Tb);
      }
    }
  };

  // the tile cell's cotangents from its four faces, in primitive order:
  // xl / xr of the right state of its left face and the left state of its
  // right face, yb / yt likewise in y
  W4 xl{0, 0, 0, 0, 0}, xr{0, 0, 0, 0, 0}, yb{0, 0, 0, 0, 0}, yt{0, 0, 0, 0, 0};
  if constexpr (OWNF) {
    // one phase: a tile cell's thread takes the face to its right and the
    // face above it; spare thread e the left face of tile row e and the
    // bottom face of tile column e.  The far side goes to LDS for the cell
    // that owns it.
    const int e = tid - TX * TY;
    FS Lb{0, 0, 0, 0}, Rb{0, 0, 0, 0}, Bb{0, 0, 0, 0}, Tb{0, 0, 0, 0};
    if (own || (e >= 0 && e < TY && y0 + e < ny)) {
      const int fx = own ? tx + 1 : 0, fy = own ? ty : e;
      xface(fx, fy, Lb, Rb);
      if (fx < TX) {
        S.fo.XR[0][fy][fx] = Rb.r;
        S.fo.XR[1][fy][fx] = Rb.n;
        S.fo.XR[2][fy][fx] = Rb.t;
        S.fo.XR[3][fy][fx] = Rb.p;
      }
    }
    if (own || (e >= 0 && e < TX && x0 + e < nx)) {
      const int fx = own ? tx : e, fy = own ? ty + 1 : 0;
      yface(fx, fy, true, Bb, Tb);
      if (fy < TY) {
        S.fo.YT[0][fy][fx] = Tb.r;
        S.fo.YT[1][fy][fx] = Tb.t;
        S.fo.YT[2][fy][fx] = Tb.n;
        S.fo.YT[3][fy][fx] = Tb.p;
      }
    }
    __syncthreads();
    if (own) {
      xl = W4{S.fo.XR[0][ty][tx], S.fo.XR[1][ty][tx], S.fo.XR[2][ty][tx], S.fo.XR[3][ty][tx]};
      xr = W4{Lb.r, Lb.n, Lb.t, Lb.p};
      yb = W4{S.fo.YT[0][ty][tx], S.fo.YT[1][ty][tx], S.fo.YT[2][ty][tx], S.fo.YT[3][ty][tx]};
      yt = W4{Bb.r, Bb.t, Bb.n, Bb.p};
    }
  } else {
    // x faces, all of the tile's in a loop, both sides through LDS
    for (int k = tid; k < (TX + 1) * TY; k += NT) {
      const int fx = k % (TX + 1), fy = k / (TX + 1);
      FS Lb{0, 0, 0, 0}, Rb{0, 0, 0, 0};
      if (y0 + fy < ny) xface(fx, fy, Lb, Rb);
      // x-frame (r, n = u, t = v, p) is the primitive order
      S.fx.XL[0][fy][fx] = Lb.r;
      S.fx.XL[1][fy][fx] = Lb.n;
      S.fx.XL[2][fy][fx] = Lb.t;
      S.fx.XL[3][fy][fx] = Lb.p;
      S.fx.XR[0][fy][fx] = Rb.r;
      S.fx.XR[1][fy][fx] = Rb.n;
      S.fx.XR[2][fy][fx] = Rb.t;
      S.fx.XR[3][fy][fx] = Rb.p;
    }
    __syncthreads();
    if (own) {
      xl = W4{S.fx.XR[0][ty][tx], S.fx.XR[1][ty][tx], S.fx.XR[2][ty][tx], S.fx.XR[3][ty][tx]};
      xr = W4{S.fx.XL[0][ty][tx + 1], S.fx.XL[1][ty][tx + 1], S.fx.XL[2][ty][tx + 1], S.fx.XL[3][ty][tx + 1]};
    }
    __syncthreads();
    // y faces, the thread index rotated by one wavefront so that a second
    // pass of this loop and of the x-face loop fall on different wavefronts
    for (int k = (tid + NT - 64) % NT; k < TX * (TY + 1); k += NT) {
      const int fx = k % TX, fy = k / TX;
      FS Bb{0, 0, 0, 0}, Tb{0, 0, 0, 0};
      yface(fx, fy, x0 + fx < nx, Bb, Tb);
      // y-frame (r, n = v, t = u, p) -> primitive order (r, u, v, p)
      S.fy.YB[0][fy][fx] = Bb.r;
      S.fy.YB[1][fy][fx] = Bb.t;
      S.fy.YB[2][fy][fx] = Bb.n;
      S.fy.YB[3][fy][fx] = Bb.p;
      S.fy.YT[0][fy][fx] = Tb.r;
      S.fy.YT[1][fy][fx] = Tb.t;
      S.fy.YT[2][fy][fx] = Tb.n;
      S.fy.YT[3][fy][fx] = Tb.p;
    }
    __syncthreads();
    if (own) {
      yb = W4{S.fy.YT[0][ty][tx], S.fy.YT[1][ty][tx], S.fy.YT[2][ty][tx], S.fy.YT[3][ty][tx]};
      yt = W4{S.fy.YB[0][ty + 1][tx], S.fy.YB[1][ty + 1][tx], S.fy.YB[2][ty + 1][tx], S.fy.YB[3][ty + 1][tx]};
    }
  }

  if (own) {
    const int lx = tx + 1, ly = ty + 1;
    // q-bar from the four faces, sx-bar and sy-bar
    const W4 qx{xl.r + xr.r, xl.u + xr.u, xl.v + xr.v, xl.p + xr.p};
    W4 sxb{0.5 * (xr.r - xl.r), 0.5 * (xr.u - xl.u), 0.5 * (xr.v - xl.v), 0.5 * (xr.p - xl.p)};
    const W4 qb{qx.r + yb.r + yt.r, qx.u + yb.u + yt.u, qx.v + yb.v + yt.v, qx.p + yb.p + yt.p};
    W4 syb{0.5 * (yt.r - yb.r), 0.5 * (yt.u - yb.u), 0.5 * (yt.v - yb.v), 0.5 * (yt.p - yb.p)};
    W4 wb{0.0, 0.0, 0.0, 0.0};
    const W4 w = cons_to_prim(P, u0, u1, u2, u3);
    const W4 sx = ldQ(S, 1, lx, ly), sy = ldQ(S, 2, lx, ly);
    predict_adj(P, w, sx, sy, 0.5 * dt * P.inv_dx, 0.5 * dt * P.inv_dy, qb, wb, sxb, syb);
    if constexpr (DTD) {
      double l[4];
      lam(lx, ly, l);
      const double ri = w.ri;
      const double axr = w.u * sx.r + w.r * sx.u, axu = w.u * sx.u + sx.p * ri, axv = w.u * sx.v,
                   axp = P.gamma * w.p * sx.u + w.u * sx.p;
      const double ayr = w.v * sy.r + w.r * sy.v, ayu = w.v * sy.u, ayv = w.v * sy.v + sy.p * ri,
                   ayp = P.gamma * w.p * sy.v + w.v * sy.p;
      mu += P.g_y * l[2] * u0 - 0.5 * P.inv_dx * (qb.r * axr + qb.u * axu + qb.v * axv + qb.p * axp) -
            0.5 * P.inv_dy * (qb.r * ayr + qb.u * ayu + qb.v * ayv + qb.p * ayp) + 0.5 * P.g_y * qb.v;
    }
    // planes 0..3: the part of lambda^n the gather does not touch, in
    // conservative variables -- the primitive-map adjoint of this cell's
    // own primitive cotangent plus the identity and gravity terms of the
    // update (the map is linear in the cotangent, so the gather maps only
    // its slope terms and adds these)
    double ln[4];
    if constexpr (FOLD) {
      ln[0] = S.L[0][ly][lx];
      ln[1] = S.L[1][ly][lx];
      ln[2] = S.L[2][ly][lx];
      ln[3] = S.L[3][ly][lx];
    } else {
      ln[0] = ldg(Lm, c);
      ln[1] = ldg(Lm + N, c);
      ln[2] = ldg(Lm + 2 * N, c);
      ln[3] = ldg(Lm + 3 * N, c);
    }
    double ud[4];
    prim_adj(P, w, wb, ud);
    double* Z = a.Z + (size_t)b * 12 * N;
    stg(Z, c, ud[0] + ln[0] + dt * P.g_y * ln[2]);
    stg(Z + N, c, ud[1] + ln[1]);
    stg(Z + 2 * N, c, ud[2] + ln[2]);
    stg(Z + 3 * N, c, ud[3] + ln[3]);
    stg(Z + 4 * N, c, sxb.r);
    stg(Z + 5 * N, c, sxb.u);
    stg(Z + 6 * N, c, sxb.v);
    stg(Z + 7 * N, c, sxb.p);
    stg(Z + 8 * N, c, syb.r);
    stg(Z + 9 * N, c, syb.u);
    stg(Z + 10 * N, c, syb.v);
    stg(Z + 11 * N, c, syb.p);
  }
  if (bad) atomicOr(&a.flags->err_unphys, 1);
  if constexpr (DTD) {
    __shared__ double rmu[NT / 64], rsp[NT / 64];
    __shared__ int rix[NT / 64];
    double sp = -1.0;
    int ix = 0x7fffffff;
    if (own) {
      sp = signal_speed(P, u0, u1, u2, u3);
      ix = (int)c;
    }
    const double m = block_sum<NT>(mu, rmu);
    block_argmax<NT>(sp, ix, rsp, rix);
    if (tid == 0) {
      const size_t o = (size_t)b * a.dtd.stride + (size_t)tby * gridDim.x + tbx;
      a.dtd.mu[o] = m;
      a.dtd.smax[o] = sp;
      a.dtd.imax[o] = ix;
    }
  }
}

// ----------------------------------------------------------------- adjoint B
template <bool BAL>
__global__ __launch_bounds__(256) void k_adj_b(Params P, AdjArgs a) {
  const int nx = P.nx;
  const size_t N = (size_t)nx * P.ny;
  // rows in XCD bands, so that the rows above and below are in the same L2
  const uint32_t idx = (uint32_t)xcd_band((int)blockIdx.x, (int)gridDim.x) * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (idx >= N) return;
  GatherSrc g;
  g.Z = a.Z + (size_t)b * 12 * N;
  g.codes = a.codes + (size_t)b * N;
  g.U = a.U + (size_t)b * 4 * N;
  g.lam_next = a.lam_next + (size_t)b * 4 * N;
  g.pass = a.nsteps_limit && a.dt_index >= a.nsteps_limit[b];
  double l[4];
  lambda_at<BAL>(P, g, (int)(idx % nx), (int)(idx / nx), l);
  double* Lo = a.lam + (size_t)b * 4 * N;
  stg(Lo, idx, l[0]);
  stg(Lo + N, idx, l[1]);
  stg(Lo + 2 * N, idx, l[2]);
  stg(Lo + 3 * N, idx, l[3]);
}

// ----------------------------------------------------------------- step-size derivative
// The step n of member b is dt_n = cfl / S(U^n) unless it is the last one,
// which is T - t_n and so takes -1 times every earlier step's change.  The
// reverse sweep meets the last step first and keeps its mu; every earlier
// step adds (mu_n - mu_last) d dt_n / dU^n = (mu_n - mu_last) (-cfl / S^2)
// dS/dU at the one cell that holds the largest speed S.
__global__ __launch_bounds__(256) void k_dt_correct(Params P, AdjArgs a) {
  __shared__ double rm[4], rs[4];
  __shared__ int ri[4];
  const int b = blockIdx.x;
  const int n = a.dt_index, last = a.nsteps_limit[b] - 1;
  if (n > last) return;
  const size_t o = (size_t)b * a.dtd.stride;
  double m = 0.0, sp = -1.0;
  int ix = 0x7fffffff;
  for (int k = threadIdx.x; k < a.dtd.count; k += 256) {
    m += a.dtd.mu[o + k];
    argmax_merge(sp, ix, a.dtd.smax[o + k], a.dtd.imax[o + k]);
  }
  m = block_sum<256>(m, rm);
  block_argmax<256>(sp, ix, rs, ri);
  if (threadIdx.x != 0) return;
  if (n == last) {
    a.dtd.mu_last[b] = m;
    return;
  }
  const size_t N = (size_t)P.nx * P.ny;
  if (ix < 0 || (size_t)ix >= N) return;
  const double* U = a.U + (size_t)b * 4 * N;
  double d[4];
  const double S = signal_speed_grad(P, U[ix], U[N + ix], U[2 * N + ix], U[3 * N + ix], d);
  const double coef = (m - a.dtd.mu_last[b]) * (-P.cfl / (S * S));
  double* L = a.lam + (size_t)b * 4 * N;
  L[ix] += coef * d[0];
  L[N + ix] += coef * d[1];
  L[2 * N + ix] += coef * d[2];
  L[3 * N + ix] += coef * d[3];
}

// ----------------------------------------------------------------- small kernels
// Background pressure of the well-balanced variant, one value per row: the
// closed form at the bottom row's centre, then
// p_{j+1} = p_j + g_y dy (rho0_j + rho0_{j+1}) / 2 upward.  One thread.
__global__ void k_background_rows(Params P, double* prow) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double p = p0_at(P, 0.5 * P.dy);
  prow[0] = p;
  for (int j = 0; j + 1 < P.ny; ++j) {
    p = p + P.g_y * P.dy * (0.5 * (rho0_at(P, (j + 0.5) * P.dy) + rho0_at(P, (j + 1.5) * P.dy)));
    prow[j + 1] = p;
  }
}

// prow: the background pressure per row (well-balanced variant), or null
// for the closed form.
__global__ void k_init_state(Params P, const double* uv0, double* U, const double* prow) {
  const size_t N = (size_t)P.nx * P.ny;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (idx >= N) return;
  const int j = (int)(idx / P.nx);
  const double y = (j + 0.5) * P.dy;
  const double r = rho0_at(P, y), p = prow ? prow[j] : p0_at(P, y);
  const double* q = uv0 + (size_t)b * 2 * N;
  const double u = (P.comp_mask & 1) ? q[idx] : 0.0;
  const double v = (P.comp_mask & 2) ? q[N + idx] : 0.0;
  double* o = U + (size_t)b * 4 * N;
  o[idx] = r;
  o[N + idx] = r * u;
  o[2 * N + idx] = r * v;
  o[3 * N + idx] = p * P.inv_gm1 + 0.5 * r * (u * u + v * v);
}

// Per-member reduction, pass 1.  kind: 0 max signal speed of a state;
// 1 kinetic energy sum of a state; 2/3/4 weighted |uv|^2 of a velocity field
// (weights 1, 1, rho0/2) honouring comp_mask; 5 dot product of two velocity
// fields; 6 largest magnitude of a velocity field.
__global__ __launch_bounds__(256) void k_reduce_partial(Params P, int kind, const double* A, const double* Bv,
                                                        double* partial) {
  __shared__ double red[4];
  const size_t N = (size_t)P.nx * P.ny;
  const int b = blockIdx.y;
  const int nblk = gridDim.x;
  double acc = 0.0;
  if (kind == 0 || kind == 1) {
    const double* U = A + (size_t)b * 4 * N;
    for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < N; c += (size_t)nblk * 256) {
      if (kind == 0) {
        acc = fmax(acc, signal_speed(P, U[c], U[N + c], U[2 * N + c], U[3 * N + c]));
      } else {
        const double mx = U[N + c], my = U[2 * N + c];
        acc += 0.5 * (mx * mx + my * my) / U[c];
      }
    }
  } else if (kind <= 4) {
    const double* q = A + (size_t)b * 2 * N;
    const bool mu = (P.comp_mask & 1) != 0, mv = (P.comp_mask & 2) != 0;
    for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < N; c += (size_t)nblk * 256) {
      const double u = mu ? q[c] : 0.0, v = mv ? q[N + c] : 0.0;
      double w = 1.0;
      if (kind == 4) w = 0.5 * rho0_at(P, ((int)(c / P.nx) + 0.5) * P.dy);
      acc += w * (u * u + v * v);
    }
  } else if (kind == 7) {
    // (e_k(U) - e_k,base)^2 summed over the cells (objective of Eq. 8)
    const double* U = A + (size_t)b * 4 * N;
    const double* ekb = Bv + (size_t)b * N;
    for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < N; c += (size_t)nblk * 256) {
      const double mx = U[N + c], my = U[2 * N + c];
      const double d = 0.5 * (mx * mx + my * my) / U[c] - ekb[c];
      acc += d * d;
    }
  } else if (kind == 5) {
    const double* x = A + (size_t)b * 2 * N;
    const double* y = Bv + (size_t)b * 2 * N;
    for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < 2 * N; c += (size_t)nblk * 256) acc += x[c] * y[c];
  } else {
    const double* x = A + (size_t)b * 2 * N;
    for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < 2 * N; c += (size_t)nblk * 256)
      acc = fmax(acc, fabs(x[c]));
  }
  const bool is_max = kind == 0 || kind == 6;
  const double r = is_max ? block_max<256>(acc, red) : block_sum<256>(acc, red);
  if (threadIdx.x == 0) partial[(size_t)b * nblk + blockIdx.x] = r;
}

// Pass 2: one block per member combines the partials in a fixed order.
__global__ __launch_bounds__(256) void k_reduce_final(Params P, int kind, const double* partial, int nblk,
                                                      double* out) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  double acc = 0.0;
  const bool is_max = kind == 0 || kind == 6;
  for (int k = threadIdx.x; k < nblk; k += 256) {
    const double v = partial[(size_t)b * nblk + k];
    acc = is_max ? fmax(acc, v) : acc + v;
  }
  const double r = is_max ? block_max<256>(acc, red) : block_sum<256>(acc, red);
  if (threadIdx.x != 0) return;
  const double dV = P.dx * P.dy;
  const double N = (double)P.nx * (double)P.ny;
  switch (kind) {
    case 0: out[b] = r; break;             // max signal speed
    case 1: out[b] = r * dV; break;        // kinetic energy
    case 2: out[b] = sqrt(r * dV); break;  // velocity L2 norm
    case 3: out[b] = sqrt(r / N); break;   // RMS
    case 4: out[b] = r * dV; break;        // energy C of Eq. 9
    case 7: out[b] = r * dV; break;        // objective of Eq. 8
    default: out[b] = r; break;            // dot product
  }
}

__global__ void k_march_begin(Params P, const double* ms, double T, Ctl* ctl, uint64_t* acc, Flags* flags) {
  const int b = threadIdx.x + blockIdx.x * blockDim.x;
  if (b == 0) flags->n_active = P.nb;
  if (b >= P.nb) return;
  Ctl c;
  c.t = 0.0;
  c.T = T;
  c.dt_last = 0.0;
  c.nsteps = 0;
  c.done = 0;
  ctl[b] = c;
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < kAccSlots; ++k)
      acc[((size_t)r * P.nb + b) * kAccRow + k * kAccStride] =
          (r == 0 && k == 0) ? (uint64_t)__double_as_longlong(ms[b]) : 0ull;
}

__global__ void k_cfl_from_bits(Params P, const uint64_t* acc, double* dt) {
  const int b = threadIdx.x + blockIdx.x * blockDim.x;
  if (b < P.nb) dt[b] = P.cfl / __longlong_as_double((long long)acc[b]);
}

__global__ void k_cfl_from_speed(Params P, const double* ms, double* dt) {
  const int b = threadIdx.x + blockIdx.x * blockDim.x;
  if (b < P.nb) dt[b] = P.cfl / ms[b];
}

__global__ void k_copy_final(Params P, const Ctl* ctl, const double* A, const double* Bb, double* U) {
  const size_t N4 = (size_t)4 * P.nx * P.ny;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (idx >= N4) return;
  const double* src = (ctl[b].nsteps & 1) ? Bb : A;
  U[(size_t)b * N4 + idx] = src[(size_t)b * N4 + idx];
}

__global__ void k_copy_meta(Params, const Ctl* ctl, double* t_out, int32_t* n_out, const double* ls, int32_t lcap,
                            double* ld, int32_t dcap) {
  const int b = blockIdx.x;
  const int n = ctl[b].nsteps;
  if (threadIdx.x == 0) {
    if (t_out) t_out[b] = ctl[b].t;
    if (n_out) n_out[b] = n;
  }
  if (ld && ls) {
    int m = n < dcap ? n : dcap;
    m = m < lcap ? m : lcap;
    for (int k = threadIdx.x; k < m; k += blockDim.x) ld[(size_t)b * dcap + k] = ls[(size_t)b * lcap + k];
  }
}

__global__ void k_copy(const double* src, double* dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_fill_i32(int32_t* p, int32_t v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// lambda^N = dR/dU^N = (1/KE0) (-|m|^2/(2 rho^2), m_x/rho, m_y/rho, 0) dV.
__global__ void k_terminal_adjoint(Params P, const double* U, const double* ke0, double* lam) {
  const size_t N = (size_t)P.nx * P.ny;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (idx >= N) return;
  const double* u = U + (size_t)b * 4 * N;
  double* l = lam + (size_t)b * 4 * N;
  const double s = P.dx * P.dy / ke0[b];
  const double ri = 1.0 / u[idx];
  const double vx = u[N + idx] * ri, vy = u[2 * N + idx] * ri;
  l[idx] = -0.5 * (vx * vx + vy * vy) * s;
  l[N + idx] = vx * s;
  l[2 * N + idx] = vy * s;
  l[3 * N + idx] = 0.0;
}

// Terminal adjoint of J (Eq. 8): 2 (e_k - e_k,base) dV times de_k/dU =
// (-(u^2 + v^2)/2, u, v, 0).
__global__ void k_terminal_adjoint_ek(Params P, const double* U, const double* ek_base, double* lam) {
  const size_t N = (size_t)P.nx * P.ny;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (idx >= N) return;
  const double* u = U + (size_t)b * 4 * N;
  double* l = lam + (size_t)b * 4 * N;
  const double mx = u[N + idx], my = u[2 * N + idx];
  const double ri = 1.0 / u[idx];
  const double vx = mx * ri, vy = my * ri;
  // e_k exactly as the field and the objective compute it, so that the
  // unperturbed run gives a zero terminal adjoint
  const double ek = 0.5 * (mx * mx + my * my) / u[idx];
  const double w = 2.0 * (ek - ek_base[(size_t)b * N + idx]) * (P.dx * P.dy);
  l[idx] = -0.5 * (vx * vx + vy * vy) * w;
  l[N + idx] = vx * w;
  l[2 * N + idx] = vy * w;
  l[3 * N + idx] = 0.0;
}

// Gradient of an objective that depends on uv0 only through U^0:
// grad_u = rho0 (lam_mx + u0 lam_E) (and v), masked components zero.
__global__ void k_initial_adjoint_plain(Params P, const double* uv0, const double* lam0, double* grad) {
  const size_t N = (size_t)P.nx * P.ny;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (idx >= N) return;
  const int j = (int)(idx / P.nx);
  const double r0 = rho0_at(P, (j + 0.5) * P.dy);
  const double* q = uv0 + (size_t)b * 2 * N;
  const double* l = lam0 + (size_t)b * 4 * N;
  double* g = grad + (size_t)b * 2 * N;
  const double u = (P.comp_mask & 1) ? q[idx] : 0.0;
  const double v = (P.comp_mask & 2) ? q[N + idx] : 0.0;
  g[idx] = (P.comp_mask & 1) ? r0 * (l[N + idx] + u * l[3 * N + idx]) : 0.0;
  g[N + idx] = (P.comp_mask & 2) ? r0 * (l[2 * N + idx] + v * l[3 * N + idx]) : 0.0;
}

// Mixing width (Eqs. 13-14), pass 1: the horizontal mean of the density of
// every row, rowmean[B][ny]; one block per row, fixed summation order.
__global__ __launch_bounds__(256) void k_row_mean(Params P, const double* U, double* rowmean) {
  __shared__ double red[4];
  const int j = blockIdx.x, b = blockIdx.y;
  const size_t N = (size_t)P.nx * P.ny;
  const double* r = U + (size_t)b * 4 * N + (size_t)j * P.nx;
  double s = 0.0;
  for (int i = threadIdx.x; i < P.nx; i += 256) s += r[i];
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) rowmean[(size_t)b * P.ny + j] = s / P.nx;
}

// Pass 2: h_mix = sum over rows of 4 f (1 - f) dy with
// f = clip((<rho>_x - rho_l)/(rho_h - rho_l), 0, 1); one block per member.
__global__ __launch_bounds__(256) void k_mix_width(Params P, const double* rowmean, double* h) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  const double inv = 1.0 / (P.rho_h - P.rho_l);
  double s = 0.0;
  for (int j = threadIdx.x; j < P.ny; j += 256) {
    double f = (rowmean[(size_t)b * P.ny + j] - P.rho_l) * inv;
    f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
    s += 4.0 * f * (1.0 - f);
  }
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) h[b] = s * P.dy;
}

// e_k = |m|^2 / (2 rho) of every cell, [B][ny][nx].
__global__ void k_ek_field(Params P, const double* U, double* ek) {
  const size_t N = (size_t)P.nx * P.ny;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (idx >= N) return;
  const double* u = U + (size_t)b * 4 * N;
  const double mx = u[N + idx], my = u[2 * N + idx];
  ek[(size_t)b * N + idx] = 0.5 * (mx * mx + my * my) / u[idx];
}

// grad_u = rho0 (lam_mx + u0 lam_E) - (R/KE0) rho0 u0 dV (and v), R = KE_N/KE0.
__global__ void k_initial_adjoint(Params P, const double* uv0, const double* lam0, const double* ke0,
                                  const double* keN, double* R, double* grad) {
  const size_t N = (size_t)P.nx * P.ny;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (idx >= N) return;
  const double Rb = keN[b] / ke0[b];
  if (idx == 0 && R) R[b] = Rb;
  const int j = (int)(idx / P.nx);
  const double r0 = rho0_at(P, (j + 0.5) * P.dy);
  const double* q = uv0 + (size_t)b * 2 * N;
  const double* l = lam0 + (size_t)b * 4 * N;
  double* g = grad + (size_t)b * 2 * N;
  const double k = Rb / ke0[b] * P.dx * P.dy;
  const double u = (P.comp_mask & 1) ? q[idx] : 0.0;
  const double v = (P.comp_mask & 2) ? q[N + idx] : 0.0;
  g[idx] = (P.comp_mask & 1) ? r0 * (l[N + idx] + u * l[3 * N + idx]) - k * r0 * u : 0.0;
  g[N + idx] = (P.comp_mask & 2) ? r0 * (l[2 * N + idx] + v * l[3 * N + idx]) - k * r0 * v : 0.0;
}

__global__ void k_scale_project(Params P, double* uv, const double* m, double delta, int norm, int set) {
  const size_t N = (size_t)P.nx * P.ny;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (idx >= N) return;
  const double mb = m[b];
  double s = norm == 2 ? sqrt(delta / mb) : delta / mb;
  if (set == 1 && mb <= delta) s = 1.0;
  double* q = uv + (size_t)b * 2 * N;
  q[idx] = (P.comp_mask & 1) ? q[idx] * s : 0.0;
  q[N + idx] = (P.comp_mask & 2) ? q[N + idx] * s : 0.0;
}

__global__ void k_axpy(Params P, const double* x, const double* alpha, const double* y, double* out) {
  const size_t N2 = (size_t)2 * P.nx * P.ny;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (idx >= N2) return;
  const size_t o = (size_t)b * N2 + idx;
  out[o] = x[o] + alpha[b] * y[o];
}

__global__ void k_ratio(int nb, const double* num, const double* den, double* out) {
  const int b = threadIdx.x + blockIdx.x * blockDim.x;
  if (b < nb) out[b] = num[b] / den[b];
}

inline dim3 cells_grid(const Params& P, size_t per_member) {
  return dim3((unsigned)((per_member + 255) / 256), (unsigned)P.nb, 1);
}

}  // namespace

void tile_dims(int tile, int* tx, int* ty, int* nt) {
  int a = 16, b = 16, t = 256;
  switch (tile) {
    case TILE_32x8: a = 32; b = 8; break;
    case TILE_64x4: a = 64; b = 4; break;
    case TILE_16x16W: t = 576; break;
    case TILE_32x8W: a = 32; b = 8; t = 576; break;
    case TILE_16x8: b = 8; t = 128; break;
    case TILE_8x8: a = 8; b = 8; t = 64; break;
    case TILE_16x8W: b = 8; t = 320; break;
    case TILE_8x8W: a = 8; b = 8; t = 192; break;
    case TILE_32x16: a = 32; b = 16; t = 512; break;
    case TILE_16x15: b = 15; break;
    case TILE_15x16: a = 15; break;
    default: break;
  }
  *tx = a;
  *ty = b;
  if (nt) *nt = t;
}

int step_blocks(const Params& P, int tile) {
  int tx, ty;
  tile_dims(tile, &tx, &ty, nullptr);
  return ((P.nx + tx - 1) / tx) * ((P.ny + ty - 1) / ty);
}

#ifndef RT_ALIAS_MODE
#define RT_ALIAS_MODE 2
#endif
template <int TX, int TY, int NT>
static hipError_t launch_step_t(const Params& P, const StepArgs& a, hipStream_t s) {
  dim3 grid((P.nx + TX - 1) / TX, (P.ny + TY - 1) / TY, P.nb);
  const long blocks = (long)grid.x * grid.y * grid.z;
  // the separate-buffer layout fits min(3, 160 KiB / its size) blocks per CU
  const long per_cu = std::min(3L, 163840L / (long)sizeof(StepLDS<TX, TY, false>));
  const bool alias = RT_ALIAS_MODE == 1 || (RT_ALIAS_MODE == 2 && blocks > per_cu * 256);
  if (P.recon == 1) {
    if (alias)
      hipLaunchKernelGGL((k_step<TX, TY, NT, true, true>), grid, dim3(NT), 0, s, P, a);
    else
      hipLaunchKernelGGL((k_step<TX, TY, NT, true, false>), grid, dim3(NT), 0, s, P, a);
  } else {
    if (alias)
      hipLaunchKernelGGL((k_step<TX, TY, NT, false, true>), grid, dim3(NT), 0, s, P, a);
    else
      hipLaunchKernelGGL((k_step<TX, TY, NT, false, false>), grid, dim3(NT), 0, s, P, a);
  }
  return hipGetLastError();
}

hipError_t launch_step(const Params& P, int tile, const StepArgs& a, hipStream_t s) {
  switch (tile) {
    case TILE_32x8: return launch_step_t<32, 8, 256>(P, a, s);
    case TILE_64x4: return launch_step_t<64, 4, 256>(P, a, s);
    case TILE_16x16W: return launch_step_t<16, 16, 576>(P, a, s);
    case TILE_32x8W: return launch_step_t<32, 8, 576>(P, a, s);
    case TILE_16x8: return launch_step_t<16, 8, 128>(P, a, s);
    case TILE_8x8: return launch_step_t<8, 8, 64>(P, a, s);
    case TILE_16x8W: return launch_step_t<16, 8, 320>(P, a, s);
    case TILE_8x8W: return launch_step_t<8, 8, 192>(P, a, s);
    case TILE_32x16: return launch_step_t<32, 16, 512>(P, a, s);
    case TILE_16x15: return launch_step_t<16, 15, 256>(P, a, s);
    case TILE_15x16: return launch_step_t<15, 16, 256>(P, a, s);
    default: return launch_step_t<16, 16, 256>(P, a, s);
  }
}

template <int TX, int TY, int NT>
static hipError_t launch_adj_t(const Params& P, const AdjArgs& a, hipStream_t s) {
  dim3 grid((P.nx + TX - 1) / TX, (P.ny + TY - 1) / TY, P.nb);
  const bool bal = P.recon == 1;
  if (a.fold.Z != nullptr && (bal || a.dtd.mu != nullptr)) return hipErrorInvalidValue;
  if (a.dtd.mu != nullptr) {
    if (a.dtd.count != (int)(grid.x * grid.y) || a.dtd.stride < a.dtd.count) return hipErrorInvalidValue;
    if (bal)
      hipLaunchKernelGGL((k_adj_a<TX, TY, NT, false, true, true>), grid, dim3(NT), 0, s, P, a);
    else
      hipLaunchKernelGGL((k_adj_a<TX, TY, NT, false, true, false>), grid, dim3(NT), 0, s, P, a);
  } else if (a.fold.Z != nullptr) {
    hipLaunchKernelGGL((k_adj_a<TX, TY, NT, true, false, false>), grid, dim3(NT), 0, s, P, a);
  } else if (bal) {
    hipLaunchKernelGGL((k_adj_a<TX, TY, NT, false, false, true>), grid, dim3(NT), 0, s, P, a);
  } else {
    hipLaunchKernelGGL((k_adj_a<TX, TY, NT, false, false, false>), grid, dim3(NT), 0, s, P, a);
  }
  return hipGetLastError();
}

hipError_t launch_adj_gather(const Params& P, const AdjArgs& a, hipStream_t s) {
  if (P.recon == 1)
    hipLaunchKernelGGL(k_adj_b<true>, cells_grid(P, (size_t)P.nx * P.ny), dim3(256), 0, s, P, a);
  else
    hipLaunchKernelGGL(k_adj_b<false>, cells_grid(P, (size_t)P.nx * P.ny), dim3(256), 0, s, P, a);
  return hipGetLastError();
}

hipError_t launch_dt_correct(const Params& P, const AdjArgs& a, hipStream_t s) {
  if (!a.dtd.mu || !a.dtd.smax || !a.dtd.imax || !a.dtd.mu_last || !a.nsteps_limit || a.dtd.count < 1 ||
      a.dtd.stride < a.dtd.count)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dt_correct, dim3(P.nb), dim3(256), 0, s, P, a);
  return hipGetLastError();
}

static hipError_t launch_adj_a(const Params& P, int tile, const AdjArgs& a, hipStream_t s) {
  switch (tile) {
    case TILE_32x8: return launch_adj_t<32, 8, 256>(P, a, s);
    case TILE_64x4: return launch_adj_t<64, 4, 256>(P, a, s);
    case TILE_16x16W: return launch_adj_t<16, 16, 576>(P, a, s);
    case TILE_32x8W: return launch_adj_t<32, 8, 576>(P, a, s);
    case TILE_16x8: return launch_adj_t<16, 8, 128>(P, a, s);
    case TILE_8x8: return launch_adj_t<8, 8, 64>(P, a, s);
    case TILE_16x8W: return launch_adj_t<16, 8, 320>(P, a, s);
    case TILE_8x8W: return launch_adj_t<8, 8, 192>(P, a, s);
    case TILE_32x16: return launch_adj_t<32, 16, 512>(P, a, s);
    case TILE_16x15: return launch_adj_t<16, 15, 256>(P, a, s);
    case TILE_15x16: return launch_adj_t<15, 16, 256>(P, a, s);
    default: return launch_adj_t<16, 16, 256>(P, a, s);
  }
}

hipError_t launch_adjoint(const Params& P, int tile, const AdjArgs& a, hipStream_t s, bool gather) {
  hipError_t e = launch_adj_a(P, tile, a, s);
  if (e != hipSuccess || !gather) return e;
  return launch_adj_gather(P, a, s);
}

hipError_t launch_background_rows(const Params& P, double* prow, hipStream_t s) {
  hipLaunchKernelGGL(k_background_rows, dim3(1), dim3(64), 0, s, P, prow);
  return hipGetLastError();
}

hipError_t launch_init_state(const Params& P, const double* uv0, double* U, const double* prow, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, cells_grid(P, (size_t)P.nx * P.ny), dim3(256), 0, s, P, uv0, U, prow);
  return hipGetLastError();
}

hipError_t launch_reduce(const Params& P, int kind, const double* a, const double* b, double* partial, int nblk,
                         double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_partial, dim3(nblk, P.nb), dim3(256), 0, s, P, kind, a, b, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3(P.nb), dim3(256), 0, s, P, kind, partial, nblk, out);
  return hipGetLastError();
}

hipError_t launch_march_begin(const Params& P, const double* ms, double T, Ctl* ctl, uint64_t* acc, Flags* flags,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_march_begin, dim3((P.nb + 63) / 64), dim3(64), 0, s, P, ms, T, ctl, acc, flags);
  return hipGetLastError();
}

hipError_t launch_cfl_from_bits(const Params& P, const uint64_t* acc, double* dt, hipStream_t s) {
  hipLaunchKernelGGL(k_cfl_from_bits, dim3((P.nb + 63) / 64), dim3(64), 0, s, P, acc, dt);
  return hipGetLastError();
}

hipError_t launch_cfl_from_speed(const Params& P, const double* ms, double* dt, hipStream_t s) {
  hipLaunchKernelGGL(k_cfl_from_speed, dim3((P.nb + 63) / 64), dim3(64), 0, s, P, ms, dt);
  return hipGetLastError();
}

hipError_t launch_copy_final(const Params& P, const Ctl* ctl, const double* A, const double* Bbuf, double* U,
                             double* t_out, int32_t* nsteps_out, const double* log_src, int32_t log_src_cap,
                             double* log_dst, int32_t log_dst_cap, hipStream_t s) {
  if (U) {
    hipLaunchKernelGGL(k_copy_final, cells_grid(P, (size_t)4 * P.nx * P.ny), dim3(256), 0, s, P, ctl, A, Bbuf, U);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_copy_meta, dim3(P.nb), dim3(256), 0, s, P, ctl, t_out, nsteps_out, log_src, log_src_cap,
                     log_dst, log_dst_cap);
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_terminal_adjoint(const Params& P, const double* U, const double* ke0, double* lam, hipStream_t s) {
  hipLaunchKernelGGL(k_terminal_adjoint, cells_grid(P, (size_t)P.nx * P.ny), dim3(256), 0, s, P, U, ke0, lam);
  return hipGetLastError();
}

hipError_t launch_initial_adjoint(const Params& P, const double* uv0, const double* lam0, const double* ke0,
                                  const double* keN, double* R, double* grad, hipStream_t s) {
  hipLaunchKernelGGL(k_initial_adjoint, cells_grid(P, (size_t)P.nx * P.ny), dim3(256), 0, s, P, uv0, lam0, ke0,
                     keN, R, grad);
  return hipGetLastError();
}

hipError_t launch_terminal_adjoint_ek(const Params& P, const double* U, const double* ek_base, double* lam,
                                      hipStream_t s) {
  hipLaunchKernelGGL(k_terminal_adjoint_ek, cells_grid(P, (size_t)P.nx * P.ny), dim3(256), 0, s, P, U, ek_base,
                     lam);
  return hipGetLastError();
}

hipError_t launch_initial_adjoint_plain(const Params& P, const double* uv0, const double* lam0, double* grad,
                                       hipStream_t s) {
  hipLaunchKernelGGL(k_initial_adjoint_plain, cells_grid(P, (size_t)P.nx * P.ny), dim3(256), 0, s, P, uv0, lam0,
                     grad);
  return hipGetLastError();
}

hipError_t launch_mix_width(const Params& P, const double* U, double* rowmean, double* h, hipStream_t s) {
  hipLaunchKernelGGL(k_row_mean, dim3((unsigned)P.ny, (unsigned)P.nb), dim3(256), 0, s, P, U, rowmean);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mix_width, dim3((unsigned)P.nb), dim3(256), 0, s, P, rowmean, h);
  return hipGetLastError();
}

hipError_t launch_ek_field(const Params& P, const double* U, double* ek, hipStream_t s) {
  hipLaunchKernelGGL(k_ek_field, cells_grid(P, (size_t)P.nx * P.ny), dim3(256), 0, s, P, U, ek);
  return hipGetLastError();
}

hipError_t launch_scale_project(const Params& P, double* uv, const double* m, double delta, int norm, int set,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_scale_project, cells_grid(P, (size_t)P.nx * P.ny), dim3(256), 0, s, P, uv, m, delta, norm,
                     set);
  return hipGetLastError();
}

hipError_t launch_axpy(const Params& P, const double* x, const double* alpha, const double* y, double* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, cells_grid(P, (size_t)2 * P.nx * P.ny), dim3(256), 0, s, P, x, alpha, y, out);
  return hipGetLastError();
}

hipError_t launch_ratio(int nb, const double* num, const double* den, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_ratio, dim3((nb + 63) / 64), dim3(64), 0, s, nb, num, den, out);
  return hipGetLastError();
}

}  // namespace rtk
