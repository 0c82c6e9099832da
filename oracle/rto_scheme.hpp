// Oracle (test infrastructure only): the forward scheme, written once and
// templated on the scalar type (double, Dual or Rev from rto_ad.hpp).
//
// What it computes, and where it comes from:
//   * 2-D compressible Euler equations with uniform gravity g = (0, g_y):
//     mass, momentum and energy in conservative form with the sources rho*g
//     and rho*u.g (Sec. 2.1, Eqs. 1-3), ideal-gas closure
//     E = p/(gamma-1) + rho|u|^2/2 (Eq. 4).
//   * Periodic in x; in y the paper asks for hydrostatic boundaries
//     (dp/dy = -rho g, Sec. 2.1) and the workload asks for reflecting walls.
//     Both are honoured: ghost cells mirror the adjacent interior cell with
//     the normal velocity negated and the pressure extrapolated
//     hydrostatically, and the flux through the wall face is set to the
//     wall-pressure flux (0, 0, p*, 0) of the mirrored Riemann problem.
//   * A finite-volume Godunov-type scheme with an HLLC Riemann solver and a
//     gravity source (Sec. 2.3).  The paper names neither the reconstruction
//     nor the time integrator; this is the unsplit primitive-variable
//     MUSCL-Hancock scheme with piecewise-linear, monotonized-central (MC)
//     limited slopes (differences below a relative tolerance of the local
//     scale count as zero, 1e-10 for the workloads; Problem::tie_tol), and the
//     plain HLLC flux with Davis wave-speed bounds
//     (the "hybrid" qualifier in Sec. 2.3 is not explained there, so no HLL
//     switch is applied).
//   * Gravity source, second order in time and chosen so that total energy
//     including the potential energy rho*phi (phi = -g_y y) is conserved to
//     round-off: the y-momentum gains dt g_y (rho^n + rho^{n+1})/2, the
//     energy gains dt g_y times the mean of the two y mass fluxes of the cell.
//   * Time step from the CFL condition on the state at the start of the step,
//     dt = CFL / max over cells of max((|u|+c)/dx, (|v|+c)/dy), the last step
//     clipped so that the run ends exactly at T.
//   * Optional well-balanced variant (recon = 1; an extension, the paper
//     instead subtracts an unperturbed run): the background pressure is
//     built row by row so that p_{j+1} - p_j = g_y dy (rho_j + rho_{j+1})/2,
//     and the y slope of the pressure is the local hydrostatic slope of the
//     cell's own density plus a limited slope of the departures from it.
//     The unperturbed state is then kept to round-off: the departures vanish
//     or change sign (monotone density), the two face pressures agree, the
//     HLLC flux of a stationary contact is the pressure alone, and its
//     difference cancels the gravity source.
//
// Layout: a member's state is U[4][ny][nx] with variables
// (rho, m_x = rho u, m_y = rho v, E) and x fastest; members follow each other.
// Cell (i, j) has centre ((i+1/2) dx, (j+1/2) dy).
#pragma once
#include <array>
#include <cmath>
#include <type_traits>
#include <vector>

#include "rto_ad.hpp"

namespace rto {

struct Problem {
  int nx, ny, nb, comp_mask;  // comp_mask bit 0: u is perturbed, bit 1: v
  double lx, ly;              // domain [0, lx] x [0, ly]
  double gamma, g_y;          // adiabatic index, gravity (negative: downward)
  double rho_h, rho_l, y0, h; // two-layer profile (Sec. 2.2, Eq. 5)
  double p_int;               // pressure at the interface height y0
  double cfl;
  int recon, pad;             // recon 1: well-balanced variant (see above)
  double tie_tol;             // relative tie tolerance of the discrete decisions (see below); 0: none
};

inline double dx_of(const Problem& P) { return P.lx / P.nx; }
inline double dy_of(const Problem& P) { return P.ly / P.ny; }
inline double xc(const Problem& P, int i) { return (i + 0.5) * dx_of(P); }
inline double yc(const Problem& P, int j) { return (j + 0.5) * dy_of(P); }

// ------------------------------------------------------------ background state
// Eq. 5: rho0(y) = (rho_h + rho_l)/2 + (rho_h - rho_l)/2 tanh((y - y0)/h).
inline double rho0_at(const Problem& P, double y) {
  return 0.5 * (P.rho_h + P.rho_l) + 0.5 * (P.rho_h - P.rho_l) * std::tanh((y - P.y0) / P.h);
}
// log(cosh z) without overflow.
inline double log_cosh(double z) {
  const double a = std::fabs(z);
  return a + std::log1p(std::exp(-2.0 * a)) - std::log(2.0);
}
// Hydrostatic balance dp/dy = rho0 g_y (Sec. 2.2) integrated in closed form
// from the interface, where p = p_int:
//   p0(y) = p_int + g_y [ rbar (y - y0) + drho h log cosh((y - y0)/h) ].
inline double p0_at(const Problem& P, double y) {
  const double rbar = 0.5 * (P.rho_h + P.rho_l), drho = 0.5 * (P.rho_h - P.rho_l);
  return P.p_int + P.g_y * (rbar * (y - P.y0) + drho * P.h * log_cosh((y - P.y0) / P.h));
}

// Well-balanced variant: the background pressure of every row, the closed
// form at the bottom row's centre and then
// p_{j+1} = p_j + g_y dy (rho0_j + rho0_{j+1}) / 2 upward.
inline std::vector<double> p_background_rows(const Problem& P) {
  const double dy = dy_of(P);
  std::vector<double> p(P.ny);
  p[0] = p0_at(P, yc(P, 0));
  for (int j = 0; j + 1 < P.ny; ++j)
    p[j + 1] = p[j] + P.g_y * dy * (0.5 * (rho0_at(P, yc(P, j)) + rho0_at(P, yc(P, j + 1))));
  return p;
}

// Background pressure of row j in the selected variant.
inline double background_p(const Problem& P, int j) {
  return P.recon == 1 ? p_background_rows(P)[j] : p0_at(P, yc(P, j));
}

// ------------------------------------------------------------ primitive state
template <class T>
struct Prim {
  T r, u, v, p;
};

template <class T>
Prim<T> cons_to_prim(const Problem& P, const T& r, const T& mx, const T& my, const T& E) {
  Prim<T> w;
  w.r = r;
  w.u = mx / r;
  w.v = my / r;
  w.p = (P.gamma - 1.0) * (E - 0.5 * r * (w.u * w.u + w.v * w.v));
  return w;
}

template <class T>
bool bad_state(const Prim<T>& w) {
  const double r = val(w.r), p = val(w.p);
  return !(r > 0.0) || !(p > 0.0) || !std::isfinite(val(w.u)) || !std::isfinite(val(w.v));
}

// Problem::tie_tol is the relative tolerance below which a difference counts
// as zero when the scheme takes a discrete decision (limiter case, upwind
// side, wave-speed choice).  With 0 the decisions are the plain ones (MC
// with a*b <= 0 as the only zero case, Davis min/max, the sign of S*).  The
// workloads use 1e-10: decisions on differences at the level of round-off
// would otherwise be taken at random and make the discrete derivative of
// the march erratic (the linearisation of the compressive limiter branches
// amplifies grid-scale perturbations, so two correct implementations that
// differ by one ulp in a quiescent region would produce different
// gradients).  A slope or speed that the tolerance zeroes or switches was
// itself within that relative distance of zero or of the other case.

// Monotonized-central limited slope of one variable from its backward and
// forward differences a, b: zero at an extremum (a*b <= 0) or when either
// difference is negligible (`small(a)`), else the central difference (a+b)/2
// when it does not exceed 2|a| and 2|b|, else 2a if |a| <= |b|, else 2b.
template <class T, class Small>
T mc_slope(const T& a, const T& b, Small small) {
  const double va = val(a), vb = val(b);
  if (va * vb <= 0.0 || small(va) || small(vb)) return T(0.0);
  const T c = 0.5 * (a + b);
  const double ac = std::fabs(val(c)), aa = std::fabs(va), ab = std::fabs(vb);
  if (ac <= 2.0 * aa && ac <= 2.0 * ab) return c;
  if (aa <= ab) return 2.0 * a;
  return 2.0 * b;
}

// Slopes of the four primitives.  A difference is negligible below tie_tol
// times the cell's own density (density slope), pressure (pressure slope)
// or sound speed c = sqrt(gamma p / rho) (velocity slopes; compared as
// d^2 rho <= tie_tol^2 gamma p).
template <class T>
Prim<T> mc_slope(const Problem& P, const Prim<T>& wm, const Prim<T>& w, const Prim<T>& wp) {
  const double r = val(w.r), p = val(w.p), tol = P.tie_tol;
  const double tr = tol * r, tp = tol * p, tv2 = tol * tol * P.gamma * p;
  auto small_r = [tr](double d) { return std::fabs(d) <= tr; };
  auto small_p = [tp](double d) { return std::fabs(d) <= tp; };
  auto small_v = [tv2, r](double d) { return d * d * r <= tv2; };
  return Prim<T>{mc_slope(w.r - wm.r, wp.r - w.r, small_r), mc_slope(w.u - wm.u, wp.u - w.u, small_v),
                 mc_slope(w.v - wm.v, wp.v - w.v, small_v), mc_slope(w.p - wm.p, wp.p - w.p, small_p)};
}

// y slopes of the well-balanced variant: as mc_slope, except the pressure,
// which is the cell's hydrostatic slope h = rho g_y dy plus the limited slope
// of the departures from it, a' = (p - p_below) - h, b' = (p_above - p) - h.
template <class T>
Prim<T> mc_slope_y_balanced(const Problem& P, const Prim<T>& wm, const Prim<T>& w, const Prim<T>& wp) {
  Prim<T> s = mc_slope(P, wm, w, wp);
  const double tp = P.tie_tol * val(w.p);
  auto small_p = [tp](double d) { return std::fabs(d) <= tp; };
  const T h = w.r * (P.g_y * dy_of(P));
  s.p = h + mc_slope((w.p - wm.p) - h, (wp.p - w.p) - h, small_p);
  return s;
}

// Face-normal Riemann data: n is the normal velocity, t the tangential one.
template <class T>
struct FaceState {
  T r, n, t, p;
};

// HLLC flux (Toro, Spruce and Speares 1994) across a face with normal
// velocity n.  Returns (mass, normal momentum, tangential momentum, energy).
// Davis estimates S_L = min(n_L - c_L, n_R - c_R), S_R = max(n_L + c_L,
// n_R + c_R); contact speed S*; four cases S_L >= 0, S* >= 0, S_R > 0, else
// (a tie at S* = 0, within the tie tolerance, takes the left star state).
template <class T>
std::array<T, 4> hllc(const Problem& P, const FaceState<T>& L, const FaceState<T>& R) {
  const double gm = P.gamma;
  const T cL = sqrt(gm * L.p / L.r);
  const T cR = sqrt(gm * R.p / R.r);
  // Near-ties (within tie_tol of the sound speeds) resolve to the left state.
  const double tie = P.tie_tol * (val(cL) + val(cR));
  const T aL = L.n - cL, bL = R.n - cR;
  const T SL = val(aL) <= val(bL) + tie ? aL : bL;
  const T aR = L.n + cL, bR = R.n + cR;
  const T SR = val(aR) >= val(bR) - tie ? aR : bR;
  const T EL = L.p / (gm - 1.0) + 0.5 * L.r * (L.n * L.n + L.t * L.t);
  const T ER = R.p / (gm - 1.0) + 0.5 * R.r * (R.n * R.n + R.t * R.t);
  const T SS = (R.p - L.p + L.r * L.n * (SL - L.n) - R.r * R.n * (SR - R.n)) /
               (L.r * (SL - L.n) - R.r * (SR - R.n));
  const std::array<T, 4> FL = {L.r * L.n, L.r * L.n * L.n + L.p, L.r * L.n * L.t, L.n * (EL + L.p)};
  const std::array<T, 4> FR = {R.r * R.n, R.r * R.n * R.n + R.p, R.r * R.n * R.t, R.n * (ER + R.p)};
  if (val(SL) >= 0.0) return FL;
  if (val(SS) >= -tie) {
    const T f = L.r * (SL - L.n) / (SL - SS);
    const std::array<T, 4> Us = {f, f * SS, f * L.t,
                                 f * (EL / L.r + (SS - L.n) * (SS + L.p / (L.r * (SL - L.n))))};
    const std::array<T, 4> UL = {L.r, L.r * L.n, L.r * L.t, EL};
    return {FL[0] + SL * (Us[0] - UL[0]), FL[1] + SL * (Us[1] - UL[1]),
            FL[2] + SL * (Us[2] - UL[2]), FL[3] + SL * (Us[3] - UL[3])};
  }
  if (val(SR) > 0.0) {
    const T f = R.r * (SR - R.n) / (SR - SS);
    const std::array<T, 4> Us = {f, f * SS, f * R.t,
                                 f * (ER / R.r + (SS - R.n) * (SS + R.p / (R.r * (SR - R.n))))};
    const std::array<T, 4> UR = {R.r, R.r * R.n, R.r * R.t, ER};
    return {FR[0] + SR * (Us[0] - UR[0]), FR[1] + SR * (Us[1] - UR[1]),
            FR[2] + SR * (Us[2] - UR[2]), FR[3] + SR * (Us[3] - UR[3])};
  }
  return FR;
}

// Pressure at a reflecting wall: the HLLC star pressure of the Riemann problem
// between the interior face state and its mirror image (normal velocity
// negated).  For that problem S* = 0 and the HLLC flux reduces to
// (0, p*, 0, 0) in face-normal order.  `interior_left` is true at the top
// wall (the interior is below the face), false at the bottom wall.
template <class T>
T wall_pressure(const Problem& P, const FaceState<T>& w, bool interior_left) {
  const T c = sqrt(P.gamma * w.p / w.r);
  // |n|, with normal speeds within the tie tolerance of zero taken as >= 0
  const T an = val(w.n) < -P.tie_tol * val(c) ? -w.n : w.n;
  if (interior_left) return w.p + w.r * w.n * (an + c + w.n);
  return w.p - w.r * w.n * (an + c - w.n);
}

// MUSCL-Hancock half step of one cell in primitive variables: the
// quasi-linear form W_t + A_x(W) W_x + A_y(W) W_y = (0, 0, g_y, 0) of Eqs. 1-4
// advanced by dt/2 with the limited slopes sx, sy (per cell width) standing
// in for dx W_x, dy W_y:
//   A_x dW = (u dr + r du, u du + dp/r, u dv, gamma p du + u dp),
//   A_y dW = (v dr + r dv, v du, v dv + dp/r, gamma p dv + v dp).
template <class T, class D>
Prim<T> predict_half_step(const Problem& P, const Prim<T>& w, const Prim<T>& sx, const Prim<T>& sy, D dt) {
  const D hx = 0.5 * dt / dx_of(P), hy = 0.5 * dt / dy_of(P);
  Prim<T> q;
  q.r = w.r - hx * (w.u * sx.r + w.r * sx.u) - hy * (w.v * sy.r + w.r * sy.v);
  q.u = w.u - hx * (w.u * sx.u + sx.p / w.r) - hy * (w.v * sy.u);
  q.v = w.v - hx * (w.u * sx.v) - hy * (w.v * sy.v + sy.p / w.r) + 0.5 * dt * P.g_y;
  q.p = w.p - hx * (P.gamma * w.p * sx.u + w.u * sx.p) - hy * (P.gamma * w.p * sy.v + w.v * sy.p);
  return q;
}

// Threads over the rows of the double-precision step, for timing the oracle
// on several cores (1 unless rto_set_threads changes it; the AD types always
// run on one thread).  Every cell is computed as on one thread, so the
// result does not depend on the count.
inline int& omp_threads() {
  static int n = 1;
  return n;
}
template <class T, class D>
bool omp_rows() {
  return std::is_same<T, double>::value && std::is_same<D, double>::value && omp_threads() > 1;
}

// ------------------------------------------------------------------ one step
// Advance one member from U (4*ny*nx) to Un by dt.  Returns nonzero if a cell
// or face state is unphysical (rho <= 0, p <= 0, or not finite).  The step
// dt has its own scalar type D, so that reverse mode can also follow the
// dependence of the state on dt (a D other than double needs T == D).
template <class T, class D = double>
int step_member(const Problem& P, const T* U, T* Un, D dt) {
  const int nx = P.nx, ny = P.ny, N = nx * ny;
  const double dx = dx_of(P), dy = dy_of(P), g = P.g_y;
  int bad = 0;

  // Primitive variables with one ghost row below (row -1) and above (row ny).
  std::vector<Prim<T>> W(static_cast<size_t>(ny + 2) * nx);
  auto Wat = [&](int i, int j) -> Prim<T>& { return W[static_cast<size_t>(j + 1) * nx + i]; };
#pragma omp parallel for if (omp_rows<T, D>()) num_threads(omp_threads()) reduction(| : bad) schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int c = j * nx + i;
      Wat(i, j) = cons_to_prim(P, U[c], U[N + c], U[2 * N + c], U[3 * N + c]);
      if (bad_state(Wat(i, j))) bad = 1;
    }
  for (int i = 0; i < nx; ++i) {
    const Prim<T>& b = Wat(i, 0);
    Wat(i, -1) = Prim<T>{b.r, b.u, -b.v, b.p + g * b.r * (-dy)};
    const Prim<T>& t = Wat(i, ny - 1);
    Wat(i, ny) = Prim<T>{t.r, t.u, -t.v, t.p + g * t.r * dy};
  }

  // Limited slopes, MUSCL-Hancock half-step prediction, and the four face
  // states of every cell (x: left/right, y: bottom/top).
  std::vector<Prim<T>> xl(N), xr(N), yb(N), yt(N);
#pragma omp parallel for if (omp_rows<T, D>()) num_threads(omp_threads()) reduction(| : bad) schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const Prim<T>& w = Wat(i, j);
      const Prim<T> sx = mc_slope(P, Wat((i + nx - 1) % nx, j), w, Wat((i + 1) % nx, j));
      const Prim<T> sy = P.recon == 1 ? mc_slope_y_balanced(P, Wat(i, j - 1), w, Wat(i, j + 1))
                                      : mc_slope(P, Wat(i, j - 1), w, Wat(i, j + 1));
      const Prim<T> q = predict_half_step(P, w, sx, sy, dt);
      const int c = j * nx + i;
      xl[c] = Prim<T>{q.r - 0.5 * sx.r, q.u - 0.5 * sx.u, q.v - 0.5 * sx.v, q.p - 0.5 * sx.p};
      xr[c] = Prim<T>{q.r + 0.5 * sx.r, q.u + 0.5 * sx.u, q.v + 0.5 * sx.v, q.p + 0.5 * sx.p};
      yb[c] = Prim<T>{q.r - 0.5 * sy.r, q.u - 0.5 * sy.u, q.v - 0.5 * sy.v, q.p - 0.5 * sy.p};
      yt[c] = Prim<T>{q.r + 0.5 * sy.r, q.u + 0.5 * sy.u, q.v + 0.5 * sy.v, q.p + 0.5 * sy.p};
      if (bad_state(xl[c]) || bad_state(xr[c]) || bad_state(yb[c]) || bad_state(yt[c])) bad = 1;
    }

  // Fluxes.  F[j][i] is the x-flux through the left face of cell (i, j);
  // G[j][i] (j = 0..ny) is the y-flux through the bottom face of row j, with
  // G[0] and G[ny] at the walls.  Components: (rho, m_x, m_y, E).
  std::vector<std::array<T, 4>> F(N), G(static_cast<size_t>(ny + 1) * nx);
#pragma omp parallel for if (omp_rows<T, D>()) num_threads(omp_threads()) reduction(| : bad) schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const Prim<T>& a = xr[j * nx + (i + nx - 1) % nx];
      const Prim<T>& b = xl[j * nx + i];
      const std::array<T, 4> f = hllc(P, FaceState<T>{a.r, a.u, a.v, a.p}, FaceState<T>{b.r, b.u, b.v, b.p});
      F[j * nx + i] = {f[0], f[1], f[2], f[3]};
    }
#pragma omp parallel for if (omp_rows<T, D>()) num_threads(omp_threads()) reduction(| : bad) schedule(static)
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i < nx; ++i) {
      std::array<T, 4> gf;
      if (j == 0) {
        const Prim<T>& b = yb[i];
        gf = {T(0.0), T(0.0), wall_pressure(P, FaceState<T>{b.r, b.v, b.u, b.p}, false), T(0.0)};
      } else if (j == ny) {
        const Prim<T>& a = yt[(ny - 1) * nx + i];
        gf = {T(0.0), T(0.0), wall_pressure(P, FaceState<T>{a.r, a.v, a.u, a.p}, true), T(0.0)};
      } else {
        const Prim<T>& a = yt[(j - 1) * nx + i];
        const Prim<T>& b = yb[j * nx + i];
        const std::array<T, 4> f = hllc(P, FaceState<T>{a.r, a.v, a.u, a.p}, FaceState<T>{b.r, b.v, b.u, b.p});
        gf = {f[0], f[2], f[1], f[3]};  // normal momentum is m_y
      }
      G[static_cast<size_t>(j) * nx + i] = gf;
    }

  // Conservative update plus the gravity source.
  const D ax = dt / dx, ay = dt / dy;
#pragma omp parallel for if (omp_rows<T, D>()) num_threads(omp_threads()) reduction(| : bad) schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int c = j * nx + i;
      const std::array<T, 4>& Fl = F[c];
      const std::array<T, 4>& Fr = F[j * nx + (i + 1) % nx];
      const std::array<T, 4>& Gb = G[static_cast<size_t>(j) * nx + i];
      const std::array<T, 4>& Gt = G[static_cast<size_t>(j + 1) * nx + i];
      std::array<T, 4> u;
      for (int k = 0; k < 4; ++k) u[k] = U[k * N + c] - ax * (Fr[k] - Fl[k]) - ay * (Gt[k] - Gb[k]);
      u[2] = u[2] + dt * g * 0.5 * (U[c] + u[0]);
      u[3] = u[3] + dt * g * 0.5 * (Gb[0] + Gt[0]);
      for (int k = 0; k < 4; ++k) Un[k * N + c] = u[k];
    }
  return bad;
}

// Largest signal speed max((|u|+c)/dx, (|v|+c)/dy) over one member's cells;
// the first cell in storage order wins a tie, and within a cell the y speed
// wins a tie with the x speed.  With T = Rev the result carries the
// derivative of the selected cell's speed (the subgradient of that choice).
template <class T>
T max_signal_speed(const Problem& P, const T* U) {
  const int N = P.nx * P.ny;
  const double dx = dx_of(P), dy = dy_of(P);
  T m(0.0);
  for (int c = 0; c < N; ++c) {
    const Prim<T> w = cons_to_prim(P, U[c], U[N + c], U[2 * N + c], U[3 * N + c]);
    const T cs = sqrt(P.gamma * w.p / w.r);
    const T sx = (fabs(w.u) + cs) / dx, sy = (fabs(w.v) + cs) / dy;
    const T s = val(sx) > val(sy) ? sx : sy;
    if (val(s) > val(m)) m = s;
  }
  return m;
}

// Total kinetic energy sum over cells of (m_x^2 + m_y^2)/(2 rho) dx dy: the
// volume integral of Eq. 7 on the grid.
template <class T>
T kinetic_energy(const Problem& P, const T* U) {
  const int N = P.nx * P.ny;
  const double dV = dx_of(P) * dy_of(P);
  T s(0.0);
  for (int c = 0; c < N; ++c) s = s + 0.5 * (U[N + c] * U[N + c] + U[2 * N + c] * U[2 * N + c]) / U[c];
  return s * dV;
}

// Kinetic-energy density field of Eq. 7, e_k = rho |u|^2 / 2 = |m|^2 / (2 rho),
// cell by cell.
template <class T>
void ek_field(const Problem& P, const T* U, T* ek) {
  const int N = P.nx * P.ny;
  for (int c = 0; c < N; ++c) ek[c] = 0.5 * (U[N + c] * U[N + c] + U[2 * N + c] * U[2 * N + c]) / U[c];
}

// Objective of Eq. 8 on the grid: the volume integral of the squared
// departure of e_k(U) from the baseline field ek_base.
template <class T>
T ek_anomaly(const Problem& P, const T* U, const double* ek_base) {
  const int N = P.nx * P.ny;
  const double dV = dx_of(P) * dy_of(P);
  std::vector<T> ek(N);
  ek_field<T>(P, U, ek.data());
  T s(0.0);
  for (int c = 0; c < N; ++c) {
    const T d = ek[c] - ek_base[c];
    s = s + d * d;
  }
  return s * dV;
}

// Initial state of one member from the velocity perturbation (u0, v0) laid
// out [2][ny][nx]: the hydrostatic two-layer background (Sec. 2.2) plus the
// perturbation velocity, evaluated at cell centres (the pressure from
// p_background_rows in the well-balanced variant).  Components switched off
// by comp_mask are taken as zero.
template <class T>
void init_member(const Problem& P, const T* uv, T* U) {
  const int nx = P.nx, ny = P.ny, N = nx * ny;
  const bool use_u = (P.comp_mask & 1) != 0, use_v = (P.comp_mask & 2) != 0;
  const std::vector<double> pb = P.recon == 1 ? p_background_rows(P) : std::vector<double>();
  for (int j = 0; j < ny; ++j) {
    const double y = yc(P, j);
    const double r = rho0_at(P, y), p = P.recon == 1 ? pb[j] : p0_at(P, y);
    for (int i = 0; i < nx; ++i) {
      const int c = j * nx + i;
      const T u = use_u ? uv[c] : T(0.0);
      const T v = use_v ? uv[N + c] : T(0.0);
      U[c] = T(r);
      U[N + c] = r * u;
      U[2 * N + c] = r * v;
      U[3 * N + c] = p / (P.gamma - 1.0) + 0.5 * r * (u * u + v * v);
    }
  }
}

}  // namespace rto
