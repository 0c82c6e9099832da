// Oracle (test infrastructure only): plain, slow FP64 CPU implementation of
// the CNOP hot path, exported as a C ABI on host pointers for the tests.
// Nothing in the product path may link or call this library; it shares no
// code with the GPU implementation.
//
// Calls (all arrays host, contiguous, members stacked; return 0 or < 0):
//   rto_init_state     background + velocity perturbation -> U (Sec. 2.2, 3.1)
//   rto_cfl_dt         CFL time step of each member (unclipped)
//   rto_step           one step with a given dt per member (Sec. 2.1, 2.3)
//   rto_integrate      adaptive-dt march to exactly T, optional dt log
//   rto_kinetic_energy volume integral of Eq. 7
//   rto_step_jvp       exact tangent of one step (forward-mode AD)
//   rto_step_vjp       exact adjoint of one step (reverse-mode AD)
//   rto_grad_u0        R = KE(T)/KE(0) and its exact gradient with respect to
//                      the initial velocity field, by reverse-mode AD through
//                      the whole discrete march with the time steps of the
//                      forward run held fixed (Sec. 3.4)
//   rto_mix_width      mixing-layer width of Eqs. 13-14
//   rto_row_spectrum   horizontal power spectrum of rows (Eq. 12's E_n
//                      before normalisation)
//   rto_power_spectrum_2d  2-D power spectrum (App. B's reconstruction)
//   rto_ek_field       kinetic-energy density field of Eq. 7
//   rto_ek_anomaly_frozen  objective J of Eq. 8 after a march with given steps
//   rto_grad_ek_anomaly    J and its exact gradient (same reverse sweep as
//                      rto_grad_u0, terminal adjoint dJ/dU^N)
//   rto_objective_adaptive  R or J after the adaptive march (the map whose
//                      full derivative rto_grad_adaptive gives)
//   rto_grad_adaptive  R or J and its exact gradient through the adaptive
//                      march, the dependence of every CFL step on the state
//                      and of the clipped last step on the earlier ones
//                      included
//   rto_project_to_constraint  scaling onto the constraint set (Eq. 11)
//   rto_hllc, rto_wall_pressure  single-face fluxes for unit tests
//   rto_count_flops    algorithmic flops of one step (measurement only)
//   rto_mc_slope, rto_slopes, rto_predict  one limited slope (with its
//                      derivatives), the four slopes of a cell, and the
//                      MUSCL-Hancock half step of one cell, for unit tests
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "rto_ad.hpp"
#include "rto_count.hpp"
#include "rto_scheme.hpp"

namespace rto {
// One tape per thread, so that independent reverse-mode calls (the adjoints
// of separate members or blocks) may run on separate threads.
Tape& tape() {
  static thread_local Tape t;
  return t;
}
}  // namespace rto

using rto::Dual;
using rto::Problem;
using rto::Rev;

namespace {
constexpr int kEInval = -1;
constexpr int kENomem = -3;
constexpr int kEUnphys = -4;

bool valid(const Problem* P) {
  return P && P->nx >= 3 && P->ny >= 2 && P->nb >= 1 && P->lx > 0 && P->ly > 0 && P->gamma > 1.0 &&
         P->h > 0 && P->cfl > 0 && (P->recon == 0 || P->recon == 1) && P->tie_tol >= 0.0 && P->tie_tol < 1e-3;
}
size_t cells(const Problem* P) { return static_cast<size_t>(P->nx) * P->ny; }

// Reverse-mode adjoint of one step of one member: lam = (dUn/dU)^T lam_next.
int vjp_member(const Problem& P, const double* U, double dt, const double* lam_next, double* lam) {
  const size_t n4 = 4 * static_cast<size_t>(P.nx) * P.ny;
  rto::Tape& tp = rto::tape();
  tp.clear();
  std::vector<Rev> x(n4), y(n4);
  for (size_t k = 0; k < n4; ++k) x[k] = Rev::leaf(U[k]);
  const int bad = rto::step_member<Rev>(P, x.data(), y.data(), dt);
  tp.adj.assign(tp.nodes.size(), 0.0);
  for (size_t k = 0; k < n4; ++k)
    if (y[k].i >= 0) tp.adj[y[k].i] += lam_next[k];
  tp.sweep();
  for (size_t k = 0; k < n4; ++k) lam[k] = tp.adj[x[k].i];
  tp.clear();
  return bad;
}

// March one member to exactly T with the CFL step, the last step clipped.
// Optionally records every state (states != nullptr, appended) and every dt.
int integrate_member(const Problem& P, double* U, double T, double* t_out, int32_t* n_out,
                     std::vector<double>* dts, std::vector<std::vector<double>>* states) {
  const size_t n4 = 4 * cells(&P);
  std::vector<double> Un(n4);
  double t = 0.0;
  int32_t n = 0;
  bool last = false;
  int bad = 0;
  while (!last) {
    double dt = P.cfl / rto::max_signal_speed(P, U);
    const double rem = T - t;
    if (dt >= rem) {
      dt = rem;
      last = true;
    }
    if (states) states->emplace_back(U, U + n4);
    bad |= rto::step_member<double>(P, U, Un.data(), dt);
    std::memcpy(U, Un.data(), n4 * sizeof(double));
    t = last ? T : t + dt;
    if (dts) dts->push_back(dt);
    ++n;
    if (bad) break;
  }
  if (t_out) *t_out = t;
  if (n_out) *n_out = n;
  return bad ? kEUnphys : 0;
}

// Objective of one member at its final state: J of Eq. 8 when ek_base is
// given, else KE(U^N)/ke0.
double objective_value(const Problem& P, const double* U, const double* ek_base, double ke0) {
  if (ek_base) return rto::ek_anomaly<double>(P, U, ek_base);
  return rto::kinetic_energy<double>(P, U) / ke0;
}
}  // namespace

extern "C" {

int rto_init_state(const Problem* P, const double* uv0, double* U) {
  if (!valid(P) || !uv0 || !U) return kEInval;
  const size_t N = cells(P);
  for (int b = 0; b < P->nb; ++b) rto::init_member<double>(*P, uv0 + 2 * N * b, U + 4 * N * b);
  return 0;
}

int rto_cfl_dt(const Problem* P, const double* U, double* dt) {
  if (!valid(P) || !U || !dt) return kEInval;
  const size_t N = cells(P);
  for (int b = 0; b < P->nb; ++b) dt[b] = P->cfl / rto::max_signal_speed(*P, U + 4 * N * b);
  return 0;
}

int rto_step(const Problem* P, const double* U, double* Un, const double* dt) {
  if (!valid(P) || !U || !Un || !dt || U == Un) return kEInval;
  const size_t N = cells(P);
  int bad = 0;
  for (int b = 0; b < P->nb; ++b) bad |= rto::step_member<double>(*P, U + 4 * N * b, Un + 4 * N * b, dt[b]);
  return bad ? kEUnphys : 0;
}

int rto_integrate(const Problem* P, double* U, double T, double* t_out, int32_t* nsteps, double* dt_log,
                  int32_t cap) {
  if (!valid(P) || !U || !(T > 0)) return kEInval;
  const size_t N = cells(P);
  int rc = 0;
  for (int b = 0; b < P->nb; ++b) {
    std::vector<double> dts;
    int32_t n = 0;
    const int r = integrate_member(*P, U + 4 * N * b, T, t_out ? t_out + b : nullptr, &n, &dts, nullptr);
    if (nsteps) nsteps[b] = n;
    if (dt_log) {
      if (n > cap) return kENomem;
      for (int32_t k = 0; k < n; ++k) dt_log[static_cast<size_t>(b) * cap + k] = dts[k];
    }
    if (r) rc = r;
  }
  return rc;
}

int rto_kinetic_energy(const Problem* P, const double* U, double* ke) {
  if (!valid(P) || !U || !ke) return kEInval;
  const size_t N = cells(P);
  for (int b = 0; b < P->nb; ++b) ke[b] = rto::kinetic_energy<double>(*P, U + 4 * N * b);
  return 0;
}

int rto_step_jvp(const Problem* P, const double* U, const double* dU, const double* dt, double* Un, double* dUn) {
  if (!valid(P) || !U || !dU || !dt || !Un || !dUn) return kEInval;
  const size_t n4 = 4 * cells(P);
  std::vector<Dual> x(n4), y(n4);
  int bad = 0;
  for (int b = 0; b < P->nb; ++b) {
    const size_t o = n4 * b;
    for (size_t k = 0; k < n4; ++k) x[k] = Dual(U[o + k], dU[o + k]);
    bad |= rto::step_member<Dual>(*P, x.data(), y.data(), dt[b]);
    for (size_t k = 0; k < n4; ++k) {
      Un[o + k] = y[k].v;
      dUn[o + k] = y[k].d;
    }
  }
  return bad ? kEUnphys : 0;
}

int rto_step_vjp(const Problem* P, const double* U, const double* dt, const double* lam_next, double* lam) {
  if (!valid(P) || !U || !dt || !lam_next || !lam) return kEInval;
  const size_t n4 = 4 * cells(P);
  int bad = 0;
  for (int b = 0; b < P->nb; ++b) bad |= vjp_member(*P, U + n4 * b, dt[b], lam_next + n4 * b, lam + n4 * b);
  return bad ? kEUnphys : 0;
}

// R = KE(U^N)/KE(U^0) of each member and dR/d(u0, v0) (layout [2][ny][nx],
// Euclidean gradient with respect to the array entries).  The time steps are
// those of the forward run, held fixed while differentiating.  Every state
// of the march is stored (the oracle does not checkpoint).  dt_log, if given,
// receives each member's steps ([nb][cap]).
int rto_grad_u0(const Problem* P, const double* uv0, double T, double* R, double* grad, int32_t* nsteps,
                double* dt_log, int32_t cap) {
  if (!valid(P) || !uv0 || !R || !grad || !(T > 0)) return kEInval;
  const size_t N = cells(P), n4 = 4 * N;
  rto::Tape& tp = rto::tape();
  for (int b = 0; b < P->nb; ++b) {
    const double* uv = uv0 + 2 * N * b;
    std::vector<double> U(n4);
    rto::init_member<double>(*P, uv, U.data());
    const double ke0 = rto::kinetic_energy<double>(*P, U.data());
    if (!(ke0 > 0.0)) return kEInval;
    std::vector<double> dts;
    std::vector<std::vector<double>> states;
    int32_t n = 0;
    const int rc = integrate_member(*P, U.data(), T, nullptr, &n, &dts, &states);
    if (rc) return rc;
    if (nsteps) nsteps[b] = n;
    if (dt_log) {
      if (n > cap) return kENomem;
      for (int32_t k = 0; k < n; ++k) dt_log[static_cast<size_t>(b) * cap + k] = dts[k];
    }
    const double keN = rto::kinetic_energy<double>(*P, U.data());
    R[b] = keN / ke0;

    // Terminal adjoint: d(KE(U^N)/KE0)/dU^N with KE0 held fixed.
    std::vector<double> lam(n4), lam_prev(n4);
    {
      tp.clear();
      std::vector<Rev> x(n4);
      for (size_t k = 0; k < n4; ++k) x[k] = Rev::leaf(U[k]);
      const Rev r = rto::kinetic_energy<Rev>(*P, x.data()) / ke0;
      tp.adj.assign(tp.nodes.size(), 0.0);
      tp.adj[r.i] = 1.0;
      tp.sweep();
      for (size_t k = 0; k < n4; ++k) lam[k] = tp.adj[x[k].i];
      tp.clear();
    }
    // Reverse sweep through the stored states.
    for (int32_t s = n - 1; s >= 0; --s) {
      if (vjp_member(*P, states[s].data(), dts[s], lam.data(), lam_prev.data())) return kEUnphys;
      lam.swap(lam_prev);
    }
    // Initial adjoint: through U^0(uv0) and through KE0(uv0) in R = KE_N/KE0.
    {
      tp.clear();
      std::vector<Rev> q(2 * N), U0(n4);
      for (size_t k = 0; k < 2 * N; ++k) q[k] = Rev::leaf(uv[k]);
      rto::init_member<Rev>(*P, q.data(), U0.data());
      Rev f = keN / rto::kinetic_energy<Rev>(*P, U0.data());
      for (size_t k = 0; k < n4; ++k) f = f + lam[k] * U0[k];
      tp.adj.assign(tp.nodes.size(), 0.0);
      tp.adj[f.i] = 1.0;
      tp.sweep();
      for (size_t k = 0; k < 2 * N; ++k) grad[2 * N * b + k] = tp.adj[q[k].i];
      tp.clear();
    }
  }
  return 0;
}

// KE ratio of a march that uses a given dt sequence (the frozen schedule of
// a previous run) instead of the CFL step: the map that rto_grad_u0
// differentiates.  dt_log is [nb][cap]; nsteps[b] steps are taken.
int rto_ke_ratio_frozen(const Problem* P, const double* uv0, const double* dt_log, const int32_t* nsteps,
                        int32_t cap, double* R) {
  if (!valid(P) || !uv0 || !dt_log || !nsteps || !R) return kEInval;
  const size_t N = cells(P), n4 = 4 * N;
  std::vector<double> U(n4), Un(n4);
  for (int b = 0; b < P->nb; ++b) {
    Problem Q = *P;
    Q.nb = 1;
    rto::init_member<double>(Q, uv0 + 2 * N * b, U.data());
    const double ke0 = rto::kinetic_energy<double>(Q, U.data());
    for (int32_t s = 0; s < nsteps[b]; ++s) {
      if (rto::step_member<double>(Q, U.data(), Un.data(), dt_log[static_cast<size_t>(b) * cap + s]))
        return kEUnphys;
      U.swap(Un);
    }
    R[b] = rto::kinetic_energy<double>(Q, U.data()) / ke0;
  }
  return 0;
}

// Mixing-layer width (Eqs. 13-14): the integral over y of 4 f (1 - f),
// f the horizontally averaged density normalised between rho_l and rho_h
// and clipped to [0, 1]; midpoint rule over the rows.
int rto_mix_width(const Problem* P, const double* U, double* h) {
  if (!valid(P) || !U || !h) return kEInval;
  const size_t N = cells(P);
  const double dy = P->ly / P->ny;
  for (int b = 0; b < P->nb; ++b) {
    const double* r = U + 4 * N * b;
    double s = 0.0;
    for (int j = 0; j < P->ny; ++j) {
      double mean = 0.0;
      for (int i = 0; i < P->nx; ++i) mean += r[static_cast<size_t>(j) * P->nx + i];
      mean /= P->nx;
      double f = (mean - P->rho_l) / (P->rho_h - P->rho_l);
      if (f < 0.0) f = 0.0;
      if (f > 1.0) f = 1.0;
      s += 4.0 * f * (1.0 - f) * dy;
    }
    h[b] = s;
  }
  return 0;
}

// Horizontal power spectrum behind Eq. 12: for each member's field f
// ([ny][nx], rows of nx values, member b at f + b * member_stride),
// E[b][n] = sum over the selected rows of |sum_i f(i, j) exp(-2 pi i n i / nx)|^2,
// n = 0 .. nx/2, by the plain discrete Fourier sum (the phase n i is reduced
// modulo nx before the cosine and sine are taken).  row = -1: all rows.
int rto_row_spectrum(const Problem* P, const double* f, int64_t member_stride, int32_t row, double* E) {
  if (!valid(P) || !f || !E || row < -1 || row >= P->ny) return kEInval;
  const int nx = P->nx, nbins = nx / 2 + 1;
  const double two_pi = 2.0 * 3.14159265358979323846;
  for (int b = 0; b < P->nb; ++b) {
    const double* fb = f + static_cast<size_t>(b) * static_cast<size_t>(member_stride);
    for (int n = 0; n < nbins; ++n) {
      double e = 0.0;
      for (int j = (row < 0 ? 0 : row); j < (row < 0 ? P->ny : row + 1); ++j) {
        double re = 0.0, im = 0.0;
        for (int i = 0; i < nx; ++i) {
          const double phase = two_pi * static_cast<double>((static_cast<long>(n) * i) % nx) / nx;
          re += fb[static_cast<size_t>(j) * nx + i] * std::cos(phase);
          im -= fb[static_cast<size_t>(j) * nx + i] * std::sin(phase);
        }
        e += re * re + im * im;
      }
      E[static_cast<size_t>(b) * nbins + n] = e;
    }
  }
  return 0;
}

// 2-D power spectrum (App. B's reconstruction keeps its strongest modes):
// E[b][q][k] = |sum_{y, x} f(y, x) exp(-2 pi i (k x / nx + q y / ny))|^2 for
// q = 0 .. ny - 1, k = 0 .. nx/2, written as the transform of every row and
// then of every column of the result (the 2-D DFT factorises), each a plain
// Fourier sum with its phase reduced modulo the length.
int rto_power_spectrum_2d(const Problem* P, const double* f, int64_t member_stride, double* E) {
  if (!valid(P) || !f || !E) return kEInval;
  const int nx = P->nx, ny = P->ny, nk = nx / 2 + 1;
  const double two_pi = 2.0 * 3.14159265358979323846;
  std::vector<double> cre(static_cast<size_t>(ny) * nk), cim(static_cast<size_t>(ny) * nk);
  for (int b = 0; b < P->nb; ++b) {
    const double* fb = f + static_cast<size_t>(b) * static_cast<size_t>(member_stride);
    for (int y = 0; y < ny; ++y)
      for (int k = 0; k < nk; ++k) {
        double re = 0.0, im = 0.0;
        for (int x = 0; x < nx; ++x) {
          const double ph = two_pi * static_cast<double>((static_cast<long>(k) * x) % nx) / nx;
          re += fb[static_cast<size_t>(y) * nx + x] * std::cos(ph);
          im -= fb[static_cast<size_t>(y) * nx + x] * std::sin(ph);
        }
        cre[static_cast<size_t>(y) * nk + k] = re;
        cim[static_cast<size_t>(y) * nk + k] = im;
      }
    for (int q = 0; q < ny; ++q)
      for (int k = 0; k < nk; ++k) {
        double re = 0.0, im = 0.0;
        for (int y = 0; y < ny; ++y) {
          const double ph = two_pi * static_cast<double>((static_cast<long>(q) * y) % ny) / ny;
          const double c = std::cos(ph), s = std::sin(ph);
          const double ar = cre[static_cast<size_t>(y) * nk + k], ai = cim[static_cast<size_t>(y) * nk + k];
          re += ar * c + ai * s;
          im += ai * c - ar * s;
        }
        E[(static_cast<size_t>(b) * ny + q) * nk + k] = re * re + im * im;
      }
  }
  return 0;
}

// Kinetic-energy density e_k = |m|^2/(2 rho) of each cell (Eq. 7),
// layout [nb][ny][nx].
int rto_ek_field(const Problem* P, const double* U, double* ek) {
  if (!valid(P) || !U || !ek) return kEInval;
  const size_t N = cells(P);
  for (int b = 0; b < P->nb; ++b) rto::ek_field<double>(*P, U + 4 * N * b, ek + N * b);
  return 0;
}

// J = sum over cells of (e_k(U^N) - ek_base)^2 dx dy (Eq. 8) after the march
// with the given steps dt_log[nb][cap] (nsteps[b] of them); ek_base is
// [nb][ny][nx].
int rto_ek_anomaly_frozen(const Problem* P, const double* uv0, const double* dt_log, const int32_t* nsteps,
                          int32_t cap, const double* ek_base, double* J) {
  if (!valid(P) || !uv0 || !dt_log || !nsteps || !ek_base || !J) return kEInval;
  const size_t N = cells(P), n4 = 4 * N;
  std::vector<double> U(n4), Un(n4);
  for (int b = 0; b < P->nb; ++b) {
    Problem Q = *P;
    Q.nb = 1;
    rto::init_member<double>(Q, uv0 + 2 * N * b, U.data());
    for (int32_t s = 0; s < nsteps[b]; ++s) {
      if (rto::step_member<double>(Q, U.data(), Un.data(), dt_log[static_cast<size_t>(b) * cap + s]))
        return kEUnphys;
      U.swap(Un);
    }
    J[b] = rto::ek_anomaly<double>(Q, U.data(), ek_base + N * b);
  }
  return 0;
}

// J of Eq. 8 for each member and dJ/d(u0, v0) ([2][ny][nx]), by reverse-mode
// AD through the march with the forward run's steps held fixed (as in
// rto_grad_u0): terminal adjoint dJ/dU^N, the stored-state reverse sweep,
// then the adjoint of U^0(uv0).
int rto_grad_ek_anomaly(const Problem* P, const double* uv0, double T, const double* ek_base, double* J,
                        double* grad, int32_t* nsteps, double* dt_log, int32_t cap) {
  if (!valid(P) || !uv0 || !ek_base || !J || !grad || !(T > 0)) return kEInval;
  const size_t N = cells(P), n4 = 4 * N;
  rto::Tape& tp = rto::tape();
  for (int b = 0; b < P->nb; ++b) {
    Problem Q = *P;
    Q.nb = 1;
    const double* uv = uv0 + 2 * N * b;
    const double* ekb = ek_base + N * b;
    std::vector<double> U(n4);
    rto::init_member<double>(Q, uv, U.data());
    std::vector<double> dts;
    std::vector<std::vector<double>> states;
    int32_t n = 0;
    const int rc = integrate_member(Q, U.data(), T, nullptr, &n, &dts, &states);
    if (rc) return rc;
    if (nsteps) nsteps[b] = n;
    if (dt_log) {
      if (n > cap) return kENomem;
      for (int32_t k = 0; k < n; ++k) dt_log[static_cast<size_t>(b) * cap + k] = dts[k];
    }
    J[b] = rto::ek_anomaly<double>(Q, U.data(), ekb);

    std::vector<double> lam(n4), lam_prev(n4);
    {
      tp.clear();
      std::vector<Rev> x(n4);
      for (size_t k = 0; k < n4; ++k) x[k] = Rev::leaf(U[k]);
      const Rev r = rto::ek_anomaly<Rev>(Q, x.data(), ekb);
      tp.adj.assign(tp.nodes.size(), 0.0);
      tp.adj[r.i] = 1.0;
      tp.sweep();
      for (size_t k = 0; k < n4; ++k) lam[k] = tp.adj[x[k].i];
      tp.clear();
    }
    for (int32_t s = n - 1; s >= 0; --s) {
      if (vjp_member(Q, states[s].data(), dts[s], lam.data(), lam_prev.data())) return kEUnphys;
      lam.swap(lam_prev);
    }
    {
      tp.clear();
      std::vector<Rev> q(2 * N), U0(n4);
      for (size_t k = 0; k < 2 * N; ++k) q[k] = Rev::leaf(uv[k]);
      rto::init_member<Rev>(Q, q.data(), U0.data());
      Rev f(0.0);
      for (size_t k = 0; k < n4; ++k) f = f + lam[k] * U0[k];
      tp.adj.assign(tp.nodes.size(), 0.0);
      tp.adj[f.i] = 1.0;
      tp.sweep();
      for (size_t k = 0; k < 2 * N; ++k) grad[2 * N * b + k] = tp.adj[q[k].i];
      tp.clear();
    }
  }
  return 0;
}

// R = KE(T)/KE(0) (ek_base null) or J of Eq. 8 (ek_base [nb][ny][nx]) after
// the adaptive march to T, and nsteps[b] (may be null).
int rto_objective_adaptive(const Problem* P, const double* uv0, double T, const double* ek_base, double* val,
                           int32_t* nsteps) {
  if (!valid(P) || !uv0 || !val || !(T > 0)) return kEInval;
  const size_t N = cells(P), n4 = 4 * N;
  for (int b = 0; b < P->nb; ++b) {
    Problem Q = *P;
    Q.nb = 1;
    std::vector<double> U(n4);
    rto::init_member<double>(Q, uv0 + 2 * N * b, U.data());
    const double ke0 = rto::kinetic_energy<double>(Q, U.data());
    if (!ek_base && !(ke0 > 0.0)) return kEInval;
    int32_t n = 0;
    if (int rc = integrate_member(Q, U.data(), T, nullptr, &n, nullptr, nullptr)) return rc;
    if (nsteps) nsteps[b] = n;
    val[b] = objective_value(Q, U.data(), ek_base ? ek_base + N * b : nullptr, ke0);
  }
  return 0;
}

// R or J (as rto_objective_adaptive) and its gradient with respect to
// (u0, v0) ([nb][2][ny][nx]) through the adaptive march itself: the march
// carries (U, t), and each step is
//     dt = cfl / S(U),  clipped to T - t on the last step,
//     U <- step(U, dt),  t <- t + dt  (t = T after the last step),
// with S the largest signal speed.  Reverse mode runs on that whole map,
// one step's tape at a time, with adjoints of both U and t; which step is
// the last, and which cell holds the largest speed, are taken from the
// primal values (the number of steps is locally constant).
int rto_grad_adaptive(const Problem* P, const double* uv0, double T, const double* ek_base, double* val,
                      double* grad, int32_t* nsteps) {
  if (!valid(P) || !uv0 || !val || !grad || !(T > 0)) return kEInval;
  const size_t N = cells(P), n4 = 4 * N;
  rto::Tape& tp = rto::tape();
  for (int b = 0; b < P->nb; ++b) {
    Problem Q = *P;
    Q.nb = 1;
    const double* uv = uv0 + 2 * N * b;
    const double* ekb = ek_base ? ek_base + N * b : nullptr;
    std::vector<double> U(n4);
    rto::init_member<double>(Q, uv, U.data());
    const double ke0 = rto::kinetic_energy<double>(Q, U.data());
    if (!ekb && !(ke0 > 0.0)) return kEInval;
    std::vector<double> dts;
    std::vector<std::vector<double>> states;
    int32_t n = 0;
    if (int rc = integrate_member(Q, U.data(), T, nullptr, &n, &dts, &states)) return rc;
    if (nsteps) nsteps[b] = n;
    const double keN = rto::kinetic_energy<double>(Q, U.data());
    val[b] = objective_value(Q, U.data(), ekb, ke0);
    // times t^k at the start of each step, summed as the march sums them
    std::vector<double> times(n);
    double t = 0.0;
    for (int32_t k = 0; k < n; ++k) {
      times[k] = t;
      t = t + dts[k];
    }

    // terminal adjoint of U^N (KE(0) held fixed for R); the adjoint of t^N
    // is zero: the objective does not read the time
    std::vector<double> lam(n4);
    double lam_t = 0.0;
    {
      tp.clear();
      std::vector<Rev> x(n4);
      for (size_t k = 0; k < n4; ++k) x[k] = Rev::leaf(U[k]);
      const Rev r = ekb ? rto::ek_anomaly<Rev>(Q, x.data(), ekb) : rto::kinetic_energy<Rev>(Q, x.data()) / ke0;
      tp.adj.assign(tp.nodes.size(), 0.0);
      tp.adj[r.i] = 1.0;
      tp.sweep();
      for (size_t k = 0; k < n4; ++k) lam[k] = tp.adj[x[k].i];
      tp.clear();
    }
    for (int32_t s = n - 1; s >= 0; --s) {
      tp.clear();
      std::vector<Rev> x(n4), y(n4);
      for (size_t k = 0; k < n4; ++k) x[k] = Rev::leaf(states[s][k]);
      const Rev ts = Rev::leaf(times[s]);
      Rev dt = Q.cfl / rto::max_signal_speed<Rev>(Q, x.data());
      const Rev rem = Rev(T) - ts;
      const bool last = rto::val(dt) >= rto::val(rem);
      if (last != (s == n - 1)) return kEInval;  // must retrace the primal march
      if (last) dt = rem;
      if (rto::val(dt) != dts[s]) return kEInval;
      if (rto::step_member<Rev, Rev>(Q, x.data(), y.data(), dt)) return kEUnphys;
      const Rev tn = last ? Rev(T) : ts + dt;
      tp.adj.assign(tp.nodes.size(), 0.0);
      for (size_t k = 0; k < n4; ++k)
        if (y[k].i >= 0) tp.adj[y[k].i] += lam[k];
      if (tn.i >= 0) tp.adj[tn.i] += lam_t;
      tp.sweep();
      for (size_t k = 0; k < n4; ++k) lam[k] = tp.adj[x[k].i];
      lam_t = tp.adj[ts.i];
      tp.clear();
    }
    // initial adjoint: through U^0(uv0), and for R through KE(0) too
    {
      tp.clear();
      std::vector<Rev> q(2 * N), U0(n4);
      for (size_t k = 0; k < 2 * N; ++k) q[k] = Rev::leaf(uv[k]);
      rto::init_member<Rev>(Q, q.data(), U0.data());
      Rev f = ekb ? Rev(0.0) : keN / rto::kinetic_energy<Rev>(Q, U0.data());
      for (size_t k = 0; k < n4; ++k) f = f + lam[k] * U0[k];
      tp.adj.assign(tp.nodes.size(), 0.0);
      tp.adj[f.i] = 1.0;
      tp.sweep();
      for (size_t k = 0; k < 2 * N; ++k) grad[2 * N * b + k] = tp.adj[q[k].i];
      tp.clear();
    }
  }
  return 0;
}

// Scale each member's perturbation onto the constraint set (Eq. 11).
//   norm 0: (sum (u^2+v^2) dx dy)^(1/2)       (velocity L2 norm)
//   norm 1: (mean over cells of u^2+v^2)^(1/2) (RMS)
//   norm 2: C = sum rho0 (u^2+v^2)/2 dx dy     (Eq. 9); delta plays epsilon
//   set 0: sphere (always scaled to the bound); set 1: ball (scaled only
//   when outside, Eq. 11).  Components switched off by comp_mask are zeroed.
// norm_out[b] receives the norm (or C) before scaling.
int rto_project_to_constraint(const Problem* P, double* uv, double delta, int32_t norm, int32_t set,
                              double* norm_out) {
  if (!valid(P) || !uv || !(delta > 0) || norm < 0 || norm > 2 || set < 0 || set > 1) return kEInval;
  const int nx = P->nx, ny = P->ny;
  const size_t N = cells(P);
  const double dV = rto::dx_of(*P) * rto::dy_of(*P);
  for (int b = 0; b < P->nb; ++b) {
    double* u = uv + 2 * N * b;
    double* v = u + N;
    if (!(P->comp_mask & 1))
      for (size_t c = 0; c < N; ++c) u[c] = 0.0;
    if (!(P->comp_mask & 2))
      for (size_t c = 0; c < N; ++c) v[c] = 0.0;
    double s = 0.0;
    for (int j = 0; j < ny; ++j) {
      const double w = norm == 2 ? 0.5 * rto::rho0_at(*P, rto::yc(*P, j)) : 1.0;
      for (int i = 0; i < nx; ++i) {
        const size_t c = static_cast<size_t>(j) * nx + i;
        s += w * (u[c] * u[c] + v[c] * v[c]);
      }
    }
    double m, scale;
    if (norm == 0) {
      m = std::sqrt(s * dV);
      scale = delta / m;
    } else if (norm == 1) {
      m = std::sqrt(s / static_cast<double>(N));
      scale = delta / m;
    } else {
      m = s * dV;
      scale = std::sqrt(delta / m);
    }
    if (norm_out) norm_out[b] = m;
    if (set == 1 && m <= delta) continue;
    if (!(m > 0.0)) return kEInval;
    for (size_t c = 0; c < 2 * N; ++c) u[c] *= scale;
  }
  return 0;
}

// Single-face HLLC flux in face-normal order (mass, normal momentum,
// tangential momentum, energy); states are (rho, normal vel., tangential
// vel., p).  The workloads' tie tolerance (1e-10) applies.
int rto_hllc(double gamma, const double* L, const double* Rr, double* flux) {
  Problem P{};
  P.gamma = gamma;
  P.tie_tol = 1e-10;
  const std::array<double, 4> f =
      rto::hllc<double>(P, rto::FaceState<double>{L[0], L[1], L[2], L[3]},
                        rto::FaceState<double>{Rr[0], Rr[1], Rr[2], Rr[3]});
  for (int k = 0; k < 4; ++k) flux[k] = f[k];
  return 0;
}

double rto_wall_pressure(double gamma, const double* w, int32_t interior_left) {
  Problem P{};
  P.gamma = gamma;
  P.tie_tol = 1e-10;
  return rto::wall_pressure<double>(P, rto::FaceState<double>{w[0], w[1], w[2], w[3]}, interior_left != 0);
}

// One monotonized-central limited slope from the differences a, b, with
// differences of magnitude <= tol counting as zero: out[0] the slope,
// out[1] = d slope / d a and out[2] = d slope / d b on the selected case
// (forward-mode AD of mc_slope).
int rto_mc_slope(double a, double b, double tol, double* out) {
  if (!out || !(tol >= 0.0)) return kEInval;
  auto small = [tol](double d) { return std::fabs(d) <= tol; };
  const Dual sa = rto::mc_slope(Dual(a, 1.0), Dual(b, 0.0), small);
  const Dual sb = rto::mc_slope(Dual(a, 0.0), Dual(b, 1.0), small);
  out[0] = sa.v;
  out[1] = sa.d;
  out[2] = sb.d;
  return 0;
}

// The limited slopes (rho, u, v, p) of the cell w between its neighbours wm
// (below / left) and wp (above / right), with the problem's tie tolerance
// scaled by the cell's density, pressure and sound speed; balanced != 0 takes
// the y slopes of the well-balanced variant.  Arrays of 4 primitives.
int rto_slopes(const Problem* P, const double* wm, const double* w, const double* wp, int32_t balanced,
               double* s) {
  if (!valid(P) || !wm || !w || !wp || !s) return kEInval;
  const rto::Prim<double> a{wm[0], wm[1], wm[2], wm[3]}, c{w[0], w[1], w[2], w[3]}, b{wp[0], wp[1], wp[2], wp[3]};
  const rto::Prim<double> r = balanced ? rto::mc_slope_y_balanced(*P, a, c, b) : rto::mc_slope(*P, a, c, b);
  s[0] = r.r;
  s[1] = r.u;
  s[2] = r.v;
  s[3] = r.p;
  return 0;
}

// The MUSCL-Hancock half step of one cell: primitives w, slopes sx and sy
// (per cell width), step dt; q receives W^{n+1/2}.
int rto_predict(const Problem* P, const double* w, const double* sx, const double* sy, double dt, double* q) {
  if (!valid(P) || !w || !sx || !sy || !q) return kEInval;
  const rto::Prim<double> r = rto::predict_half_step(
      *P, rto::Prim<double>{w[0], w[1], w[2], w[3]}, rto::Prim<double>{sx[0], sx[1], sx[2], sx[3]},
      rto::Prim<double>{sy[0], sy[1], sy[2], sy[3]}, dt);
  q[0] = r.r;
  q[1] = r.u;
  q[2] = r.v;
  q[3] = r.p;
  return 0;
}

// Algorithmic floating-point work of one step of one member U ([4][ny][nx])
// at step dt (measurement only): out[0] the flops of the step (rto_count.hpp:
// every operation on state-dependent values as the scheme writes it), out[1]
// those of the largest signal speed of the new state (the CFL reduction),
// out[2] the edges of the step's computational graph (a reverse-mode
// adjoint does one multiply-add per edge after recomputing the step),
// out[3..6] the step's additions, multiplications, divisions and square
// roots.  Totals over the member's cells.
int rto_count_flops(const Problem* P, const double* U, double dt, double* out) {
  if (!valid(P) || !U || !out) return kEInval;
  const size_t n4 = 4 * cells(P);
  rto::FlopCount& fc = rto::flop_count();
  std::vector<rto::Cnt> x(n4), y(n4);
  for (size_t k = 0; k < n4; ++k) x[k] = rto::Cnt(U[k]);
  fc = rto::FlopCount{};
  const int bad = rto::step_member<rto::Cnt>(*P, x.data(), y.data(), dt);
  const rto::FlopCount step = fc;
  fc = rto::FlopCount{};
  (void)rto::max_signal_speed<rto::Cnt>(*P, y.data());
  const uint64_t cfl = fc.total();
  // edges of the step's graph, from the reverse-mode tape
  rto::Tape& tp = rto::tape();
  tp.clear();
  std::vector<Rev> xr(n4), yr(n4);
  for (size_t k = 0; k < n4; ++k) xr[k] = Rev::leaf(U[k]);
  (void)rto::step_member<Rev>(*P, xr.data(), yr.data(), dt);
  uint64_t edges = 0;
  for (const rto::Tape::Node& nd : tp.nodes) edges += (nd.a >= 0) + (nd.b >= 0);
  tp.clear();
  out[0] = (double)step.total();
  out[1] = (double)cfl;
  out[2] = (double)edges;
  out[3] = (double)step.add;
  out[4] = (double)step.mul;
  out[5] = (double)step.div;
  out[6] = (double)step.sqrt;
  return bad ? kEUnphys : 0;
}

// Threads over the rows of the double-precision forward step (timing only;
// results are the same for any count).  Returns the count in force: 1 if
// the library was built without OpenMP.
int rto_set_threads(int32_t n) {
  if (n < 1) return kEInval;
#ifdef _OPENMP
  rto::omp_threads() = n;
  return n;
#else
  return 1;
#endif
}

// Background profiles at the cell centres of row j (Eq. 5 and the
// hydrostatic integral), for tests.
int rto_background(const Problem* P, double* rho0, double* p0) {
  if (!valid(P) || !rho0 || !p0) return kEInval;
  for (int j = 0; j < P->ny; ++j) {
    rho0[j] = rto::rho0_at(*P, rto::yc(*P, j));
    p0[j] = rto::background_p(*P, j);
  }
  return 0;
}

}  // extern "C"
