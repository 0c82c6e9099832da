// Device arithmetic of the MI355X hot path: the pieces of one finite-volume
// step (primitive variables, limited slopes, MUSCL-Hancock predictor, HLLC
// flux, wall flux, update with gravity) and the hand-derived adjoint of each.
//
// Scheme (the paper fixes the PDE, Sec. 2.1 Eqs. 1-4, and the scheme family,
// a Godunov-type finite-volume method with an HLLC solver and a gravity
// source, Sec. 2.3; the rest is this implementation's reading):
//   * primitive variables W = (rho, u, v, p), p = (gamma-1)(E - |m|^2/(2 rho));
//   * monotonized-central (MC) limited slopes: zero if a*b <= 0 or a
//     difference is negligible (below 1e-10 of the local scale), else the
//     central difference (a+b)/2 if it does not exceed 2|a| and 2|b|, else
//     2a if |a| <= |b|, else 2b;
//   * unsplit MUSCL-Hancock half step in primitive variables with gravity
//     added to v, face states W^{n+1/2} -/+ dW/2;
//   * HLLC (Toro-Spruce-Speares) with Davis speeds; near-ties of the Davis
//     minimum/maximum and of the contact sign S* = 0 (within the same
//     relative tolerance) take the left state;
//   * wall faces carry (0, 0, p*, 0) with p* the star pressure of the
//     mirrored Riemann problem;
//   * U^{n+1} = U^n - dt/dx dF - dt/dy dG, then m_y += dt g_y (rho^n +
//     rho^{n+1})/2 and E += dt g_y (G_rho,bottom + G_rho,top)/2, which makes
//     E + rho*phi (phi = -g_y y) conserved.
// All branches are evaluated as selects, so a wavefront never diverges.
#pragma once
#include <hip/hip_runtime.h>

namespace rtk {

struct Params {
  int nx, ny, nb, comp_mask;
  double dx, dy, inv_dx, inv_dy;
  double gamma, gm1, inv_gm1, g_y, cfl;
  double rho_h, rho_l, y0, h, p_int;
};

struct W4 {
  double r, u, v, p;
};

#define RT_DEV __device__ __forceinline__

RT_DEV W4 cons_to_prim(const Params& P, double r, double mx, double my, double E) {
  const double ri = 1.0 / r;
  const double u = mx * ri, v = my * ri;
  W4 w;
  w.r = r;
  w.u = u;
  w.v = v;
  w.p = P.gm1 * (E - 0.5 * (mx * u + my * v));
  return w;
}

RT_DEV bool unphysical(const W4& w) {
  // also catches NaN: comparisons with NaN are false
  return !(w.r > 0.0) || !(w.p > 0.0) || !(fabs(w.u) < 1e300) || !(fabs(w.v) < 1e300);
}

// Adjoint of cons_to_prim: W-bar -> U-bar at the state (r, u, v).
RT_DEV void prim_adj(const Params& P, const W4& w, const W4& wb, double ub[4]) {
  const double ri = 1.0 / w.r;
  ub[0] = wb.r - (w.u * wb.u + w.v * wb.v) * ri + 0.5 * P.gm1 * (w.u * w.u + w.v * w.v) * wb.p;
  ub[1] = wb.u * ri - P.gm1 * w.u * wb.p;
  ub[2] = wb.v * ri - P.gm1 * w.v * wb.p;
  ub[3] = P.gm1 * wb.p;
}

// Relative tolerance below which a difference counts as zero when the scheme
// takes a discrete decision (limiter case, upwind side, wave-speed choice).
// Decisions on round-off-level differences would otherwise be random, and
// the linearised compressive limiter branches amplify grid-scale
// perturbations, which would make the discrete gradient erratic.  The
// forward state changes by at most this tolerance, relative.
constexpr double kTieTol = 1e-10;

// MC-limited slope and its case: 0 zero, 1 central, 2 -> 2a, 3 -> 2b.  The
// zero case also covers a negligible difference (small_a / small_b).
RT_DEV double mc(double a, double b, bool small_a, bool small_b, int& code) {
  const double c = 0.5 * (a + b);
  const double aa = fabs(a), ab = fabs(b), ac = fabs(c);
  const bool zero = (a * b <= 0.0) || small_a || small_b;
  const bool central = (ac <= 2.0 * aa) && (ac <= 2.0 * ab);
  const bool left = aa <= ab;
  const double s = zero ? 0.0 : (central ? c : (left ? 2.0 * a : 2.0 * b));
  code = zero ? 0 : (central ? 1 : (left ? 2 : 3));
  return s;
}

// Weights (d s/d a, d s/d b) of an MC case.
RT_DEV void mc_weights(int code, double& wa, double& wb) {
  wa = code == 1 ? 0.5 : (code == 2 ? 2.0 : 0.0);
  wb = code == 1 ? 0.5 : (code == 3 ? 2.0 : 0.0);
}

// Slopes of the four primitives; codes packed 2 bits per variable.  A
// difference is negligible below kTieTol times the centre cell's density,
// pressure, or sound speed (velocities: d^2 rho <= kTieTol^2 gamma p).
RT_DEV W4 mc4(const Params& P, const W4& m, const W4& c, const W4& p, int& codes) {
  const double tr = kTieTol * c.r, tp = kTieTol * c.p, tv2 = kTieTol * kTieTol * P.gamma * c.p;
  int k0, k1, k2, k3;
  W4 s;
  const double ar = c.r - m.r, br = p.r - c.r;
  const double au = c.u - m.u, bu = p.u - c.u;
  const double av = c.v - m.v, bv = p.v - c.v;
  const double ap = c.p - m.p, bp = p.p - c.p;
  s.r = mc(ar, br, fabs(ar) <= tr, fabs(br) <= tr, k0);
  s.u = mc(au, bu, au * au * c.r <= tv2, bu * bu * c.r <= tv2, k1);
  s.v = mc(av, bv, av * av * c.r <= tv2, bv * bv * c.r <= tv2, k2);
  s.p = mc(ap, bp, fabs(ap) <= tp, fabs(bp) <= tp, k3);
  codes = k0 | (k1 << 2) | (k2 << 4) | (k3 << 6);
  return s;
}

// Ghost cells of the y walls: mirror of the adjacent interior cell with the
// normal velocity negated and the pressure extrapolated hydrostatically
// (dp/dy = rho g_y) over the distance between the two cell centres.
RT_DEV W4 ghost_bottom(const Params& P, const W4& w) {
  return W4{w.r, w.u, -w.v, w.p - P.g_y * w.r * P.dy};
}
RT_DEV W4 ghost_top(const Params& P, const W4& w) {
  return W4{w.r, w.u, -w.v, w.p + P.g_y * w.r * P.dy};
}

// MUSCL-Hancock half step: q = W - hx A_x(W) sx - hy A_y(W) sy + (dt/2) g.
RT_DEV W4 predict(const Params& P, const W4& w, const W4& sx, const W4& sy, double hx, double hy,
                  double half_dt_g) {
  const double ri = 1.0 / w.r;
  W4 q;
  q.r = w.r - hx * (w.u * sx.r + w.r * sx.u) - hy * (w.v * sy.r + w.r * sy.v);
  q.u = w.u - hx * (w.u * sx.u + sx.p * ri) - hy * (w.v * sy.u);
  q.v = w.v - hx * (w.u * sx.v) - hy * (w.v * sy.v + sy.p * ri) + half_dt_g;
  q.p = w.p - hx * (P.gamma * w.p * sx.u + w.u * sx.p) - hy * (P.gamma * w.p * sy.v + w.v * sy.p);
  return q;
}

// Adjoint of predict: q-bar -> (W-bar, sx-bar, sy-bar), accumulated.
RT_DEV void predict_adj(const Params& P, const W4& w, const W4& sx, const W4& sy, double hx, double hy,
                        const W4& qb, W4& wb, W4& sxb, W4& syb) {
  const double ri = 1.0 / w.r;
  const double g = P.gamma;
  wb.r += qb.r - hx * qb.r * sx.u - hy * qb.r * sy.v + (hx * qb.u * sx.p + hy * qb.v * sy.p) * ri * ri;
  wb.u += qb.u - hx * (qb.r * sx.r + qb.u * sx.u + qb.v * sx.v + qb.p * sx.p);
  wb.v += qb.v - hy * (qb.r * sy.r + qb.u * sy.u + qb.v * sy.v + qb.p * sy.p);
  wb.p += qb.p - g * qb.p * (hx * sx.u + hy * sy.v);
  sxb.r += -hx * w.u * qb.r;
  sxb.u += -hx * (w.r * qb.r + w.u * qb.u + g * w.p * qb.p);
  sxb.v += -hx * w.u * qb.v;
  sxb.p += -hx * (qb.u * ri + w.u * qb.p);
  syb.r += -hy * w.v * qb.r;
  syb.u += -hy * w.v * qb.u;
  syb.v += -hy * (w.r * qb.r + w.v * qb.v + g * w.p * qb.p);
  syb.p += -hy * (qb.v * ri + w.v * qb.p);
}

// --------------------------------------------------------------------- HLLC
// States in face-normal order: r, n (normal velocity), t (tangential), p.
// Flux in face-normal order: mass, normal momentum, tangential momentum,
// energy.  F = F_K + sigma (U*_K - U_K) with K = left if S* >= 0 else right,
// sigma = min(S_L, 0) on the left, max(S_R, 0) on the right: the four cases
// S_L >= 0 / S* >= 0 / S_R > 0 / else in one formula.
struct FS {
  double r, n, t, p;
};

RT_DEV void hllc(const Params& P, const FS& L, const FS& R, double F[4]) {
  const double g = P.gamma;
  const double cL = sqrt(g * L.p / L.r), cR = sqrt(g * R.p / R.r);
  const double tie = kTieTol * (cL + cR);  // near-ties resolve to the left state
  const double aL = L.n - cL, bL = R.n - cR, aR = L.n + cL, bR = R.n + cR;
  const double SL = aL <= bL + tie ? aL : bL;
  const double SR = aR >= bR - tie ? aR : bR;
  const double mL = L.r * (SL - L.n), mR = R.r * (SR - R.n);
  const double SS = (R.p - L.p + mL * L.n - mR * R.n) / (mL - mR);
  const bool left = SS >= -tie;
  const double r = left ? L.r : R.r, n = left ? L.n : R.n, t = left ? L.t : R.t, p = left ? L.p : R.p;
  const double S = left ? SL : SR, m = left ? mL : mR;
  const double sig = left ? (SL < 0.0 ? SL : 0.0) : (SR > 0.0 ? SR : 0.0);
  const double E = p * P.inv_gm1 + 0.5 * r * (n * n + t * t);
  const double m0 = r * n;
  const double den = sig != 0.0 ? (S - SS) : 1.0;
  const double f = sig != 0.0 ? m / den : 0.0;
  const double H = E / r + (SS - n) * (SS + p / m);
  F[0] = m0 + sig * (f - r);
  F[1] = m0 * n + p + sig * (f * SS - m0);
  F[2] = m0 * t + sig * (f * t - r * t);
  F[3] = n * (E + p) + sig * (f * H - E);
}

// Adjoint of hllc: given F-bar, accumulate L-bar and R-bar.
RT_DEV void hllc_adj(const Params& P, const FS& L, const FS& R, const double Fb[4], FS& Lb, FS& Rb) {
  const double g = P.gamma;
  // ---- forward recompute
  const double cL = sqrt(g * L.p / L.r), cR = sqrt(g * R.p / R.r);
  const double tie = kTieTol * (cL + cR);
  const double aL = L.n - cL, bL = R.n - cR, aR = L.n + cL, bR = R.n + cR;
  const bool selL = aL <= bL + tie, selR = aR >= bR - tie;
  const double SL = selL ? aL : bL;
  const double SR = selR ? aR : bR;
  const double dL = SL - L.n, dR = SR - R.n;
  const double mL = L.r * dL, mR = R.r * dR;
  const double num = R.p - L.p + mL * L.n - mR * R.n;
  const double dn = mL - mR;
  const double SS = num / dn;
  const bool left = SS >= -tie;
  const double r = left ? L.r : R.r, n = left ? L.n : R.n, t = left ? L.t : R.t, p = left ? L.p : R.p;
  const double S = left ? SL : SR, m = left ? mL : mR;
  const bool act = left ? (SL < 0.0) : (SR > 0.0);
  const double sig = act ? S : 0.0;
  const double E = p * P.inv_gm1 + 0.5 * r * (n * n + t * t);
  const double m0 = r * n;
  const double den = act ? (S - SS) : 1.0;
  const double f = act ? m / den : 0.0;
  const double A = SS - n, Bq = SS + p / m;
  const double H = E / r + A * Bq;
  // ---- reverse
  // F = FK + sig (Us - Uk), FK = (m0, m0 n + p, m0 t, n (E + p)),
  // Us = (f, f SS, f t, f H), Uk = (r, m0, r t, E).
  const double sigb = act ? (Fb[0] * (f - r) + Fb[1] * (f * SS - m0) + Fb[2] * (f * t - r * t) + Fb[3] * (f * H - E))
                          : 0.0;
  const double us0 = sig * Fb[0], us1 = sig * Fb[1], us2 = sig * Fb[2], us3 = sig * Fb[3];
  double rb = 0.0, nb = 0.0, tb = 0.0, pb = 0.0, Eb = 0.0, SSb = 0.0, mb = 0.0, Sb = 0.0;
  // Us
  const double fb = us0 + us1 * SS + us2 * t + us3 * H;
  SSb += us1 * f;
  tb += us2 * f;
  const double Hb = us3 * f;
  // H = E/r + A*Bq
  Eb += Hb / r;
  rb -= Hb * E / (r * r);
  const double Ab = Hb * Bq, Bqb = Hb * A;
  SSb += Ab + Bqb;
  nb -= Ab;
  pb += Bqb / m;
  mb -= Bqb * p / (m * m);
  // f = m / (S - SS)
  if (act) {
    mb += fb / den;
    Sb -= fb * f / den;
    SSb += fb * f / den;
  }
  // -Uk part (sig * (-Uk)): Uk = (r, m0, r t, E)
  const double ukb0 = -us0, ukb1 = -us1, ukb2 = -us2, ukb3 = -us3;
  rb += ukb0 + ukb2 * t;
  tb += ukb2 * r;
  double m0b = ukb1;
  Eb += ukb3;
  // FK
  m0b += Fb[0] + Fb[1] * n + Fb[2] * t;
  nb += Fb[1] * m0 + Fb[3] * (E + p);
  pb += Fb[1] + Fb[3] * n;
  tb += Fb[2] * m0;
  Eb += Fb[3] * n;
  // m0 = r n
  rb += m0b * n;
  nb += m0b * r;
  // E = p/(g-1) + r (n^2 + t^2)/2
  pb += Eb * P.inv_gm1;
  rb += Eb * 0.5 * (n * n + t * t);
  nb += Eb * r * n;
  tb += Eb * r * t;
  // sigma = S when active
  Sb += sigb;
  // scatter the side-K quantities to L or R
  double rLb = 0, nLb = 0, tLb = 0, pLb = 0, rRb = 0, nRb = 0, tRb = 0, pRb = 0;
  double SLb = 0, SRb = 0, mLb = 0, mRb = 0;
  if (left) {
    rLb += rb; nLb += nb; tLb += tb; pLb += pb; SLb += Sb; mLb += mb;
  } else {
    rRb += rb; nRb += nb; tRb += tb; pRb += pb; SRb += Sb; mRb += mb;
  }
  // SS = num / dn
  const double numb = SSb / dn;
  const double dnb = -SSb * SS / dn;
  pRb += numb;
  pLb -= numb;
  mLb += numb * L.n + dnb;
  nLb += numb * mL;
  mRb -= numb * R.n + dnb;
  nRb -= numb * mR;
  // m_K = r_K (S_K - n_K)
  rLb += mLb * dL;
  SLb += mLb * L.r;
  nLb -= mLb * L.r;
  rRb += mRb * dR;
  SRb += mRb * R.r;
  nRb -= mRb * R.r;
  // Davis speeds
  double cLb = 0.0, cRb = 0.0;
  if (selL) { nLb += SLb; cLb -= SLb; } else { nRb += SLb; cRb -= SLb; }
  if (selR) { nLb += SRb; cLb += SRb; } else { nRb += SRb; cRb += SRb; }
  // c = sqrt(g p / r)
  pLb += cLb * g / (2.0 * cL * L.r);
  rLb -= cLb * cL / (2.0 * L.r);
  pRb += cRb * g / (2.0 * cR * R.r);
  rRb -= cRb * cR / (2.0 * R.r);
  Lb.r += rLb; Lb.n += nLb; Lb.t += tLb; Lb.p += pLb;
  Rb.r += rRb; Rb.n += nRb; Rb.t += tRb; Rb.p += pRb;
}

// Wall pressure: top wall (interior below the face, on the left of the
// face-normal problem) p* = p + r n (|n| + c + n); bottom wall (interior
// above, on the right) p* = p - r n (|n| + c - n).
RT_DEV double wall_pressure(const Params& P, const FS& w, bool top) {
  const double c = sqrt(P.gamma * w.p / w.r);
  const double an = w.n < -kTieTol * c ? -w.n : w.n;  // |n|; near-zero n counts as >= 0
  return top ? w.p + w.r * w.n * (an + c + w.n) : w.p - w.r * w.n * (an + c - w.n);
}

RT_DEV void wall_pressure_adj(const Params& P, const FS& w, bool top, double psb, FS& wb) {
  const double c = sqrt(P.gamma * w.p / w.r);
  const bool neg = w.n < -kTieTol * c;
  const double sg = neg ? -1.0 : 1.0;
  const double an = neg ? -w.n : w.n;
  double qb, nb;
  if (top) {
    const double q = an + c + w.n;
    wb.r += psb * w.n * q;
    nb = psb * w.r * q;
    qb = psb * w.r * w.n;
    nb += qb * (sg + 1.0);
  } else {
    const double q = an + c - w.n;
    wb.r -= psb * w.n * q;
    nb = -psb * w.r * q;
    qb = -psb * w.r * w.n;
    nb += qb * (sg - 1.0);
  }
  wb.n += nb;
  wb.p += psb;
  // c = sqrt(gamma p / r)
  wb.p += qb * P.gamma / (2.0 * c * w.r);
  wb.r -= qb * c / (2.0 * w.r);
}

// Largest signal speed of a state, for the CFL step.
RT_DEV double signal_speed(const Params& P, double r, double mx, double my, double E) {
  const W4 w = cons_to_prim(P, r, mx, my, E);
  const double c = sqrt(P.gamma * w.p / w.r);
  const double sx = (fabs(w.u) + c) * P.inv_dx, sy = (fabs(w.v) + c) * P.inv_dy;
  return sx > sy ? sx : sy;
}

}  // namespace rtk
