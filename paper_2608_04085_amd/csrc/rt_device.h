// Device arithmetic of the MI355X hot path: the pieces of one finite-volume
// step (primitive variables, limited slopes, MUSCL-Hancock predictor, HLLC
// flux, wall flux, update with gravity) and the hand-derived adjoint of each.
//
// Scheme (the paper fixes the PDE, Sec. 2.1 Eqs. 1-4, and the scheme family,
// a Godunov-type finite-volume method with an HLLC solver and a gravity
// source, Sec. 2.3; the rest is this implementation's reading):
//   * primitive variables W = (rho, u, v, p), p = (gamma-1)(E - |m|^2/(2 rho));
//   * monotonized-central (MC) limited slopes: zero if a*b <= 0 or a
//     difference is negligible (below 1e-10 of the local scale), else
//     sign(a) min(2|a|, 2|b|, |a+b|/2) -- the central difference when it does
//     not exceed 2|a| and 2|b|, else 2a if |a| <= |b|, else 2b;
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
//
// Arithmetic: the gfx950 reciprocal and reciprocal-square-root estimates
// (v_rcp_f64, v_rsq_f64) are good to about 2^-24; two Newton steps bring
// them to within an ulp or two of the correctly rounded result.  Divisions
// are products with shared reciprocals, and the HLLC star flux is rearranged
// so that E/rho and p/m need no division.  The forward kernel and the
// adjoint's recomputation call the same functions, so both see the same
// values and take the same decisions.
#pragma once
#include <hip/hip_runtime.h>

namespace rtk {

struct Params {
  int nx, ny, nb, comp_mask;
  double dx, dy, inv_dx, inv_dy;
  double gamma, gm1, inv_gm1, g_y, cfl;
  double rho_h, rho_l, y0, h, p_int;
  int recon, pad;  // recon 1: well-balanced variant (mc_p_balanced, row-balanced background)
};

// Primitive state plus the reciprocal density, which later steps reuse.
struct W4 {
  double r, u, v, p, ri;
};

#define RT_DEV __device__ __forceinline__

// 1/b for a normal b: hardware estimate + two Newton steps.
RT_DEV double rcp(double b) {
  double r = __builtin_amdgcn_rcp(b);
  double e = fma(-b, r, 1.0);
  r = fma(r, e, r);
  e = fma(-b, r, 1.0);
  return fma(r, e, r);
}

// sqrt(x) and 1/sqrt(x) for a positive normal x: reciprocal square-root
// estimate, then two coupled Newton (Goldschmidt) steps on both.
RT_DEV void sqrt_rsqrt(double x, double& s, double& rs) {
  const double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * y;
  double g = x * y;
  double e = fma(-g, h, 0.5);  // 1/2 - x y^2 / 2
  g = fma(g, e, g);
  h = fma(h, e, h);
  e = fma(-g, h, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  s = g;
  rs = 2.0 * h;
}

RT_DEV double sqrt_fast(double x) {
  double s, rs;
  sqrt_rsqrt(x, s, rs);
  return s;
}

RT_DEV W4 cons_to_prim(const Params& P, double r, double mx, double my, double E) {
  const double ri = rcp(r);
  const double u = mx * ri, v = my * ri;
  W4 w;
  w.r = r;
  w.u = u;
  w.v = v;
  w.p = P.gm1 * (E - 0.5 * (mx * u + my * v));
  w.ri = ri;
  return w;
}

RT_DEV bool unphysical(const W4& w) {
  // also catches NaN: comparisons with NaN are false
  return !(w.r > 0.0) || !(w.p > 0.0) || !(fabs(w.u) < 1e300) || !(fabs(w.v) < 1e300);
}

// Adjoint of cons_to_prim: W-bar -> U-bar at the state (r, u, v).
RT_DEV void prim_adj(const Params& P, const W4& w, const W4& wb, double ub[4]) {
  const double ri = w.ri;
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

// MC-limited slope: zero if a*b <= 0 or a difference is negligible, else
// sign(a) min(2|a|, 2|b|, |a+b|/2), which equals the value of the case
// (central, 2a or 2b) that the limiter selects.
RT_DEV double mc_value(double a, double b, bool small_a, bool small_b) {
  const bool zero = (a * b <= 0.0) || small_a || small_b;
  const double m = fmin(fmin(2.0 * fabs(a), 2.0 * fabs(b)), fabs(0.5 * (a + b)));
  return zero ? 0.0 : copysign(m, a);
}

// The limiter's case, for the adjoint: 0 zero, 1 central, 2 -> 2a, 3 -> 2b.
// Where two cases give the same value the central one, then 2a, is taken.
RT_DEV int mc_code(double a, double b, bool small_a, bool small_b) {
  const double c = 0.5 * (a + b);
  const double aa = fabs(a), ab = fabs(b), ac = fabs(c);
  const bool zero = (a * b <= 0.0) || small_a || small_b;
  const bool central = (ac <= 2.0 * aa) && (ac <= 2.0 * ab);
  const bool left = aa <= ab;
  return zero ? 0 : (central ? 1 : (left ? 2 : 3));
}

// Weights (d s/d a, d s/d b) of an MC case.
RT_DEV void mc_weights(int code, double& wa, double& wb) {
  wa = code == 1 ? 0.5 : (code == 2 ? 2.0 : 0.0);
  wb = code == 1 ? 0.5 : (code == 3 ? 2.0 : 0.0);
}

// Slopes of the four primitives (and, if CODES, their cases packed 2 bits
// per variable).  A difference is negligible below kTieTol times the centre
// cell's density, pressure, or sound speed (velocities: d^2 <= kTieTol^2
// gamma p / rho).
template <bool CODES>
RT_DEV W4 mc4(const Params& P, const W4& m, const W4& c, const W4& p, int& codes) {
  const double tr = kTieTol * c.r, tp = kTieTol * c.p, tv2 = kTieTol * kTieTol * P.gamma * c.p * c.ri;
  W4 s;
  const double ar = c.r - m.r, br = p.r - c.r;
  const double au = c.u - m.u, bu = p.u - c.u;
  const double av = c.v - m.v, bv = p.v - c.v;
  const double ap = c.p - m.p, bp = p.p - c.p;
  const bool sar = fabs(ar) <= tr, sbr = fabs(br) <= tr;
  const bool sau = au * au <= tv2, sbu = bu * bu <= tv2;
  const bool sav = av * av <= tv2, sbv = bv * bv <= tv2;
  const bool sap = fabs(ap) <= tp, sbp = fabs(bp) <= tp;
  s.r = mc_value(ar, br, sar, sbr);
  s.u = mc_value(au, bu, sau, sbu);
  s.v = mc_value(av, bv, sav, sbv);
  s.p = mc_value(ap, bp, sap, sbp);
  s.ri = 0.0;
  if (CODES)
    codes = mc_code(ar, br, sar, sbr) | (mc_code(au, bu, sau, sbu) << 2) | (mc_code(av, bv, sav, sbv) << 4) |
            (mc_code(ap, bp, sap, sbp) << 6);
  return s;
}

// y slope of the pressure in the well-balanced variant: the cell's own
// hydrostatic slope h = rho g_y dy plus the MC slope of the departures from
// it, a' = (p_c - p_m) - h and b' = (p_p - p_c) - h (tie tolerance as for the
// pressure in mc4).  Replaces s.p (and, if CODES, the pressure's case in
// codes).  For a row-balanced state with monotone density a' and b' vanish
// or differ in sign, so the two pressures at a face agree and the pressure
// difference across the cell cancels the gravity source.
template <bool CODES>
RT_DEV void mc_p_balanced(const Params& P, const W4& m, const W4& c, const W4& p, W4& s, int& codes) {
  const double h = c.r * (P.g_y * P.dy);
  const double tp = kTieTol * c.p;
  const double a = (c.p - m.p) - h, b = (p.p - c.p) - h;
  const bool sa = fabs(a) <= tp, sb = fabs(b) <= tp;
  s.p = h + mc_value(a, b, sa, sb);
  if (CODES) codes = (codes & ~(3 << 6)) | (mc_code(a, b, sa, sb) << 6);
}

// Ghost cells of the y walls: mirror of the adjacent interior cell with the
// normal velocity negated and the pressure extrapolated hydrostatically
// (dp/dy = rho g_y) over the distance between the two cell centres.
RT_DEV W4 ghost_bottom(const Params& P, const W4& w) {
  return W4{w.r, w.u, -w.v, w.p - P.g_y * w.r * P.dy, w.ri};
}
RT_DEV W4 ghost_top(const Params& P, const W4& w) {
  return W4{w.r, w.u, -w.v, w.p + P.g_y * w.r * P.dy, w.ri};
}

// MUSCL-Hancock half step: q = W - hx A_x(W) sx - hy A_y(W) sy + (dt/2) g.
RT_DEV W4 predict(const Params& P, const W4& w, const W4& sx, const W4& sy, double hx, double hy,
                  double half_dt_g) {
  const double ri = w.ri;
  W4 q;
  q.r = w.r - hx * (w.u * sx.r + w.r * sx.u) - hy * (w.v * sy.r + w.r * sy.v);
  q.u = w.u - hx * (w.u * sx.u + sx.p * ri) - hy * (w.v * sy.u);
  q.v = w.v - hx * (w.u * sx.v) - hy * (w.v * sy.v + sy.p * ri) + half_dt_g;
  q.p = w.p - hx * (P.gamma * w.p * sx.u + w.u * sx.p) - hy * (P.gamma * w.p * sy.v + w.v * sy.p);
  q.ri = 0.0;
  return q;
}

// Adjoint of predict: q-bar -> (W-bar, sx-bar, sy-bar), accumulated.
RT_DEV void predict_adj(const Params& P, const W4& w, const W4& sx, const W4& sy, double hx, double hy,
                        const W4& qb, W4& wb, W4& sxb, W4& syb) {
  const double ri = w.ri;
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
// S_L >= 0 / S* >= 0 / S_R > 0 / else in one formula.  With d = S_K - n_K,
// m = rho_K d and k = 1/(S_K - S*), the star state is
//   U*_K = (m k, m k S*, m k t, k (d E_K + (S* - n_K)(m S* + p_K))),
// the textbook star state with E/rho and p/m multiplied out.
struct FS {
  double r, n, t, p;
};

// Intermediates of one HLLC evaluation, shared by the flux and its adjoint.
struct HllcCore {
  double cL, cR, rcL, rcR, riL, riR;  // sound speeds, their reciprocals, 1/rho
  bool selL, selR, left, act;
  double SL, SR, dL, dR, mL, mR, rdn, SS;
  // selected side K
  double r, n, t, p, S, d, m, sig, E, m0, k, f, A, B2, G;
};

RT_DEV HllcCore hllc_core(const Params& P, const FS& L, const FS& R) {
  HllcCore h;
  const double g = P.gamma;
  h.riL = rcp(L.r);
  h.riR = rcp(R.r);
  sqrt_rsqrt(g * L.p * h.riL, h.cL, h.rcL);
  sqrt_rsqrt(g * R.p * h.riR, h.cR, h.rcR);
  const double tie = kTieTol * (h.cL + h.cR);  // near-ties resolve to the left state
  const double aL = L.n - h.cL, bL = R.n - h.cR, aR = L.n + h.cL, bR = R.n + h.cR;
  h.selL = aL <= bL + tie;
  h.selR = aR >= bR - tie;
  h.SL = h.selL ? aL : bL;
  h.SR = h.selR ? aR : bR;
  h.dL = h.SL - L.n;
  h.dR = h.SR - R.n;
  h.mL = L.r * h.dL;
  h.mR = R.r * h.dR;
  const double num = R.p - L.p + h.mL * L.n - h.mR * R.n;
  h.rdn = rcp(h.mL - h.mR);
  h.SS = num * h.rdn;
  h.left = h.SS >= -tie;
  h.r = h.left ? L.r : R.r;
  h.n = h.left ? L.n : R.n;
  h.t = h.left ? L.t : R.t;
  h.p = h.left ? L.p : R.p;
  h.S = h.left ? h.SL : h.SR;
  h.d = h.left ? h.dL : h.dR;
  h.m = h.left ? h.mL : h.mR;
  h.act = h.left ? (h.SL < 0.0) : (h.SR > 0.0);
  h.sig = h.act ? h.S : 0.0;
  h.E = h.p * P.inv_gm1 + 0.5 * h.r * (h.n * h.n + h.t * h.t);
  h.m0 = h.r * h.n;
  h.k = h.act ? rcp(h.S - h.SS) : 0.0;
  h.f = h.m * h.k;
  h.A = h.SS - h.n;
  h.B2 = h.m * h.SS + h.p;
  h.G = h.d * h.E + h.A * h.B2;
  return h;
}

RT_DEV void hllc(const Params& P, const FS& L, const FS& R, double F[4]) {
  const HllcCore h = hllc_core(P, L, R);
  const double fH = h.k * h.G;
  F[0] = h.m0 + h.sig * (h.f - h.r);
  F[1] = h.m0 * h.n + h.p + h.sig * (h.f * h.SS - h.m0);
  F[2] = h.m0 * h.t + h.sig * (h.f * h.t - h.r * h.t);
  F[3] = h.n * (h.E + h.p) + h.sig * (fH - h.E);
}

// Adjoint of hllc: given F-bar, accumulate L-bar and R-bar (reverse of the
// computational graph of hllc_core + hllc).  F, if not null, also receives
// the flux itself (as hllc gives it).
RT_DEV void hllc_adj(const Params& P, const FS& L, const FS& R, const double Fb[4], FS& Lb, FS& Rb,
                     double* F = nullptr) {
  const HllcCore h = hllc_core(P, L, R);
  const double g = P.gamma;
  const double fH = h.k * h.G;
  const double sig = h.sig;
  if (F) {
    F[0] = h.m0 + h.sig * (h.f - h.r);
    F[1] = h.m0 * h.n + h.p + h.sig * (h.f * h.SS - h.m0);
    F[2] = h.m0 * h.t + h.sig * (h.f * h.t - h.r * h.t);
    F[3] = h.n * (h.E + h.p) + h.sig * (fH - h.E);
  }
  // F0 = m0 + sig (f - r); F1 = m0 n + p + sig (f SS - m0);
  // F2 = m0 t + sig (f t - r t); F3 = n (E + p) + sig (fH - E)
  const double sigb =
      h.act ? (Fb[0] * (h.f - h.r) + Fb[1] * (h.f * h.SS - h.m0) + Fb[2] * (h.f * h.t - h.r * h.t) + Fb[3] * (fH - h.E))
            : 0.0;
  const double fb = sig * (Fb[0] + Fb[1] * h.SS + Fb[2] * h.t);
  const double fHb = sig * Fb[3];
  double SSb = sig * Fb[1] * h.f;
  double tb = Fb[2] * (h.m0 + sig * (h.f - h.r));
  double rb = -sig * (Fb[0] + Fb[2] * h.t);
  const double m0b = Fb[0] + Fb[1] * h.n + Fb[2] * h.t - sig * Fb[1];
  double nb = Fb[1] * h.m0 + Fb[3] * (h.E + h.p);
  double pb = Fb[1] + Fb[3] * h.n;
  double Eb = Fb[3] * (h.n - sig);
  // fH = k G, G = d E + A B2, A = SS - n, B2 = m SS + p
  double kb = fHb * h.G;
  const double Gb = fHb * h.k;
  const double db = Gb * h.E;
  Eb += Gb * h.d;
  const double Ab = Gb * h.B2, B2b = Gb * h.A;
  double mb = B2b * h.SS;
  SSb += B2b * h.m + Ab;
  pb += B2b;
  nb -= Ab;
  // f = m k
  mb += fb * h.k;
  kb += fb * h.m;
  // k = 1/(S - SS) when active
  double Sb = 0.0;
  if (h.act) {
    const double kk = kb * h.k * h.k;
    Sb -= kk;
    SSb += kk;
  }
  // m0 = r n
  rb += m0b * h.n;
  nb += m0b * h.r;
  // E = p/(g-1) + r (n^2 + t^2)/2
  pb += Eb * P.inv_gm1;
  rb += Eb * 0.5 * (h.n * h.n + h.t * h.t);
  nb += Eb * h.r * h.n;
  tb += Eb * h.r * h.t;
  // sigma = S when active
  Sb += sigb;
  // scatter the side-K quantities to L or R
  double rLb = 0, nLb = 0, tLb = 0, pLb = 0, rRb = 0, nRb = 0, tRb = 0, pRb = 0;
  double SLb = 0, SRb = 0, mLb = 0, mRb = 0, dLb = 0, dRb = 0;
  if (h.left) {
    rLb += rb; nLb += nb; tLb += tb; pLb += pb; SLb += Sb; mLb += mb; dLb += db;
  } else {
    rRb += rb; nRb += nb; tRb += tb; pRb += pb; SRb += Sb; mRb += mb; dRb += db;
  }
  // SS = num / dn, dn = mL - mR, num = pR - pL + mL nL - mR nR
  const double numb = SSb * h.rdn;
  const double dnb = -SSb * h.SS * h.rdn;
  pRb += numb;
  pLb -= numb;
  mLb += numb * L.n + dnb;
  nLb += numb * h.mL;
  mRb -= numb * R.n + dnb;
  nRb -= numb * h.mR;
  // m_K = r_K d_K, d_K = S_K - n_K
  rLb += mLb * h.dL;
  dLb += mLb * L.r;
  rRb += mRb * h.dR;
  dRb += mRb * R.r;
  SLb += dLb;
  nLb -= dLb;
  SRb += dRb;
  nRb -= dRb;
  // Davis speeds
  double cLb = 0.0, cRb = 0.0;
  if (h.selL) { nLb += SLb; cLb -= SLb; } else { nRb += SLb; cRb -= SLb; }
  if (h.selR) { nLb += SRb; cLb += SRb; } else { nRb += SRb; cRb += SRb; }
  // c = sqrt(g p / r): dc/dp = g/(2 c r), dc/dr = -c/(2 r)
  pLb += cLb * 0.5 * g * h.rcL * h.riL;
  rLb -= cLb * 0.5 * h.cL * h.riL;
  pRb += cRb * 0.5 * g * h.rcR * h.riR;
  rRb -= cRb * 0.5 * h.cR * h.riR;
  Lb.r += rLb; Lb.n += nLb; Lb.t += tLb; Lb.p += pLb;
  Rb.r += rRb; Rb.n += nRb; Rb.t += tRb; Rb.p += pRb;
}

// Wall pressure: top wall (interior below the face, on the left of the
// face-normal problem) p* = p + r n (|n| + c + n); bottom wall (interior
// above, on the right) p* = p - r n (|n| + c - n).
RT_DEV double wall_pressure(const Params& P, const FS& w, bool top) {
  const double c = sqrt_fast(P.gamma * w.p * rcp(w.r));
  const double an = w.n < -kTieTol * c ? -w.n : w.n;  // |n|; near-zero n counts as >= 0
  return top ? w.p + w.r * w.n * (an + c + w.n) : w.p - w.r * w.n * (an + c - w.n);
}

RT_DEV void wall_pressure_adj(const Params& P, const FS& w, bool top, double psb, FS& wb) {
  const double ri = rcp(w.r);
  double c, rc;
  sqrt_rsqrt(P.gamma * w.p * ri, c, rc);
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
  wb.p += qb * 0.5 * P.gamma * rc * ri;
  wb.r -= qb * 0.5 * c * ri;
}

// Largest signal speed of a state, for the CFL step.
RT_DEV double signal_speed(const Params& P, double r, double mx, double my, double E) {
  const W4 w = cons_to_prim(P, r, mx, my, E);
  const double c = sqrt_fast(P.gamma * w.p * w.ri);
  const double sx = (fabs(w.u) + c) * P.inv_dx, sy = (fabs(w.v) + c) * P.inv_dy;
  return sx > sy ? sx : sy;
}

// The same speed and its gradient with respect to (r, m_x, m_y, E), the
// speed's branch (x or y; y on a tie) and |.| (slope +1 at 0) taken as
// signal_speed takes them.  With c^2 = gamma p / r,
//   dc = (c/2) (dp/p - dr/r),  dp = (gamma - 1) ((u^2+v^2)/2, -u, -v, 1),
//   d|u| = sign(u) (-u/r, 1/r, 0, 0),  d|v| = sign(v) (-v/r, 0, 1/r, 0).
RT_DEV double signal_speed_grad(const Params& P, double r, double mx, double my, double E, double d[4]) {
  const W4 w = cons_to_prim(P, r, mx, my, E);
  const double c = sqrt_fast(P.gamma * w.p * w.ri);
  const double sx = (fabs(w.u) + c) * P.inv_dx, sy = (fabs(w.v) + c) * P.inv_dy;
  const double hp = 0.5 * c * rcp(w.p) * P.gm1;  // (c/2) (gamma - 1) / p
  const double dc[4] = {hp * 0.5 * (w.u * w.u + w.v * w.v) - 0.5 * c * w.ri, -hp * w.u, -hp * w.v, hp};
  const bool xs = sx > sy;
  const double a = xs ? w.u : w.v;
  const double sg = (a < 0.0 ? -1.0 : 1.0) * w.ri;
  const double inv = xs ? P.inv_dx : P.inv_dy;
  d[0] = (dc[0] - sg * a) * inv;
  d[1] = (dc[1] + (xs ? sg : 0.0)) * inv;
  d[2] = (dc[2] + (xs ? 0.0 : sg)) * inv;
  d[3] = dc[3] * inv;
  return xs ? sx : sy;
}

}  // namespace rtk
