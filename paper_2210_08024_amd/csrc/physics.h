// Device microphysics of the ISM source step (Secs. 3-4 of arXiv:2210.08024).
//
// One lane evaluates one cell.  Templated on R, the type the terms are formed and
// stored in: double on the plain path, float on the mixed path.  On both paths the
// temperature stays double and every exponent (E/T, p ln T, p ln psi, table values)
// is formed in double; Mx<R>::ex turns a double exponent into an R result.  For float
// that is a 2^k 2^f split with |f| <= 1/2 and the hardware exp2 on f only, so the
// result carries ~1 float ulp whatever the size of the exponent; the algebra around
// the transcendentals runs in R, and the few cancelling differences (x_H, x_O, the
// fit polynomials) in double.  FP64 FMA issues at the FP32 rate on CDNA4, so the
// double pieces cost little; what float saves are the transcendental sequences.
#pragma once
#include <hip/hip_runtime.h>

#include "coef.h"
#include "fmath.h"
#include <type_traits>

namespace ism {

// The double copy of the coefficients (constant memory, defined with the kernels).
__device__ __forceinline__ const CoefT<double> &coef64();

constexpr double LOG2E = 1.4426950408889634074;
constexpr double LN2 = 0.69314718055994530942;
constexpr double LN100 = 4.6051701859880913680;
constexpr double LN1E3 = 6.9077552789821370520;
constexpr double LN1E4 = 9.2103403719761827361;
constexpr double LN10D = 2.3025850929940456840;
constexpr double INV_LN10D = 0.43429448190325182765;  // 1 / ln 10

// ---------------------------------------------------------------- math policies
template <class R> struct Mx;

template <> struct Mx<double> {
  static __device__ __forceinline__ double ex(double x) { return fexp(x); }
  // every log the step takes is of a positive finite number (T, psi >= 50, 1 + c T, guarded
  // columns and densities, n, a floored xi)
  static __device__ __forceinline__ double ln(double x) { return flogp(x); }
  static __device__ __forceinline__ double sq(double x) { return ::sqrt(x); }
  static __device__ __forceinline__ double cb(double x) { return ::cbrt(x); }
};

template <> struct Mx<float> {
  // exp of a double exponent: x log2(e) = k + f, |f| <= 1/2, result 2^f (hardware) scaled by 2^k;
  // x clamped to +-200 ln 2 (beyond float range either way), k by the 1.5 2^52 shift (the
  // integer is the low word of kd), f = x log2(e) - k with one rounding.
  static __device__ __forceinline__ float ex(double x) {
    x = __builtin_fmin(__builtin_fmax(x, -200.0 * LN2), 200.0 * LN2);
    const double kd = fma(x, LOG2E, 0x1.8p52);
    const double k = kd - 0x1.8p52;
    const float r = __builtin_amdgcn_exp2f((float)fma(x, LOG2E, -k));
    return ::ldexpf(r, (int)(uint32_t)__builtin_bit_cast(uint64_t, kd));
  }
  // natural log as a double: exponent from frexp, mantissa in [0.5, 1) through the hardware log2.
  static __device__ __forceinline__ double ln(double x) {
    const int e = __builtin_amdgcn_frexp_exp(x);
    const float m = (float)__builtin_amdgcn_frexp_mant(x);
    return ((double)e + (double)__builtin_amdgcn_logf(m)) * LN2;
  }
  static __device__ __forceinline__ float sq(float x) { return __fsqrt_rn(x); }
  static __device__ __forceinline__ float cb(float x) { return ::cbrtf(x); }
};

template <class R> __device__ __forceinline__ R rmax(R a, R b) { return a > b ? a : b; }
template <class R> __device__ __forceinline__ R rmin(R a, R b) { return a < b ? a : b; }

// The kernel's own argument block (at the start of the kernarg segment) through a pointer
// laundered by an empty asm: loads through it are not hoisted above the call.  A kernel that
// takes it afresh inside its loop keeps two scalar registers live across the loop instead of
// every field it reads, which would spill into vector-register lanes and cost a lane read per use.
template <class A>
__device__ __forceinline__ const A &kernel_args() {
  const __attribute__((address_space(4))) A *p =
      (const __attribute__((address_space(4))) A *)__builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(p));
  return *(const A *)p;
}

// ---------------------------------------------------------------- tables
// a / b at a site whose denominator is a positive number in [2^-1000, 2^1000] (a sum with a
// positive floor, a temperature, a density): in double the reciprocal-based division, in float
// the plain one.
template <class R>
__device__ __forceinline__ R dvp(R a, R b) {
  if constexpr (std::is_same<R, double>::value) return fdivp(a, b);
  else return a / b;
}

// Clamp x to the grid [x0, x0 + (n-1) dx]; lower node index and fraction (in double).
// idx = 1 / dx.
__device__ __forceinline__ void axis_pos(double x, double x0, double dx, double idx, int n, int &i, double &f) {
  const double hi = x0 + (double)(n - 1) * dx;
  const double xc = x < x0 ? x0 : (x > hi ? hi : x);
  const double u = (xc - x0) * idx;
  int k = (int)floor(u);
  k = k > 0 ? k : 0;  // also maps a NaN argument to node 0
  i = k < n - 2 ? k : n - 2;
  f = u - (double)i;
}

template <class R>
__device__ __forceinline__ double cie_lookup(const R *tab, double lgT, int col) {
  const CoefT<double> &c = coef64();
  int i;
  double f;
  axis_pos(lgT, c.cie_x0, c.cie_dx, c.cie_idx, CIE_N, i, f);
  const R *v = tab + TAB_CIE;
  return (double)v[i * CIE_NC + col] * (1.0 - f) + (double)v[(i + 1) * CIE_NC + col] * f;
}

template <class R>
__device__ __forceinline__ double co_lookup(const R *tab, double lT, double lN, int col) {
  const CoefT<double> &c = coef64();
  int i, j;
  double f, g;
  axis_pos(lT, c.co_x0, c.co_dx, c.co_idx, CO_NX, i, f);
  axis_pos(lN, c.co_y0, c.co_dy, c.co_idy, CO_NY, j, g);
  const R *v = tab + TAB_CO;
  const double v00 = v[(i * CO_NY + j) * CO_NC + col], v01 = v[(i * CO_NY + j + 1) * CO_NC + col];
  const double v10 = v[((i + 1) * CO_NY + j) * CO_NC + col], v11 = v[((i + 1) * CO_NY + j + 1) * CO_NC + col];
  return (v00 * (1.0 - g) + v01 * g) * (1.0 - f) + (v10 * (1.0 - g) + v11 * g) * f;
}

// ---------------------------------------------------------------- per-cell inputs
template <class R>
struct Rad {
  R chiPE, chiLW, chiH2, chiC, phi, xi, Neff;
  // terms fixed by the cell's density and radiation for the whole step (fixed_terms)
  R G;      // dust heating per Z'_d
  R qH2;    // heat per CR ionisation of H2, erg
  R ncrit;  // critical density of the CO fit
  R qn2;    // (ncrit / n)^2
  R G0f;    // FUV field G0
};

template <class R>
struct EqS {
  R xCp, xCO, xC, xOp, xO, xe;
};

// Everything the update needs from one evaluation; Gamma/Lambda/H in double.  Tds is dT_d/dT
// at the dust temperature found (0 where none was), for the next solve's starting point.
template <class R>
struct Eval {
  R F, D, I, Rr;
  double CH2, CHp, Td, Tds, Gamma, Lambda, H;
  bool td_bad;
};

// Temperature-derived quantities shared by every term of one evaluation (sqrtT serves the
// double terms; the float path takes its own root of T).
struct Tq {
  double T, lnT, invT, lnT4, sqrtT;
};

// ln T in double on both paths: it feeds polynomial fits in log T whose terms cancel (the
// nebular and rovibrational cooling), which would magnify the float log's absolute error.
template <class R>
__device__ __forceinline__ Tq make_tq(double T) {
  Tq q;
  q.T = T;
  q.lnT = flogp(T);
  q.invT = fdivp(1.0, T);
  q.lnT4 = q.lnT - LN1E4;
  q.sqrtT = Mx<double>::sq(T);
  return q;
}

// The same quantities at T (1 + fd_rel), the second point of the finite-difference derivative
// of Sec. 6.1: ln, reciprocal and root of T there follow from those at T and the host's values
// for 1 + fd_rel (one rounding each, against a log, a division and a root).
template <class R>
__device__ __forceinline__ Tq shift_tq(const Tq &q, const ParT<double> &pd) {
  Tq s;
  s.T = q.T * (1.0 + pd.fd_rel);
  s.lnT = q.lnT + pd.fd_ln;
  s.invT = q.invT * pd.fd_inv;
  s.lnT4 = s.lnT - LN1E4;
  s.sqrtT = q.sqrtT * pd.fd_sqrt;
  return s;
}

// ---------------------------------------------------------------- rate coefficients (Sec. 3)
template <class R>
__device__ __forceinline__ R k_gr(const Tq &q, R sqrtT, const CoefT<R> &c, const ParT<R> &p) {
  if (p.kgr_const) return c.kgr0 * p.Zd;
  const R T2 = R(q.T * 0.01);
  // (T / 100)^1/2: from sqrt T in double; in float its own root (a float product there moved the
  // mixed path's most sensitive cells past their tolerance)
  const R s = std::is_same<R, double>::value ? sqrtT * R(0.1) : Mx<R>::sq(T2);
  return dvp<R>(c.kgr0 * p.Zd * c.kgr_shape[0] * s,
                R(1) + c.kgr_shape[1] * s + c.kgr_shape[2] * T2 + c.kgr_shape[3] * T2 * T2);
}

// Grain-assisted recombination 1e-14 C0 Z'_d / (1 + C1 psi^C2 (1 + C3 T^C4 psi^(-C5 - C6 ln T))).
template <class R>
__device__ __forceinline__ R alpha_gr(const Tq &q, double lnpsi, const double *k, R Zd) {
  const R a = Mx<R>::ex(k[2] * lnpsi);
  const R b = Mx<R>::ex(k[4] * q.lnT + (-k[5] - k[6] * q.lnT) * lnpsi);
  return dvp<R>(R(1e-14 * k[0]) * Zd, R(1) + R(k[1]) * a * (R(1) + R(k[3]) * b));
}

// FUV field G0 of a cell from its attenuation factors (Sec. 4.2).
template <class R>
__device__ __forceinline__ R g0_field(R chiPE, R chiLW, const CoefT<R> &c) {
  return c.G0_per_chi * ((c.J_PE * chiPE + c.J_LW * chiLW) * c.inv_J_FUV);
}

// Grain charging parameter G0 T^1/2 / n_e + 50 (Sec. 4.2), n_e floored at 1e-20 n.
template <class R>
__device__ __forceinline__ R psi_charge(R sqrtT, R n, R xe, R G0, const CoefT<R> &c) {
  return dvp<R>(G0 * sqrtT, n * rmax(xe, R(1e-20))) + c.psi_off;
}

// ---------------------------------------------------------------- C / O / e closure
// Secs. 3.2-3.3: x_O+ = x_O,tot x_H+; C+ from Eq. eq:C+_frac with n_e = n (x_e0 + x_C+)
// (positive root of the quadratic, psi iterated to a fixed point in x_e) below 2e4 K,
// Eq. e:xELhot above; CO from Eqs. e:CO, e:CO_fit with chi_CO = chi_LW.
template <class R>
__device__ EqS<R> eq_species(const Tq &q, R n, double xH2_d, double xHp_d, const Rad<R> &r, const CoefT<R> &c,
                             const ParT<R> &p, const R *tab, R tol, int maxit) {
  const CoefT<double> &cd = coef64();
  EqS<R> e;
  const double T = q.T;
  const R xH2 = R(xH2_d), xHp = R(xHp_d);
  const R sqrtT = std::is_same<R, double>::value ? R(q.sqrtT) : Mx<R>::sq(R(T));
  const R xCt = p.xCt, xOt = p.xOt, Zd = p.Zd;
  e.xOp = xOt * xHp;
  const R a = c.zeta_pi_C * r.chiC + c.zeta_pi_C_cr * R(2) * xH2 * r.xi + c.zeta_cr_C * r.xi;
  const R cc = R(cd.arrdr_Cp[0]) * Mx<R>::ex(cd.arrdr_Cp[2] * (q.lnT - cd.ln_arrdr_T0)) * n;
  const R kch = R(cd.k_CpH2[0]) * Mx<R>::ex(cd.k_CpH2[1] * q.lnT - cd.k_CpH2[2] * q.invT) * n * xH2;
  // comp = 1 - x_C+ / x_C,tot, the neutral share of the carbon.  The float path takes it from the
  // C+ balance itself rather than by subtraction: with the carbon nearly all ionised the quotient
  // sits within a few ulps of 1 and the subtraction would keep none of the complement's digits.
  //   hot:  y = x_C,tot a / (a + B + c x_e)            =>  comp = (B + c x_e) / (a + B + c x_e)
  //   cold: c y^2 + (a + B + c x_e0) y = x_C,tot a     =>  comp = y (B + c (x_e0 + y)) / (a x_C,tot)
  // with B the value the final root was taken with.
  R y, xe, comp;
  if (T >= cd.xe_T_switch) {
    const double lgT = q.lnT * INV_LN10D;
    xe = xHp + R(cie_lookup(tab, lgT, 2)) + p.Zg * R(cie_lookup(tab, lgT, 3));
    const R psi = psi_charge(sqrtT, n, xe, r.G0f, c);
    const R B = alpha_gr<R>(q, Mx<R>::ln((double)psi), cd.agr_Cp, Zd) * n + kch;
    const R dh = a + B + cc * xe;
    y = a > R(0) ? xCt * a / (dh > R(0) ? dh : R(1)) : R(0);
    comp = a > R(0) ? (B + cc * xe) / (dh > R(0) ? dh : R(1)) : R(1);
  } else {
    const R amh = R(cd.x_MH[1]) * Mx<R>::ex(cd.x_MH[3] * (q.lnT - cd.ln_xMH_T0));
    const R xmh = R(2) * xH2 * Mx<R>::sq(dvp<R>(c.x_MH[0] * r.xi, amh * n));
    const R xe0 = xHp + e.xOp + xmh;
    xe = xe0 + xCt;
    y = R(0);
    R B = R(0);
    for (int it = 0; it < maxit; ++it) {
      const R psi = psi_charge(sqrtT, n, xe, r.G0f, c);
      B = alpha_gr<R>(q, Mx<R>::ln((double)psi), cd.agr_Cp, Zd) * n + kch;
      const R pp = a + B + cc * xe0;
      const R den = pp + Mx<R>::sq(pp * pp + R(4) * cc * xCt * a);
      // (a can be as small as the shielded photoionisation rate alone: the plain division)
      y = a > R(0) ? R(2) * xCt * a / (den > R(0) ? den : R(1)) : R(0);
      const R xn = xe0 + y;
      const bool conv = fabs(xn - xe) <= tol * xn;
      xe = xn;
      if (conv) break;
    }
    comp = a > R(0) ? y * (B + cc * (xe0 + y)) / (a * xCt) : R(1);
  }
  // y <= x_C,tot and frac <= 1 hold exactly; in float the quotient can land one ulp above, which
  // would leave x_C and x_CO at -ulp
  y = y < xCt ? y : xCt;
  e.xCp = y;
  e.xe = xe;
  if (std::is_same<R, double>::value) {
    // FP64: 1 - max(x_C+ / x_C,tot, x_H+) as a true quotient and difference (Eq. e:CO as written)
    // (1 - frac) cancels as the carbon ionises fully: the correctly rounded quotient
    const R fr = rmax(y / xCt, xHp);
    const R frac = fr < R(1) ? fr : R(1);
    // (ncrit / n)^2 overflows to inf where the CO fit's critical density is huge (no cosmic
    // rays): the plain division then gives 0
    e.xCO = xCt * R(2) * xH2 * (R(1) - frac) / (R(1) + r.qn2);
    e.xC = xCt - y - e.xCO;
  } else {
    // float: 1 - max(y / x_C,tot, x_H+) = min(comp, 1 - x_H+), 1 - x_H+ from the double x_H+; the
    // neutral carbon x_C + x_CO = x_C,tot comp, so x_C needs no subtraction of x_C+ either
    comp = comp < R(0) ? R(0) : (comp > R(1) ? R(1) : comp);
    const R omh = R(1.0 - xHp_d);
    const R om = comp < omh ? comp : omh;
    e.xCO = xCt * om * (R(2) * xH2 / (R(1) + r.qn2));
    e.xC = rmax(xCt * comp - e.xCO, R(0));
  }
  e.xO = R((double)xOt * (1.0 - xHp_d)) - e.xCO;  // x_O,tot - x_O+ formed in double (x_H+ -> 1)
  return e;
}

template <class R>
__device__ __forceinline__ EqS<R> eq_species(double T, R n, double xH2_d, double xHp_d, const Rad<R> &r,
                                             const CoefT<R> &c, const ParT<R> &p, const R *tab, R tol, int maxit) {
  return eq_species<R>(make_tq<R>(T), n, xH2_d, xHp_d, r, c, p, tab, tol, maxit);
}

// ---------------------------------------------------------------- dust temperature
// Eq. eq:dust_en with sigma_IR(T_d) = 2e-25 Z'_d (T_d/10)^2 and Eq. eq:gas-dust, divided by
// Z'_d:  A T_d^2 (T_d^4 - T_bb^4) + B T_d - (G + B T) = 0, increasing in T_d above T_bb.
// Newton from `guess`, kept inside the bracket [min(T_bb, T), 1e4] and bisecting when a
// Newton step leaves it.  A step is the last one when the error it leaves, |g''| step^2 /
// (2 |g'|), is below 1e-16 T_d.  slope returns dT_d/dT at the root, -(dg/dT) / g' with
// dg/dT = B (T_d / (2 T) - 3/2) (B goes as T^1/2), through the hardware reciprocal: it only
// places the next solve's starting point.
template <class R>
__device__ __forceinline__ R dust_heating_per_Zd(const Rad<R> &r, const CoefT<R> &c, const ParT<R> &p) {
  const R fourpi = R(12.566370614359172954);
  const R uv = fourpi * (c.sig_d_abs[2] * c.J_PE * r.chiPE + c.sig_d_abs[1] * c.J_LW * r.chiLW) +
               c.sig_d_abs[0] * r.phi * (c.hnu_LyC_eV * R(EV));
  const R tau = c.sig_d_Neff * p.Zd * r.Neff;
  const R opt = fourpi * (c.sig_d_abs[2] * c.J_PE + c.sig_d_abs[1] * c.J_LW) * p.chi0 *
                Mx<R>::ex(-(double)tau / (double)p.tau_ratio);
  return uv + opt;
}

// The terms of one cell that depend only on its density and radiation, so are the same in
// every evaluation of the step: the dust heating G, the CR heating per H2 ionisation (piecewise
// linear in log10 n) and the CO critical density n_CO,crit = (4e3 Z'_d xi16^-2)^(chi^1/3)
// (50 xi16 / Z'_d^1.4) of Eq. e:CO_fit with chi_CO = chi_LW.
template <class R>
__device__ __forceinline__ void fixed_terms(Rad<R> &r, double n_d, const CoefT<R> &c, const ParT<R> &p) {
  const CoefT<double> &cd = coef64();
  r.G = dust_heating_per_Zd(r, c, p);
  r.G0f = g0_field(r.chiPE, r.chiLW, c);
  const double *qq = cd.q_cr_H2;  // values qq[0..3] at log10 n = qq[4..7], linear between, flat outside
  const double ln = Mx<R>::ln(n_d) * INV_LN10D;
  double val;
  if (ln <= qq[4]) val = qq[0];
  else if (ln >= qq[7]) val = qq[3];
  else if (ln < qq[5]) val = (qq[1] - qq[0]) / (qq[5] - qq[4]) * (ln - qq[4]) + qq[0];
  else if (ln < qq[6]) val = (qq[2] - qq[1]) / (qq[6] - qq[5]) * (ln - qq[5]) + qq[1];
  else val = (qq[3] - qq[2]) / (qq[7] - qq[6]) * (ln - qq[6]) + qq[2];
  r.qH2 = R(val) * R(EV);
  const R xi16 = rmax(r.xi / R(1e-16), R(1e-10));
  const double lxi = Mx<R>::ln((double)xi16);
  r.ncrit = Mx<R>::ex((double)Mx<R>::cb(r.chiLW) * (cd.ln_co0 + (double)p.lnZd - 2.0 * lxi)) *
            (c.co_fit[1] * xi16 / Mx<R>::ex(cd.co_fit[2] * (double)p.lnZd));
  const R qn = r.ncrit / R(n_d);
  r.qn2 = qn * qn;
}

template <class R> struct RootTol;
template <> struct RootTol<double> { static constexpr double v = 1e-14; static constexpr int it = 80; };
template <> struct RootTol<float> { static constexpr float v = 2e-7f; static constexpr int it = 40; };

template <class R>
__device__ R dust_T(R T, R sqrtT, R n, R G, R guess, R Tbb, const CoefT<R> &c, bool &bad, R &slope) {
  const R A = c.dust_A;  // sigma_IR(10 K)/100 c a_rad
  const R B = n * c.alpha_gd * sqrtT;
  const R Tbb2 = Tbb * Tbb, Tbb4 = Tbb2 * Tbb2;
  const R rhs = G + B * T;
  R lo = rmin(Tbb, T), hi = R(1e4);
  const R h2 = hi * hi;
  slope = R(0);
  if (A * h2 * (h2 * h2 - Tbb4) + B * hi - rhs < R(0)) { bad = true; return hi; }
  bad = false;
  R x = guess;
  if (!(x > lo && x < hi)) {
    // cold start from the smaller of two one-term estimates: radiation alone, (rhs / A)^(1/6),
    // and gas-dust coupling alone, rhs / B.  The second bounds the root from above (g >= 0
    // there once it exceeds T_bb); where coupling dominates (dense gas) the first lies far
    // above the root, and Newton on the degree-6 polynomial would walk down from it by only
    // about a sixth per iteration.
    x = Mx<R>::ex(Mx<R>::ln((double)(rhs / A)) / 6.0);
    if (B > R(0)) x = rmin(x, rhs / B);
    if (!(x > lo && x < hi)) x = R(0.5) * (lo + hi);
  }
  R dg = R(1);
  for (int it = 0; it < RootTol<R>::it; ++it) {
    const R x2 = x * x;
    const R x4 = x2 * x2;
    const R g = A * x2 * (x4 - Tbb4) + B * x - rhs;
    if (g >= R(0)) hi = x; else lo = x;
    dg = A * (R(6) * x4 * x - R(2) * Tbb4 * x) + B;
    // (dg > 0 above 0.76 T_bb; below it a step that leaves the bracket is replaced by bisection,
    // whatever its value)
    const R step = dvp<R>(g, dg);
    R xn = x - step;
    // converged: tested before the bracket safeguard, which would otherwise take a root hit
    // exactly (g = 0 makes x the new upper end, so the step lands on it) for a Newton step
    // leaving the bracket and fall back to bisection
    const R g2 = A * (R(30) * x4 - R(2) * Tbb4);
    if (fabs(step) <= RootTol<R>::v * x || fabs(g2) * step * step <= R(2e-16) * x * fabs(dg)) {
      x = xn;
      break;
    }
    if (!(xn > lo && xn < hi)) xn = R(0.5) * (lo + hi);
    const R dx = fabs(xn - x);
    x = xn;
    if (dx <= RootTol<R>::v * x || hi - lo <= RootTol<R>::v * x) break;
  }
  slope = B * (R(1.5) - R(0.5) * x * __builtin_amdgcn_rcp(T)) * __builtin_amdgcn_rcp(dg);
  return x;
}

// One Newton step in double on the dust-temperature balance above, from x (a root found in float).
__device__ __forceinline__ double dust_polish(double T, double sqrtT, double n, double G, double Tbb,
                                              const CoefT<double> &c, double x) {
  const double A = c.dust_A, B = n * c.alpha_gd * sqrtT;
  const double Tbb2 = Tbb * Tbb, Tbb4 = Tbb2 * Tbb2;
  const double x2 = x * x, x4 = x2 * x2;
  const double g = A * x2 * (x4 - Tbb4) + B * x - (G + B * T);
  const double dg = A * (6.0 * x4 * x - 2.0 * Tbb4 * x) + B;
  return dg > 0.0 ? x - fdivp(g, dg) : x;
}

// ---------------------------------------------------------------- fine structure (Sec. 4.6.2)
// 3-level atom (levels 0, 1, 2); H-impact de-excitation k10 follows the printed critical
// densities as a power law in T (slope precomputed on the host), other partners and
// transitions are stand-in ratios.  Populations by Cramer's rule with p0 = 1, normalised.
// rat: g1/g0, g2/g0, g2/g1 and A10 / n_crit,H, formed on the host.
template <class R>
__device__ __forceinline__ R three_level_cool(const Tq &q, R n, R inv_n, R xH, R xH2, R xe, const double *lv,
                                              const double *rat, const double *co, const double *nc,
                                              double slope) {
  const R A10 = R(lv[5]), A20 = R(lv[6]), A21 = R(lv[7]);
  const double E1 = lv[3], E2 = lv[4];
  const R kH = R(rat[3]) * Mx<R>::ex(slope * (q.lnT - LN10D));
  const R ke = R(co[3]) * Mx<R>::ex(co[4] * q.lnT4);
  const R part = xH * kH + xH2 * R(co[2]) * kH + xe * ke;
  const R C10 = n * part, C20 = n * R(co[0]) * part, C21 = n * R(co[1]) * part;
  const double b1 = (double)Mx<R>::ex(-E1 * q.invT), b2 = (double)Mx<R>::ex(-E2 * q.invT);
  const R R01 = C10 * R(rat[0]) * R(b1);
  const R R02 = C20 * R(rat[1]) * R(b2);
  // in double the 1-2 Boltzmann factor is the quotient of the other two, a division in place of an
  // exp
  // (below ~0.3 K b1 leaves the normal range for O I: then the factor is formed on its own)
  const R b12 = (std::is_same<R, double>::value && b1 > 1e-300) ? R(fdivp(b2, b1)) : Mx<R>::ex(-(E2 - E1) * q.invT);
  const R R12 = C21 * R(rat[2]) * b12;
  const R R10 = C10 + A10, R20 = C20 + A20, R21 = C21 + A21;
  const R det = R10 * R20 + R10 * R21 + R12 * R20;
  const R idet = dvp<R>(R(1), det);
  R p1 = (R01 * (R20 + R21) + R21 * R02) * idet;
  R p2 = (R02 * (R10 + R12) + R12 * R01) * idet;
  const R isum = dvp<R>(R(1), R(1) + p1 + p2);
  p1 *= isum;
  p2 *= isum;
  return (p1 * A10 * R(E1) + p2 * (A20 * R(E2) + A21 * R(E2 - E1))) * R(K_B) * inv_n;
}

// ---------------------------------------------------------------- diagnostics layout
enum Diag {
  DG_XCP, DG_XCO, DG_XE, DG_TD, DG_KGR, DG_ZCRH2, DG_ZPD, DG_ZPIH2, DG_ZCD, DG_ZPIH, DG_ZCRH, DG_ZCI, DG_AB,
  DG_AGRH, DG_PSI, DG_GPE, DG_GCR, DG_GPI, DG_GH2, DG_GAMMA, DG_LLYA, DG_LCI, DG_LROVIB, DG_LCD, DG_LFF, DG_LRR,
  DG_LCP, DG_LC, DG_LO, DG_LCO, DG_LGRREC, DG_LNEB, DG_LGD, DG_LCIE, DG_S, DG_LAMBDA, DG_H, DG_CH2, DG_CHP,
  NDIAG
};

// ---------------------------------------------------------------- full evaluation
// Rates (Sec. 3), heating (Secs. 4.1-4.5), cooling (Sec. 4.6) at temperature T with the
// abundances (xH2, xHp) and closure e.  CHEM_ONLY skips heating/cooling; DIAG writes
// every term into diag[NDIAG].
// The logs in the cooling terms that do not depend on T: log10 of the CO column n x_CO dr/dv and
// ln(n_e / 100), the same in every evaluation of a substep.
struct PreLogs {
  double lNt, lne2;
};

template <class R>
__device__ __forceinline__ PreLogs pre_logs(R n, const EqS<R> &e, const ParT<R> &p) {
  PreLogs g;
  const R Nt = n * e.xCO * R(PC_CM) * p.idvdr;
  g.lNt = Nt > R(0) ? Mx<R>::ln((double)Nt) * INV_LN10D : -300.0;
  const R ne2 = n * e.xe * R(0.01);
  g.lne2 = ne2 > R(0) ? Mx<R>::ln((double)ne2) : 0.0;
  return g;
}

template <class R, bool CHEM_ONLY, bool DIAG>
__device__ Eval<R> evaluate(const Tq &q, double n_d, double xH2_d, double xHp_d, const EqS<R> &e, const Rad<R> &r,
                            const CoefT<R> &c, const ParT<R> &p, const R *tab, double td_guess, R *diag,
                            bool chem = true, const PreLogs *pre = nullptr) {
  const CoefT<double> &cd = coef64();
  Eval<R> v;
  const double T = q.T;
  const R Tr = R(T);
  const R sqrtT = std::is_same<R, double>::value ? R(q.sqrtT) : Mx<R>::sq(Tr);
  const R n = R(n_d);
  const R Zd = p.Zd, Zg = p.Zg;
  const R xe = e.xe;
  const R xH2 = R(xH2_d), xHp = R(xHp_d);
  // x_H = 1 - 2 x_H2 - x_H+ cancels when hydrogen is nearly all molecular or ionised: formed in double
  const double xHd = 1.0 - 2.0 * xH2_d - xHp_d;
  const R xH = R(xHd > 0.0 ? xHd : 0.0);
  const R psi = psi_charge(sqrtT, n, xe, r.G0f, c);
  const double lnpsi = Mx<R>::ln((double)psi);
  // chemistry, Eqs. e:HH and e:HII
  const R kgr = k_gr(q, sqrtT, c, p);
  const R zcrH2 = c.cr_coef[0] * r.xi * (c.cr_coef[1] * xH2 + c.cr_coef[2] * xH);
  const R zcrH = R(0.5) * zcrH2;
  const R zpd = c.zeta_pd * r.chiH2;
  const R zpiH2 = c.sig_pi_H2 * r.phi;
  const R zpiH = c.sig_pi_H * r.phi;
  const R kcdH = c.k_cd_H[0] * sqrtT * Mx<R>::ex(-(1.0 + cd.k_cd_H[1] * q.invT));
  // power laws and the Boltzmann factor in one exponent
  const R kcdH2 = c.k_cd_H2[0] * Mx<R>::ex(cd.k_cd_H2[1] * q.lnT - cd.k_cd_H2[3] * Mx<R>::ln(1.0 + cd.k_cd_H2[2] * T) -
                                           cd.k_cd_H2[4] * q.invT);
  const R zcd = n * (xH * kcdH + xH2 * kcdH2);
  const R kci = dvp<R>(c.k_ci_H[0] * sqrtT * Mx<R>::ex(-cd.k_ci_H[1] * q.invT),
                       R(1) + (std::is_same<R, double>::value ? sqrtT * R(cd.rsqrt_kci_T) : Mx<R>::sq(R(T * cd.inv_kci_T))));
  const R zci = kci * n * xe;
  const R aB = c.alpha_B[0] * Mx<R>::ex((cd.alpha_B[1] + cd.alpha_B[2] * q.lnT4) * q.lnT4);
  // H+ grain recombination enters only the rates; skipped (chem = false) where a caller takes
  // nothing but the heating and cooling from this evaluation
  const R agrH = chem ? alpha_gr<R>(q, lnpsi, cd.agr_Hp, Zd) : R(0);
  v.F = kgr * n;
  v.D = c.cr_destr * zcrH2 + zpd + zpiH2 + zcd;
  v.I = zpiH + zcrH + zci;
  v.Rr = aB * n * xe + agrH * n;
  // net rates in double from the rate coefficients: near balance the two terms cancel, and
  // the substep size follows 1 / |C|
  v.CH2 = (double)v.F * (xHd > 0.0 ? xHd : 0.0) - (double)v.D * xH2_d;
  v.CHp = (double)v.I * (xHd > 0.0 ? xHd : 0.0) - (double)v.Rr * xHp_d;
  v.Td = 0.0;
  v.Tds = 0.0;
  v.td_bad = false;
  v.Gamma = v.Lambda = v.H = 0.0;
  if (DIAG) {
    diag[DG_XCP] = e.xCp; diag[DG_XCO] = e.xCO; diag[DG_XE] = e.xe; diag[DG_KGR] = kgr; diag[DG_ZCRH2] = zcrH2;
    diag[DG_ZPD] = zpd; diag[DG_ZPIH2] = zpiH2; diag[DG_ZCD] = zcd; diag[DG_ZPIH] = zpiH; diag[DG_ZCRH] = zcrH;
    diag[DG_ZCI] = zci; diag[DG_AB] = aB; diag[DG_AGRH] = agrH; diag[DG_PSI] = psi; diag[DG_CH2] = R(v.CH2);
    diag[DG_CHP] = R(v.CHp);
  }
  if (CHEM_ONLY) return v;
  const R ev = R(EV);
  const R inv_n = dvp<R>(R(1), n);
  // heating, Secs. 4.1-4.5
  const R G0 = r.G0f;
  const R eps = dvp<R>(c.pe_C[0] + c.pe_C[1] * Mx<R>::ex(cd.pe_C[4] * q.lnT),
                       R(1) + c.pe_C[2] * Mx<R>::ex(cd.pe_C[5] * lnpsi) * (R(1) + c.pe_C[3] * Mx<R>::ex(cd.pe_C[6] * lnpsi)));
  const R g_pe = c.pe_pref * G0 * eps * Zd;
  const R qH = (c.q_cr_H[0] + c.q_cr_H[1] * Mx<R>::sq(dvp<R>(xe, xe + c.q_cr_H[2]))) * ev;
  const R qH2 = r.qH2;
  const R g_cr = r.xi * (xH * qH + R(2) * xH2 * qH2);
  const R g_pi = xH * (c.q_pi_H_eV * ev) * zpiH + xH2 * (c.q_pi_H2_eV * ev) * zpiH2;
  const R kHH = c.k_H2_H[0] * sqrtT * Mx<R>::ex(-cd.k_H2_H[1] * q.invT);
  const R kHH2 = c.k_H2_H2[0] * sqrtT * Mx<R>::ex(-fdivp(cd.k_H2_H2[1], T + cd.k_H2_H2[2]));
  const R dcol = xH * kHH + xH2 * kHH2;
  const R eff = dvp<R>(n * dcol, n * dcol + c.A_eff + zpd);
  const R g_h2 = kgr * n * xH * (c.h2form_eV[0] * ev + c.h2form_eV[1] * ev * eff) +
                 zpd * xH2 * c.f_pump * (c.pump_eV * ev) * eff + zpd * xH2 * (c.pd_eV * ev);
  v.Gamma = (double)g_pe + (double)g_cr + (double)g_pi + (double)g_h2;
  // cooling, Sec. 4.6
  const R sqrtT4 = std::is_same<R, double>::value ? sqrtT * R(0.01) : Mx<R>::sq(R(T * 1e-4));  // (T / 1e4)^1/2
  const R k12 = dvp<R>(c.lya[0] * Mx<R>::ex(cd.lya[1] * q.lnT4 - cd.lya[4] * 1e4 * q.invT),
                       R(1) + Mx<R>::ex(cd.lya[3] * (q.lnT4 - cd.ln_lya_T)));
  const R l_lya = xH * xe * R(K_B) * c.lya_E21 * k12;
  const R l_ci = (c.ci_eV * ev) * xH * xe * kci;
  const R l_cd = (c.cd_eV * ev) * xH2 * (xH * kcdH + xH2 * kcdH2);
  R l_rv = R(0);
  if (p.h2_rovib) {
    const double *a = cd.rovib_lte;
    const double lnT3 = q.lnT - LN1E3;
    const double iT3 = 1e3 * q.invT;
    const double q3 = a[4] * iT3;
    const R Lrot = dvp<R>(R(a[0]) * Mx<R>::ex(a[1] * lnT3), R(1) + R(a[2]) * Mx<R>::ex(a[3] * lnT3)) *
                       Mx<R>::ex(-(q3 * q3 * q3)) +
                   R(a[5]) * Mx<R>::ex(-a[6] * iT3);
    const R Lvib = R(a[7]) * Mx<R>::ex(-a[8] * iT3) + R(a[9]) * Mx<R>::ex(-a[10] * iT3);
    const R Llte = Lrot + Lvib;
    // the quartic in log10 T cancels terms of ~1e2 down to ~-24: kept in double
    const double *b = cd.rovib_low;
    double lg = q.lnT * INV_LN10D;
    lg = lg < b[5] ? b[5] : (lg > b[6] ? b[6] : lg);
    const R L0 = Mx<R>::ex(LN10D * (b[0] + lg * (b[1] + lg * (b[2] + lg * (b[3] + lg * b[4])))));
    const R np_ = n * (xH + xH2);
    const R nL0 = np_ * L0;
    // = Llte n L0 / (n L0 + Llte), 0 when either rate is 0: in double as one quotient (both can
    // be tiny: the plain division), in float without forming the product, which can underflow
    const R L = !(nL0 > R(0) && Llte > R(0)) ? R(0)
                : std::is_same<R, double>::value ? nL0 * Llte / (nL0 + Llte) : nL0 / (R(1) + nL0 / Llte);
    l_rv = xH2 * L * inv_n;
  }
  // the cooling terms are summed as they are formed, each partial sum pinned by an empty asm, so
  // that a term's registers are free once it is added (holding the thirteen terms to one final
  // sum made this the kernel's register peak)
  double hyd = (double)l_lya + (double)l_ci + (double)l_rv + (double)l_cd;
  asm volatile("" : "+v"(hyd));
  const R l_ff = c.ff[0] * c.ff[1] * sqrtT * xe * xHp;
  const R l_rr = aB * R(K_B) * Tr * R(cd.rr_energy[0] + cd.rr_energy[1] * q.lnT4) * xe * xHp;
  hyd = hyd + (double)l_ff + (double)l_rr;
  asm volatile("" : "+v"(hyd));
  // C+ 2-level
  R l_cp;
  {
    const R E10 = c.cp_levels[2], A10 = c.cp_levels[3];
    const double lnT2 = q.lnT - LN100;
    const R k10H = c.cp_rat[0] * Mx<R>::ex((cd.cp_ncrit_H[1] + cd.cp_ncrit_H[2] * lnT2) * lnT2);
    const R k10e = dvp<R>(A10, c.cp_ncrit_e * sqrtT4);
    const R C10 = n * (xH * k10H + xH2 * c.cp_h2_over_h * k10H + xe * k10e);
    const R C01 = C10 * c.cp_rat[1] * Mx<R>::ex(-cd.cp_levels[2] * q.invT);
    const R f1 = dvp<R>(C01, C01 + C10 + A10);
    l_cp = e.xCp * f1 * A10 * R(K_B) * E10 * inv_n;
  }
  double mid = (double)l_cp;
  asm volatile("" : "+v"(mid));
  const R l_c = e.xC * three_level_cool<R>(q, n, inv_n, xH, xH2, xe, cd.c_levels, cd.c_rat, cd.c_coll, cd.c_ncrit_H,
                                             cd.fs_slope_C);
  mid = mid + (double)l_c;
  asm volatile("" : "+v"(mid));
  const R l_o = e.xO * three_level_cool<R>(q, n, inv_n, xH, xH2, xe, cd.o_levels, cd.o_rat, cd.o_coll, cd.o_ncrit_H,
                                             cd.fs_slope_O);
  mid = mid + (double)l_o;
  asm volatile("" : "+v"(mid));
  R l_co;
  {
    const double lT = q.lnT * INV_LN10D;
    const double lN = (pre ? *pre : pre_logs<R>(n, e, p)).lNt;
    // log10 columns are stored as log10(value) + TAB_LOG_OFFSET (see coef.h)
    const R L0 = Mx<R>::ex(LN10D * (co_lookup(tab, lT, lN, 0) - TAB_LOG_OFFSET));
    const R nh = Mx<R>::ex(LN10D * co_lookup(tab, lT, lN, 1));
    // L0 / (1 + n / n_half) as one division; n + n_half >= n
    l_co = dvp<R>(e.xCO * L0 * nh, nh + n);
  }
  mid = mid + (double)l_co;
  asm volatile("" : "+v"(mid));
  const R l_gr =
      c.grrec[0] * Mx<R>::ex(cd.grrec[1] * q.lnT + cd.grrec[2] * (double)Mx<R>::ex(-cd.grrec[3] * q.lnT) * lnpsi) *
      xe * Zd;
  R l_neb;
  {
    // the degree-6 fit cancels terms several times its value: Horner in double
    double f = 0.0;
    for (int k = 6; k >= 0; --k) f = f * q.lnT4 + cd.neb_a[k];
    // exp(-E/T4) f_neb as one exponent: each factor alone can leave float range
    const R ef = Mx<R>::ex(LN10D * f - cd.neb[1] * 1e4 * q.invT);
    const R ne2 = n * xe * R(0.01);
    const double lne2 = (pre ? *pre : pre_logs<R>(n, e, p)).lne2;
    const double expo = cd.neb[3] - cd.neb[4] * q.lnT4;
    const R dens = ne2 > R(0) ? Mx<R>::ex(expo * lne2)
                              : (expo > 0.0 ? R(0) : (expo < 0.0 ? R(INFINITY) : R(1)));
    l_neb = Zg * xe * xHp * c.neb[0] * ef / (sqrtT4 * (R(1) + c.neb[2] * dens));
  }
  mid = mid + (double)l_gr + (double)l_neb;
  asm volatile("" : "+v"(mid));
  // dust temperature to double accuracy on both paths: where gas and dust are coupled T_d -> T,
  // and the gas-dust term goes as T - T_d.  The float path solves in float and takes one Newton
  // step in double from the float root (relative error ~1e-7 before it, ~1e-14 after)
  bool bad;
  const double sqrtTd = q.sqrtT;
  double Td;
  if constexpr (std::is_same<R, float>::value) {
    float slope;
    const float Tdf = dust_T<float>((float)T, (float)sqrtTd, (float)n_d, r.G, (float)td_guess, p.T_bb, c, bad, slope);
    Td = bad ? (double)Tdf : dust_polish(T, sqrtTd, n_d, (double)r.G, (double)p.T_bb, cd, (double)Tdf);
    v.Tds = slope;
  } else {
    Td = dust_T<double>(T, sqrtTd, n_d, (double)r.G, td_guess, (double)p.T_bb, cd, bad, v.Tds);
  }
  v.Td = Td;
  v.td_bad = bad;
  const R l_gd = R(cd.alpha_gd * sqrtTd * (T - Td) * (double)Zd);
  const R S = dvp<R>(R(1), R(1) + Mx<R>::ex(-cd.sigmoid[0] * (T - 0.5 * (cd.sigmoid[1] + cd.sigmoid[2])) *
                                              cd.sigmoid_iw));
  const double lgT = q.lnT * INV_LN10D;
  const R l_cie = Mx<R>::ex(LN10D * (cie_lookup(tab, lgT, 0) - TAB_LOG_OFFSET)) +
                  Zg * Mx<R>::ex(LN10D * (cie_lookup(tab, lgT, 1) - TAB_LOG_OFFSET));
  mid = mid + (double)l_gd;
  v.Lambda = hyd + (1.0 - (double)S) * mid + (double)S * (double)l_cie;
  v.H = n_d * v.Gamma - n_d * n_d * v.Lambda;
  if (DIAG) {
    diag[DG_TD] = Td; diag[DG_GPE] = g_pe; diag[DG_GCR] = g_cr; diag[DG_GPI] = g_pi; diag[DG_GH2] = g_h2;
    diag[DG_GAMMA] = R(v.Gamma); diag[DG_LLYA] = l_lya; diag[DG_LCI] = l_ci; diag[DG_LROVIB] = l_rv;
    diag[DG_LCD] = l_cd; diag[DG_LFF] = l_ff; diag[DG_LRR] = l_rr; diag[DG_LCP] = l_cp; diag[DG_LC] = l_c;
    diag[DG_LO] = l_o; diag[DG_LCO] = l_co; diag[DG_LGRREC] = l_gr; diag[DG_LNEB] = l_neb; diag[DG_LGD] = l_gd;
    diag[DG_LCIE] = l_cie; diag[DG_S] = S; diag[DG_LAMBDA] = R(v.Lambda); diag[DG_H] = R(v.H);
  }
  return v;
}

template <class R, bool CHEM_ONLY, bool DIAG>
__device__ __forceinline__ Eval<R> evaluate(double T, double n_d, double xH2_d, double xHp_d, const EqS<R> &e,
                                            const Rad<R> &r, const CoefT<R> &c, const ParT<R> &p, const R *tab,
                                            double td_guess, R *diag, bool chem = true) {
  return evaluate<R, CHEM_ONLY, DIAG>(make_tq<R>(T), n_d, xH2_d, xHp_d, e, r, c, p, tab, td_guess, diag, chem);
}

}  // namespace ism
