// Device microphysics of the ISM source step (Secs. 3-4 of arXiv:2210.08024),
// templated on the evaluation type R (double: plain path, float: mixed path).
// One lane evaluates one cell; nothing here touches memory except the LDS tables.
#pragma once
#include <hip/hip_runtime.h>

#include "coef.h"

namespace ism {

// ---------------------------------------------------------------- math wrappers
// double: ROCm device libm; float: hardware transcendentals (v_exp_f32 / v_log_f32).
__device__ __forceinline__ double m_exp(double x) { return ::exp(x); }
__device__ __forceinline__ float m_exp(float x) { return __expf(x); }
__device__ __forceinline__ double m_log(double x) { return ::log(x); }
__device__ __forceinline__ float m_log(float x) { return __logf(x); }
__device__ __forceinline__ double m_log10(double x) { return ::log10(x); }
__device__ __forceinline__ float m_log10(float x) { return __log10f(x); }
__device__ __forceinline__ double m_pow(double x, double y) { return ::pow(x, y); }
__device__ __forceinline__ float m_pow(float x, float y) { return __powf(x, y); }
__device__ __forceinline__ double m_sqrt(double x) { return ::sqrt(x); }
__device__ __forceinline__ float m_sqrt(float x) { return __fsqrt_rn(x); }
__device__ __forceinline__ double m_cbrt(double x) { return ::cbrt(x); }
__device__ __forceinline__ float m_cbrt(float x) { return ::cbrtf(x); }
__device__ __forceinline__ double m_expm1(double x) { return ::expm1(x); }
__device__ __forceinline__ float m_expm1(float x) { return ::expm1f(x); }
template <class R> __device__ __forceinline__ R m_pow10(R x) { return m_exp(R(LN10) * x); }
template <class R> __device__ __forceinline__ R rmax(R a, R b) { return a > b ? a : b; }
template <class R> __device__ __forceinline__ R rmin(R a, R b) { return a < b ? a : b; }

template <class R> struct Tiny;
template <> struct Tiny<double> { static constexpr double v = 1e-300; };
template <> struct Tiny<float> { static constexpr float v = 1e-37f; };

// ---------------------------------------------------------------- tables
// Clamp x to the grid [x0, x0 + (n-1) dx]; lower node index and fraction.
template <class R>
__device__ __forceinline__ void axis_pos(R x, R x0, R dx, int n, int &i, R &f) {
  R hi = x0 + R(n - 1) * dx;
  R xc = x < x0 ? x0 : (x > hi ? hi : x);
  R u = (xc - x0) / dx;
  int k = (int)floor(u);
  k = k > 0 ? k : 0;  // also maps a NaN argument to node 0
  i = k < n - 2 ? k : n - 2;
  f = u - R(i);
}

template <class R>
__device__ __forceinline__ R cie_lookup(const R *tab, const CoefT<R> &c, R lgT, int col) {
  int i;
  R f;
  axis_pos(lgT, c.cie_x0, c.cie_dx, CIE_N, i, f);
  const R *v = tab + TAB_CIE;
  return v[i * CIE_NC + col] * (R(1) - f) + v[(i + 1) * CIE_NC + col] * f;
}

template <class R>
__device__ __forceinline__ R co_lookup(const R *tab, const CoefT<R> &c, R lT, R lN, int col) {
  int i, j;
  R f, g;
  axis_pos(lT, c.co_x0, c.co_dx, CO_NX, i, f);
  axis_pos(lN, c.co_y0, c.co_dy, CO_NY, j, g);
  const R *v = tab + TAB_CO;
  R v00 = v[(i * CO_NY + j) * CO_NC + col], v01 = v[(i * CO_NY + j + 1) * CO_NC + col];
  R v10 = v[((i + 1) * CO_NY + j) * CO_NC + col], v11 = v[((i + 1) * CO_NY + j + 1) * CO_NC + col];
  return (v00 * (R(1) - g) + v01 * g) * (R(1) - f) + (v10 * (R(1) - g) + v11 * g) * f;
}

// ---------------------------------------------------------------- per-cell inputs
template <class R>
struct Rad {
  R chiPE, chiLW, chiH2, chiC, phi, xi, Neff;
};

template <class R>
struct EqS {
  R xCp, xCO, xC, xOp, xO, xe;
};

// Everything the update needs from one evaluation; Gamma/Lambda/H in double.
template <class R>
struct Eval {
  R F, D, I, Rr, CH2, CHp, Td;
  double Gamma, Lambda, H;
  bool td_bad;
};

// ---------------------------------------------------------------- rate coefficients
template <class R>
__device__ __forceinline__ R k_gr(R T, const CoefT<R> &c, const ParT<R> &p) {
  if (p.kgr_const) return c.kgr0 * p.Zd;
  R T2 = T / R(100);
  R s = m_sqrt(T2);
  return c.kgr0 * p.Zd * c.kgr_shape[0] * s /
         (R(1) + c.kgr_shape[1] * s + c.kgr_shape[2] * T2 + c.kgr_shape[3] * T2 * T2);
}

template <class R>
__device__ __forceinline__ R alpha_B(R T, const CoefT<R> &c) {
  R T4 = T / R(1e4);
  return c.alpha_B[0] * m_pow(T4, c.alpha_B[1] + c.alpha_B[2] * m_log(T4));
}

template <class R>
__device__ __forceinline__ R k_ci_H(R T, const CoefT<R> &c) {
  return c.k_ci_H[0] * m_sqrt(T) * m_exp(-c.k_ci_H[1] / T) / (R(1) + m_sqrt(T / c.k_ci_H[2]));
}

template <class R>
__device__ __forceinline__ R k_cd_H(R T, const CoefT<R> &c) {
  return c.k_cd_H[0] * m_sqrt(T) * m_exp(-(R(1) + c.k_cd_H[1] / T));
}

template <class R>
__device__ __forceinline__ R k_cd_H2(R T, const CoefT<R> &c) {
  return c.k_cd_H2[0] * m_pow(T, c.k_cd_H2[1]) * m_pow(R(1) + c.k_cd_H2[2] * T, -c.k_cd_H2[3]) *
         m_exp(-c.k_cd_H2[4] / T);
}

template <class R>
__device__ __forceinline__ R alpha_gr(R T, R psi, const R *k, R Zd) {
  return R(1e-14) * k[0] * Zd /
         (R(1) + k[1] * m_pow(psi, k[2]) * (R(1) + k[3] * m_pow(T, k[4]) * m_pow(psi, -k[5] - k[6] * m_log(T))));
}

template <class R>
__device__ __forceinline__ R psi_charge(R T, R n, R xe, R chiPE, R chiLW, const CoefT<R> &c) {
  R G0 = c.G0_per_chi * ((c.J_PE * chiPE + c.J_LW * chiLW) / c.J_FUV);
  return G0 * m_sqrt(T) / (n * rmax(xe, R(1e-20))) + c.psi_off;
}

// ---------------------------------------------------------------- C / O / e closure
// Secs. 3.2-3.3: x_O+ = x_O,tot x_H+; C+ from Eq. eq:C+_frac with n_e = n (x_e0 + x_C+)
// (positive root of the quadratic, psi iterated to a fixed point in x_e) below 2e4 K,
// Eq. e:xELhot above; CO from Eqs. e:CO, e:CO_fit with chi_CO = chi_LW.
template <class R>
__device__ EqS<R> eq_species(R T, R n, R xH2, R xHp, const Rad<R> &r, const CoefT<R> &c, const ParT<R> &p,
                             const R *tab, R tol, int maxit) {
  EqS<R> e;
  const R xCt = p.xCt, xOt = p.xOt, Zd = p.Zd;
  e.xOp = xOt * xHp;
  const R a = c.zeta_pi_C * r.chiC + c.zeta_pi_C_cr * R(2) * xH2 * r.xi + c.zeta_cr_C * r.xi;
  const R cc = c.arrdr_Cp[0] * m_pow(T / c.arrdr_Cp[1], c.arrdr_Cp[2]) * n;
  const R kch = c.k_CpH2[0] * m_pow(T, c.k_CpH2[1]) * m_exp(-c.k_CpH2[2] / T) * n * xH2;
  R y, xe;
  if (T >= c.xe_T_switch) {
    R lgT = m_log10(T);
    xe = xHp + cie_lookup(tab, c, lgT, 2) + p.Zg * cie_lookup(tab, c, lgT, 3);
    R psi = psi_charge(T, n, xe, r.chiPE, r.chiLW, c);
    R B = alpha_gr(T, psi, c.agr_Cp, Zd) * n + kch;
    R dh = a + B + cc * xe;
    y = a > R(0) ? xCt * a / (dh > R(0) ? dh : R(1)) : R(0);
  } else {
    const R xmh = R(2) * xH2 * m_sqrt(c.x_MH[0] * r.xi / (c.x_MH[1] * m_pow(T / c.x_MH[2], c.x_MH[3]) * n));
    const R xe0 = xHp + e.xOp + xmh;
    xe = xe0 + xCt;
    y = R(0);
    for (int it = 0; it < maxit; ++it) {
      R psi = psi_charge(T, n, xe, r.chiPE, r.chiLW, c);
      R B = alpha_gr(T, psi, c.agr_Cp, Zd) * n + kch;
      R pp = a + B + cc * xe0;
      R den = pp + m_sqrt(pp * pp + R(4) * cc * xCt * a);
      y = a > R(0) ? R(2) * xCt * a / (den > R(0) ? den : R(1)) : R(0);
      R xn = xe0 + y;
      bool conv = fabs(xn - xe) <= tol * xn;
      xe = xn;
      if (conv) break;
    }
  }
  e.xCp = y;
  e.xe = xe;
  R xi16 = rmax(r.xi / R(1e-16), R(1e-10));
  R ncrit = m_pow(c.co_fit[0] * Zd / (xi16 * xi16), m_cbrt(r.chiLW)) * (c.co_fit[1] * xi16 / m_pow(Zd, c.co_fit[2]));
  R frac = rmax(y / xCt, xHp);
  R q = ncrit / n;
  e.xCO = xCt * R(2) * xH2 * (R(1) - frac) / (R(1) + q * q);
  e.xC = xCt - y - e.xCO;
  e.xO = xOt - e.xCO - e.xOp;
  return e;
}

// ---------------------------------------------------------------- dust temperature
// Eq. eq:dust_en with sigma_IR(T_d) = 2e-25 Z'_d (T_d/10)^2 and Eq. eq:gas-dust, divided by
// Z'_d:  A T_d^2 (T_d^4 - T_bb^4) + B T_d - (G + B T) = 0, increasing in T_d above T_bb.
// Newton from `guess`, kept inside the bracket [min(T_bb, T), 1e4] and bisecting when a
// Newton step leaves it.
template <class R>
__device__ __forceinline__ R dust_heating_per_Zd(const Rad<R> &r, const CoefT<R> &c, const ParT<R> &p) {
  const R fourpi = R(12.566370614359172954);
  R uv = fourpi * (c.sig_d_abs[2] * c.J_PE * r.chiPE + c.sig_d_abs[1] * c.J_LW * r.chiLW) +
         c.sig_d_abs[0] * r.phi * (c.hnu_LyC_eV * R(EV));
  R tau = c.sig_d_Neff * p.Zd * r.Neff;
  R opt = fourpi * (c.sig_d_abs[2] * c.J_PE + c.sig_d_abs[1] * c.J_LW) * p.chi0 * m_exp(-tau / p.tau_ratio);
  return uv + opt;
}

template <class R> struct RootTol;
template <> struct RootTol<double> { static constexpr double v = 1e-14; static constexpr int it = 80; };
template <> struct RootTol<float> { static constexpr float v = 2e-7f; static constexpr int it = 40; };

template <class R>
__device__ R dust_T(R T, R n, R G, R guess, const CoefT<R> &c, const ParT<R> &p, bool &bad) {
  const R A = c.sigma_IR10 / R(100) * R(C_LIGHT) * c.a_rad;
  const R B = n * c.alpha_gd * m_sqrt(T);
  const R Tbb2 = p.T_bb * p.T_bb, Tbb4 = Tbb2 * Tbb2;
  const R rhs = G + B * T;
  R lo = rmin(p.T_bb, T), hi = R(1e4);
  R h2 = hi * hi;
  if (A * h2 * (h2 * h2 - Tbb4) + B * hi - rhs < R(0)) { bad = true; return hi; }
  bad = false;
  R x = (guess > lo && guess < hi) ? guess : R(0.5) * (lo + hi);
  for (int it = 0; it < RootTol<R>::it; ++it) {
    R x2 = x * x;
    R g = A * x2 * (x2 * x2 - Tbb4) + B * x - rhs;
    if (g >= R(0)) hi = x; else lo = x;
    R dg = A * (R(6) * x2 * x2 * x - R(2) * Tbb4 * x) + B;
    R xn = x - g / dg;
    if (!(xn > lo && xn < hi)) xn = R(0.5) * (lo + hi);
    R dx = fabs(xn - x);
    x = xn;
    if (dx <= RootTol<R>::v * x || hi - lo <= RootTol<R>::v * x) break;
  }
  return x;
}

// ---------------------------------------------------------------- fine structure (Sec. 4.2.2)
template <class R>
__device__ __forceinline__ R three_level_cool(R T, R n, R xH, R xH2, R xe, const R *lv, const R *co, const R *nc,
                                              const CoefT<R> &c) {
  const R g0 = lv[0], g1 = lv[1], g2 = lv[2], E1 = lv[3], E2 = lv[4], A10 = lv[5], A20 = lv[6], A21 = lv[7];
  const R s = m_log(nc[0] / nc[1]) / m_log(R(500));
  R kH = (A10 / nc[0]) * m_pow(T / R(10), s);
  R ke = co[3] * m_pow(T / R(1e4), co[4]);
  R part = xH * kH + xH2 * co[2] * kH + xe * ke;
  R C10 = n * part, C20 = n * co[0] * part, C21 = n * co[1] * part;
  R R01 = C10 * (g1 / g0) * m_exp(-E1 / T);
  R R02 = C20 * (g2 / g0) * m_exp(-E2 / T);
  R R12 = C21 * (g2 / g1) * m_exp(-(E2 - E1) / T);
  R R10 = C10 + A10, R20 = C20 + A20, R21 = C21 + A21;
  R det = R10 * R20 + R10 * R21 + R12 * R20;
  R p1 = (R01 * (R20 + R21) + R21 * R02) / det;
  R p2 = (R02 * (R10 + R12) + R12 * R01) / det;
  R sum = R(1) + p1 + p2;
  p1 /= sum;
  p2 /= sum;
  return (p1 * A10 * E1 + p2 * (A20 * E2 + A21 * (E2 - E1))) * R(K_B) / n;
}

// ---------------------------------------------------------------- diagnostics layout
enum Diag {
  DG_XCP, DG_XCO, DG_XE, DG_TD, DG_KGR, DG_ZCRH2, DG_ZPD, DG_ZPIH2, DG_ZCD, DG_ZPIH, DG_ZCRH, DG_ZCI, DG_AB,
  DG_AGRH, DG_PSI, DG_GPE, DG_GCR, DG_GPI, DG_GH2, DG_GAMMA, DG_LLYA, DG_LCI, DG_LROVIB, DG_LCD, DG_LFF, DG_LRR,
  DG_LCP, DG_LC, DG_LO, DG_LCO, DG_LGRREC, DG_LNEB, DG_LGD, DG_LCIE, DG_S, DG_LAMBDA, DG_H, DG_CH2, DG_CHP,
  NDIAG
};

// ---------------------------------------------------------------- full evaluation
// Rates (Sec. 3), heating (Sec. 4.1), cooling (Sec. 4.2) at temperature T with the
// abundances (xH2, xHp) and closure e.  CHEM_ONLY skips heating/cooling; DIAG writes
// every term into diag[NDIAG].
template <class R, bool CHEM_ONLY, bool DIAG>
__device__ Eval<R> evaluate(R T, double n_d, R xH2, R xHp, const EqS<R> &e, const Rad<R> &r, const CoefT<R> &c,
                            const ParT<R> &p, const R *tab, R td_guess, R *diag) {
  Eval<R> v;
  const R n = R(n_d);
  const R Zd = p.Zd, Zg = p.Zg;
  const R xe = e.xe;
  R xH = R(1) - R(2) * xH2 - xHp;
  xH = xH > R(0) ? xH : R(0);
  const R psi = psi_charge(T, n, xe, r.chiPE, r.chiLW, c);
  // chemistry, Eqs. e:HH and e:HII
  const R kgr = k_gr(T, c, p);
  const R zcrH2 = c.cr_coef[0] * r.xi * (c.cr_coef[1] * xH2 + c.cr_coef[2] * xH);
  const R zcrH = R(0.5) * zcrH2;
  const R zpd = c.zeta_pd * r.chiH2;
  const R zpiH2 = c.sig_pi_H2 * r.phi;
  const R zpiH = c.sig_pi_H * r.phi;
  const R kcdH = k_cd_H(T, c), kcdH2 = k_cd_H2(T, c);
  const R zcd = n * (xH * kcdH + xH2 * kcdH2);
  const R kci = k_ci_H(T, c);
  const R zci = kci * n * xe;
  const R aB = alpha_B(T, c);
  const R agrH = alpha_gr(T, psi, c.agr_Hp, Zd);
  v.F = kgr * n;
  v.D = c.cr_destr * zcrH2 + zpd + zpiH2 + zcd;
  v.I = zpiH + zcrH + zci;
  v.Rr = aB * n * xe + agrH * n;
  v.CH2 = v.F * xH - v.D * xH2;
  v.CHp = v.I * xH - v.Rr * xHp;
  v.Td = R(0);
  v.td_bad = false;
  v.Gamma = v.Lambda = v.H = 0.0;
  if (DIAG) {
    diag[DG_XCP] = e.xCp; diag[DG_XCO] = e.xCO; diag[DG_XE] = e.xe; diag[DG_KGR] = kgr; diag[DG_ZCRH2] = zcrH2;
    diag[DG_ZPD] = zpd; diag[DG_ZPIH2] = zpiH2; diag[DG_ZCD] = zcd; diag[DG_ZPIH] = zpiH; diag[DG_ZCRH] = zcrH;
    diag[DG_ZCI] = zci; diag[DG_AB] = aB; diag[DG_AGRH] = agrH; diag[DG_PSI] = psi; diag[DG_CH2] = v.CH2;
    diag[DG_CHP] = v.CHp;
  }
  if (CHEM_ONLY) return v;
  const R ev = R(EV);
  // heating, Sec. 4.1
  const R G0 = c.G0_per_chi * ((c.J_PE * r.chiPE + c.J_LW * r.chiLW) / c.J_FUV);
  const R eps = (c.pe_C[0] + c.pe_C[1] * m_pow(T, c.pe_C[4])) /
                (R(1) + c.pe_C[2] * m_pow(psi, c.pe_C[5]) * (R(1) + c.pe_C[3] * m_pow(psi, c.pe_C[6])));
  const R g_pe = c.pe_pref * G0 * eps * Zd;
  const R qH = (c.q_cr_H[0] + c.q_cr_H[1] * m_sqrt(xe / (xe + c.q_cr_H[2]))) * ev;
  R qH2;
  {
    const R *q = c.q_cr_H2;  // values q[0..3] at log10 n = q[4..7]
    R ln = m_log10(n);
    if (ln <= q[4]) qH2 = q[0];
    else if (ln >= q[7]) qH2 = q[3];
    else {
      int j = ln < q[5] ? 0 : (ln < q[6] ? 1 : 2);
      qH2 = (q[j + 1] - q[j]) / (q[j + 5] - q[j + 4]) * (ln - q[j + 4]) + q[j];
    }
    qH2 *= ev;
  }
  const R g_cr = r.xi * (xH * qH + R(2) * xH2 * qH2);
  const R g_pi = xH * (c.q_pi_H_eV * ev) * zpiH + xH2 * (c.q_pi_H2_eV * ev) * zpiH2;
  const R kHH = c.k_H2_H[0] * m_sqrt(T) * m_exp(-c.k_H2_H[1] / T);
  const R kHH2 = c.k_H2_H2[0] * m_sqrt(T) * m_exp(-c.k_H2_H2[1] / (T + c.k_H2_H2[2]));
  const R dcol = xH * kHH + xH2 * kHH2;
  const R eff = n * dcol / (n * dcol + c.A_eff + zpd);
  const R g_h2 = kgr * n * xH * (c.h2form_eV[0] * ev + c.h2form_eV[1] * ev * eff) +
                 zpd * xH2 * c.f_pump * (c.pump_eV * ev) * eff + zpd * xH2 * (c.pd_eV * ev);
  v.Gamma = (double)g_pe + (double)g_cr + (double)g_pi + (double)g_h2;
  // cooling, Sec. 4.2
  const R T4 = T / R(1e4);
  const R k12 = c.lya[0] * m_pow(T4, c.lya[1]) / (R(1) + m_pow(T4 / c.lya[2], c.lya[3])) * m_exp(-c.lya[4] / T4);
  const R l_lya = xH * xe * R(K_B) * c.lya_E21 * k12;
  const R l_ci = (c.ci_eV * ev) * xH * xe * kci;
  const R l_cd = (c.cd_eV * ev) * xH2 * (xH * kcdH + xH2 * kcdH2);
  R l_rv = R(0);
  if (p.h2_rovib) {
    const R *a = c.rovib_lte;
    const R T3 = T / R(1e3);
    const R q3 = a[4] / T3;
    const R Lrot = a[0] * m_pow(T3, a[1]) / (R(1) + a[2] * m_pow(T3, a[3])) * m_exp(-(q3 * q3 * q3)) +
                   a[5] * m_exp(-a[6] / T3);
    const R Lvib = a[7] * m_exp(-a[8] / T3) + a[9] * m_exp(-a[10] / T3);
    const R Llte = Lrot + Lvib;
    const R *b = c.rovib_low;
    R lg = m_log10(T);
    lg = lg < b[5] ? b[5] : (lg > b[6] ? b[6] : lg);
    const R L0 = m_pow10(b[0] + lg * (b[1] + lg * (b[2] + lg * (b[3] + lg * b[4]))));
    const R np_ = n * (xH + xH2);
    const R L = Llte * np_ * L0 / (np_ * L0 + Llte);
    l_rv = xH2 * L / n;
  }
  const R l_ff = c.ff[0] * c.ff[1] * m_sqrt(T) * xe * xHp;
  const R l_rr = aB * R(K_B) * T * (c.rr_energy[0] + c.rr_energy[1] * m_log(T4)) * xe * xHp;
  // C+ 2-level
  R l_cp;
  {
    const R g0 = c.cp_levels[0], g1 = c.cp_levels[1], E10 = c.cp_levels[2], A10 = c.cp_levels[3];
    const R T2 = T / R(100);
    const R k10H = (A10 / c.cp_ncrit_H[0]) * m_pow(T2, c.cp_ncrit_H[1] + c.cp_ncrit_H[2] * m_log(T2));
    const R k10e = A10 / (c.cp_ncrit_e * m_sqrt(T4));
    const R C10 = n * (xH * k10H + xH2 * c.cp_h2_over_h * k10H + xe * k10e);
    const R C01 = C10 * (g1 / g0) * m_exp(-E10 / T);
    const R f1 = C01 / (C01 + C10 + A10);
    l_cp = e.xCp * f1 * A10 * R(K_B) * E10 / n;
  }
  const R l_c = e.xC * three_level_cool(T, n, xH, xH2, xe, c.c_levels, c.c_coll, c.c_ncrit_H, c);
  const R l_o = e.xO * three_level_cool(T, n, xH, xH2, xe, c.o_levels, c.o_coll, c.o_ncrit_H, c);
  R l_co;
  {
    const R Nt = n * e.xCO * R(PC_CM) / p.dvdr;
    const R lT = m_log10(T);
    const R lN = m_log10(rmax(Nt, Tiny<R>::v));
    const R L0 = m_pow10(co_lookup(tab, c, lT, lN, 0));
    const R nh = m_pow10(co_lookup(tab, c, lT, lN, 1));
    l_co = e.xCO * L0 / (R(1) + n / nh);
  }
  const R l_gr = c.grrec[0] * m_pow(T, c.grrec[1]) * m_pow(psi, c.grrec[2] * m_pow(T, -c.grrec[3])) * xe * Zd;
  R l_neb;
  {
    const R lnT4 = m_log(T4);
    R f = R(0);
    for (int k = 6; k >= 0; --k) f = f * lnT4 + c.neb_a[k];
    f = m_pow10(f);
    const R ne2 = n * xe / R(100);
    l_neb = Zg * xe * xHp * c.neb[0] * m_exp(-c.neb[1] / T4) * f /
            (m_sqrt(T4) * (R(1) + c.neb[2] * m_pow(ne2, c.neb[3] - c.neb[4] * lnT4)));
  }
  const R G = dust_heating_per_Zd(r, c, p);
  bool bad;
  const R Td = dust_T(T, n, G, td_guess, c, p, bad);
  v.Td = Td;
  v.td_bad = bad;
  const R l_gd = c.alpha_gd * m_sqrt(T) * (T - Td) * Zd;
  const R S = R(1) / (R(1) + m_exp(-c.sigmoid[0] * (T - R(0.5) * (c.sigmoid[1] + c.sigmoid[2])) /
                                     (c.sigmoid[2] - c.sigmoid[1])));
  const R lgT = m_log10(T);
  const R l_cie = m_pow10(cie_lookup(tab, c, lgT, 0)) + Zg * m_pow10(cie_lookup(tab, c, lgT, 1));
  const double l_hyd = (double)l_lya + (double)l_ci + (double)l_rv + (double)l_cd + (double)l_ff + (double)l_rr;
  const double mid = (double)l_cp + (double)l_c + (double)l_o + (double)l_co + (double)l_gr + (double)l_neb +
                     (double)l_gd;
  v.Lambda = l_hyd + (1.0 - (double)S) * mid + (double)S * (double)l_cie;
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

}  // namespace ism
