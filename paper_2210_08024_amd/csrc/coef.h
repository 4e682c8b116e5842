// Coefficients of the source step, as stored on the device.
//
// Every printed constant (with its section/equation in the coefficient file) and
// every stand-in coefficient is loaded from the coefficient file by ism_init and
// kept twice: once in double (plain path) and once in float (mixed path).  The
// three tables (CIE, CO LVG, C shielding) are stored contiguously in `tab` order:
// CIE [101 x 4] at TAB_CIE, CO [13 x 15 x 2] at TAB_CO, C shielding [23 x 29] at
// TAB_CS.  The step kernels stage CIE + CO into LDS per workgroup.
#pragma once
#include <cstdint>

namespace ism {

// physical constants (CODATA 2018, cgs); the paper's own constants come from the file
constexpr double K_B = 1.380649e-16;
constexpr double EV = 1.602176634e-12;
constexpr double C_LIGHT = 2.99792458e10;
constexpr double M_H = 1.67262192369e-24 + 9.1093837015e-28;  // g: hydrogen atom, proton + electron
constexpr double PC_CM = 3.0856775814913673e18;
constexpr double LN10 = 2.302585092994045684;

constexpr int TAB_CIE = 0;
constexpr int CIE_N = 101, CIE_NC = 4;
constexpr int TAB_CO = TAB_CIE + CIE_N * CIE_NC;         // 404
constexpr int CO_NX = 13, CO_NY = 15, CO_NC = 2;
constexpr int TAB_CS = TAB_CO + CO_NX * CO_NY * CO_NC;     // 794
constexpr int CS_NX = 23, CS_NY = 29;
constexpr int TAB_TOTAL = TAB_CS + CS_NX * CS_NY;          // 1461
constexpr int TAB_STEP = TAB_CS;                           // CIE + CO, staged in LDS by the step
// The device copies of the log10 cooling columns (CIE columns 0-1, CO column 0) hold
// log10(value) + TAB_LOG_OFFSET; lookups multiply 10^(entry) by TAB_LOG_SCALE.
constexpr double TAB_LOG_OFFSET = 24.0;
constexpr double TAB_LOG_SCALE = 1e-24;

template <class R>
struct CoefT {
  // ---- printed ----
  R xCt_per_Zg, xOt_per_Zg, muH0, muH_slope, gamma;
  R kgr0, kgr_shape[4];
  R cr_coef[3], cr_destr;
  R zeta_pd, sig_pi_H2, sig_pi_H, hnu_LyC_eV;
  R zeta_pi_C, zeta_pi_C_cr, zeta_cr_C, co_fit[3], xe_T_switch;
  R J_PE, J_LW, J_FUV, G0_per_chi, pe_pref, pe_C[7], psi_off;
  R q_pi_H_eV, q_pi_H2_eV, h2form_eV[2], f_pump, pump_eV, pd_eV, A_eff;
  R sigmoid[3], lya[5], lya_E21, ci_eV, cd_eV, neb[5], neb_a[7];
  R alpha_gd, sigma_IR10, a_rad, cp_ncrit_e, cp_ncrit_H[3], o_ncrit_H[2], c_ncrit_H[2];
  R sig_d_abs[4], sig_d_Neff, N0_cr, fshld[4], b5;
  // ---- stand-ins ----
  R alpha_B[3], k_ci_H[3], k_cd_H[2], k_cd_H2[5], agr_Hp[7], agr_Cp[7], arrdr_Cp[3], k_CpH2[3], x_MH[4];
  R q_cr_H[3], q_cr_H2[8], k_H2_H[2], k_H2_H2[3], ff[2], rr_energy[2], grrec[4];
  R rovib_lte[11], rovib_low[7], cp_levels[4], cp_h2_over_h, c_levels[8], c_coll[5], o_levels[8], o_coll[5];
  // ---- derived on the host after loading (logs of constants used inside exponents) ----
  R ln_arrdr_T0, ln_xMH_T0, fs_slope_C, fs_slope_O, ln_lya_T, ln_co0;
  // ---- quotients of constants, formed once on the host so the kernels multiply ----
  R c_rat[4], o_rat[4];  // C and O atoms: g1/g0, g2/g0, g2/g1, A10/n_crit,H
  R cp_rat[2];           // C+: A10/n_crit,H, g1/g0
  R dust_A;              // sigma_IR(10 K)/100 c a_rad
  R inv_J_FUV, inv_kci_T, rsqrt_kci_T, sigmoid_iw;  // 1 / k_ci_H[2] and its square root
  R inv_fshld_N, inv_b5;  // 1 / the H2 shielding column scale, 1 / b5
  R cie_idx, co_idx, co_idy, cs_idx, cs_idy;  // 1 / table spacing
  // ---- table axes ----
  R cie_x0, cie_dx;
  R co_x0, co_dx, co_y0, co_dy;
  R cs_x0, cs_dx, cs_y0, cs_dy;
};

// Per-call parameters, derived on the host from ism_params.
template <class R>
struct ParT {
  R Zg, Zd, chi0, dvdr, eps_sub, fd_rel, T_floor, T_bb, tau_ratio;
  R xCt, xOt, muH, lnZd, idvdr;  // idvdr = 1 / dvdr
  R fd_ln, fd_inv, fd_sqrt;       // ln, reciprocal and square root of 1 + fd_rel
  int32_t kgr_const, h2_rovib, max_sub, cr_mode;
};

}  // namespace ism
