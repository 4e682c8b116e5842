// Host-only: parse the coefficient file into CoefT<double> and the flat table array.
#pragma once
#include <cmath>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "coef.h"
#include "json_mini.h"

namespace ism {
namespace host {

struct Binder {
  const ismjson::Value *sec;
  std::string err;
  bool get(const char *name, double *dst, size_t n) {
    const ismjson::Value *e = sec ? sec->get(name) : nullptr;
    const ismjson::Value *v = e ? e->get("value") : nullptr;
    std::vector<double> vals;
    if (!v || !v->numbers(vals)) { err = std::string("missing coefficient '") + name + "'"; return false; }
    if (vals.size() != n) {
      err = std::string("coefficient '") + name + "' has " + std::to_string(vals.size()) + " values, expected " +
            std::to_string(n);
      return false;
    }
    for (size_t k = 0; k < n; ++k) dst[k] = vals[k];
    return true;
  }
};

#define BIND(b, name, field) ok = ok && b.get(name, &(field), 1)
#define BINDA(b, name, field) ok = ok && b.get(name, field, sizeof(field) / sizeof(field[0]))

inline bool bind_table(const ismjson::Value &tables, const char *name, const std::vector<int> &dims, int ncol,
                std::vector<double> &tab, size_t offset, double *x0, double *dx, std::string &err) {
  const ismjson::Value *t = tables.get(name);
  const ismjson::Value *axes = t ? t->get("axes") : nullptr;
  const ismjson::Value *vals = t ? t->get("values") : nullptr;
  if (!t || !axes || axes->kind != ismjson::Value::Arr || axes->arr.size() != dims.size() || !vals) {
    err = std::string("table '") + name + "' missing or malformed";
    return false;
  }
  size_t total = (size_t)ncol;
  for (size_t d = 0; d < dims.size(); ++d) {
    const ismjson::Value &ax = axes->arr[d];
    const ismjson::Value *n = ax.get("n"), *a0 = ax.get("x0"), *ad = ax.get("dx");
    if (!n || !a0 || !ad || (int)n->num != dims[d] || !(ad->num > 0)) {
      err = std::string("table '") + name + "' axis " + std::to_string(d) + " does not match the expected grid";
      return false;
    }
    x0[d] = a0->num;
    dx[d] = ad->num;
    total *= (size_t)dims[d];
  }
  std::vector<double> v;
  if (!vals->numbers(v) || v.size() != total) {
    err = std::string("table '") + name + "' has the wrong number of values";
    return false;
  }
  for (size_t k = 0; k < total; ++k) tab[offset + k] = v[k];
  return true;
}

inline bool load_coefficients(const char *path, CoefT<double> &c, std::vector<double> &tab, std::string &err) {
  std::ifstream f(path);
  if (!f) { err = std::string("cannot open coefficient file '") + (path ? path : "(null)") + "'"; return false; }
  std::stringstream ss;
  ss << f.rdbuf();
  std::string text = ss.str();
  ismjson::Value doc;
  ismjson::Parser parser(text);
  if (!parser.parse(doc, err)) return false;
  const ismjson::Value *pr = doc.get("printed"), *sd = doc.get("standin"), *tb = doc.get("tables");
  if (!pr || !sd || !tb) { err = "coefficient file lacks printed/standin/tables sections"; return false; }
  std::memset(&c, 0, sizeof(c));
  Binder P{pr, ""}, S{sd, ""};
  bool ok = true;
  BIND(P, "xC_tot_per_Zg", c.xCt_per_Zg); BIND(P, "xO_tot_per_Zg", c.xOt_per_Zg); BIND(P, "muH_0", c.muH0);
  BIND(P, "muH_slope", c.muH_slope); BIND(P, "gamma", c.gamma); BIND(P, "kgr_0", c.kgr0);
  BINDA(P, "kgr_shape", c.kgr_shape); BINDA(P, "cr_H2_coef", c.cr_coef); BIND(P, "cr_H2_destr_factor", c.cr_destr);
  BIND(P, "zeta_pd_ISRF", c.zeta_pd); BIND(P, "sigma_pi_H2", c.sig_pi_H2); BIND(P, "sigma_pi_H", c.sig_pi_H);
  BIND(P, "hnu_LyC_eV", c.hnu_LyC_eV); BIND(P, "zeta_pi_C_ISRF", c.zeta_pi_C);
  BIND(P, "zeta_pi_C_cr_factor", c.zeta_pi_C_cr); BIND(P, "zeta_cr_C_factor", c.zeta_cr_C);
  BINDA(P, "co_fit", c.co_fit); BIND(P, "xe_T_switch", c.xe_T_switch); BIND(P, "J_PE_Draine", c.J_PE);
  BIND(P, "J_LW_Draine", c.J_LW); BIND(P, "J_FUV_norm", c.J_FUV); BIND(P, "G0_per_chiFUV", c.G0_per_chi);
  BIND(P, "pe_prefactor", c.pe_pref); BINDA(P, "pe_C", c.pe_C); BIND(P, "psi_offset", c.psi_off);
  BIND(P, "q_pi_H_eV", c.q_pi_H_eV); BIND(P, "q_pi_H2_eV", c.q_pi_H2_eV); BINDA(P, "h2form_heat_eV", c.h2form_eV);
  BIND(P, "f_pump", c.f_pump); BIND(P, "pump_heat_eV", c.pump_eV); BIND(P, "pd_heat_eV", c.pd_eV);
  BIND(P, "A_eff", c.A_eff); BINDA(P, "sigmoid", c.sigmoid); BINDA(P, "lya_k12", c.lya);
  BIND(P, "lya_E21_K", c.lya_E21); BIND(P, "ci_H_eV", c.ci_eV); BIND(P, "cd_H2_eV", c.cd_eV);
  BINDA(P, "neb", c.neb); BINDA(P, "neb_a", c.neb_a); BIND(P, "alpha_gd", c.alpha_gd);
  BIND(P, "sigma_IR_10K", c.sigma_IR10); BIND(P, "a_rad", c.a_rad); BIND(P, "cp_ncrit_e", c.cp_ncrit_e);
  BINDA(P, "cp_ncrit_H", c.cp_ncrit_H); BINDA(P, "o_ncrit_H", c.o_ncrit_H); BINDA(P, "c_ncrit_H", c.c_ncrit_H);
  BINDA(P, "sigma_d_abs", c.sig_d_abs); BIND(P, "sigma_d_Neff", c.sig_d_Neff); BIND(P, "N0_cr", c.N0_cr);
  BINDA(P, "fshld_H2", c.fshld); BIND(P, "b5", c.b5);
  BINDA(S, "alpha_B", c.alpha_B); BINDA(S, "k_ci_H", c.k_ci_H); BINDA(S, "k_cd_H", c.k_cd_H);
  BINDA(S, "k_cd_H2", c.k_cd_H2); BINDA(S, "alpha_gr_Hp", c.agr_Hp); BINDA(S, "alpha_gr_Cp", c.agr_Cp);
  BINDA(S, "alpha_rrdr_Cp", c.arrdr_Cp); BINDA(S, "k_CpH2", c.k_CpH2); BINDA(S, "x_MH", c.x_MH);
  BINDA(S, "q_cr_H", c.q_cr_H); BINDA(S, "q_cr_H2", c.q_cr_H2); BINDA(S, "k_H2_H", c.k_H2_H);
  BINDA(S, "k_H2_H2", c.k_H2_H2); BINDA(S, "ff", c.ff); BINDA(S, "rr_energy", c.rr_energy);
  BINDA(S, "grrec", c.grrec); BINDA(S, "rovib_lte", c.rovib_lte); BINDA(S, "rovib_low", c.rovib_low);
  BINDA(S, "cp_levels", c.cp_levels); BIND(S, "cp_h2_over_h", c.cp_h2_over_h); BINDA(S, "c_levels", c.c_levels);
  BINDA(S, "c_coll", c.c_coll); BINDA(S, "o_levels", c.o_levels); BINDA(S, "o_coll", c.o_coll);
  if (!ok) { err = !P.err.empty() ? P.err : S.err; return false; }
  tab.assign(TAB_TOTAL, 0.0);
  double x0[2], dx[2];
  if (!bind_table(*tb, "cie", {CIE_N}, CIE_NC, tab, TAB_CIE, x0, dx, err)) return false;
  c.cie_x0 = x0[0]; c.cie_dx = dx[0];
  if (!bind_table(*tb, "co", {CO_NX, CO_NY}, CO_NC, tab, TAB_CO, x0, dx, err)) return false;
  c.co_x0 = x0[0]; c.co_dx = dx[0]; c.co_y0 = x0[1]; c.co_dy = dx[1];
  if (!bind_table(*tb, "cshield", {CS_NX, CS_NY}, 1, tab, TAB_CS, x0, dx, err)) return false;
  c.cs_x0 = x0[0]; c.cs_dx = dx[0]; c.cs_y0 = x0[1]; c.cs_dy = dx[1];
  c.ln_arrdr_T0 = std::log(c.arrdr_Cp[1]);
  c.ln_xMH_T0 = std::log(c.x_MH[2]);
  c.fs_slope_C = std::log(c.c_ncrit_H[0] / c.c_ncrit_H[1]) / std::log(500.0);
  c.fs_slope_O = std::log(c.o_ncrit_H[0] / c.o_ncrit_H[1]) / std::log(500.0);
  c.ln_lya_T = std::log(c.lya[2]);
  c.ln_co0 = std::log(c.co_fit[0]);
  const double *lvs[2] = {c.c_levels, c.o_levels}, *ncs[2] = {c.c_ncrit_H, c.o_ncrit_H};
  double *rats[2] = {c.c_rat, c.o_rat};
  for (int k = 0; k < 2; ++k) {
    rats[k][0] = lvs[k][1] / lvs[k][0];
    rats[k][1] = lvs[k][2] / lvs[k][0];
    rats[k][2] = lvs[k][2] / lvs[k][1];
    rats[k][3] = lvs[k][5] / ncs[k][0];
  }
  c.cp_rat[0] = c.cp_levels[3] / c.cp_ncrit_H[0];
  c.cp_rat[1] = c.cp_levels[1] / c.cp_levels[0];
  c.dust_A = c.sigma_IR10 / 100.0 * C_LIGHT * c.a_rad;
  c.inv_J_FUV = 1.0 / c.J_FUV;
  c.inv_kci_T = 1.0 / c.k_ci_H[2];
  c.rsqrt_kci_T = 1.0 / std::sqrt(c.k_ci_H[2]);
  c.sigmoid_iw = 1.0 / (c.sigmoid[2] - c.sigmoid[1]);
  c.inv_fshld_N = 1.0 / c.fshld[3];
  c.inv_b5 = 1.0 / c.b5;
  c.cie_idx = 1.0 / c.cie_dx;
  c.co_idx = 1.0 / c.co_dx;
  c.co_idy = 1.0 / c.co_dy;
  c.cs_idx = 1.0 / c.cs_dx;
  c.cs_idy = 1.0 / c.cs_dy;
  // log10 cooling columns are kept relative to 1e-24 erg cm^3 s^-1 on the device (see coef.h)
  for (int i = 0; i < CIE_N; ++i)
    for (int k = 0; k < 2; ++k) tab[TAB_CIE + i * CIE_NC + k] += TAB_LOG_OFFSET;
  for (int i = 0; i < CO_NX * CO_NY; ++i) tab[TAB_CO + i * CO_NC] += TAB_LOG_OFFSET;
  return true;
}


// Every field of CoefT is R or an array of R: convert member-wise through a flat view.
inline void coef_to_f32(const CoefT<double> &d, CoefT<float> &f) {
  static_assert(sizeof(CoefT<double>) % sizeof(double) == 0, "CoefT must hold only doubles");
  static_assert(sizeof(CoefT<double>) / sizeof(double) == sizeof(CoefT<float>) / sizeof(float), "layout");
  const double *s = reinterpret_cast<const double *>(&d);
  float *t = reinterpret_cast<float *>(&f);
  for (size_t k = 0; k < sizeof(CoefT<double>) / sizeof(double); ++k) t[k] = (float)s[k];
}

}  // namespace host
}  // namespace ism
