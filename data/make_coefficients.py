"""Write ``ism_coefficients.json``: every number the ISM source step consumes.

The file is input data, read at run time by both the CPU oracle and the HIP
library (``ism_init``).  It has three sections:

``printed``  constants the paper states, each with the section/equation/table
             it comes from (Kim, Gong, Kim & Ostriker, arXiv:2210.08024).
``standin``  coefficients of processes the paper only cites (Gnat & Ferland
             2012, Omukai+2010, Tielens & Hollenbach 1985, Gong+2017 tables,
             Janev+1987, Glover+2007/2010, Weingartner & Draine 2001b,c,
             Draine 2011, Glassgold+2012, Visser+2018, Moseley+2021).  None of
             those sources is available here, so each entry is a labelled
             stand-in: a published fitting form recalled from the literature or
             a smooth made-up shape of the right magnitude.  ``paper_pinned`` is
             false for all of them.
``tables``   the three tabulated stand-ins (CIE cooling/ionisation, CO LVG
             cooling, C shielding) on regular log grids.  The interpolation
             rule that turns a table into a function is part of the method
             definition: piecewise linear in the tabulated column along each
             axis, arguments clamped to the grid.

Run ``python data/make_coefficients.py`` to regenerate the JSON.  Uses numpy
only; imports nothing from the oracle or the library.
"""
import json
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def printed():
    """Constants printed in the paper (value, citation)."""
    P = {}

    def add(name, value, cite):
        P[name] = {"value": value, "cite": cite}

    # gas state (Sec. 2.1, Table t:param)
    add("xC_tot_per_Zg", 1.6e-4, "Sec. 3.2 / Table t:param: x_C,tot = 1.6e-4 Z'_g")
    add("xO_tot_per_Zg", 3.2e-4, "Sec. 3.2 / Table t:param: x_O,tot = 3.2e-4 Z'_g")
    add("muH_0", 1.40, "Sec. 2.1: mu_H = 1.40 - 0.02 (Z'_g - 1)")
    add("muH_slope", 0.02, "Sec. 2.1: mu_H = 1.40 - 0.02 (Z'_g - 1)")
    add("x_He_tot", 0.1, "Sec. 2.1: helium abundance 0.1 (P = (1.1 + x_e - x_H2) n k T)")
    add("gamma", 5.0 / 3.0, "Sec. 2.1: adiabatic index 5/3")
    # H2 (Sec. 3.1.1)
    add("kgr_0", 3.0e-17, "Eq. e:H2form: 3.0e-17 Z'_d cm^3 s^-1")
    add("kgr_shape", [2.0, 0.4, 0.2, 0.08], "Eq. e:H2form: 2 T2^1/2 / (1 + 0.4 T2^1/2 + 0.2 T2 + 0.08 T2^2)")
    add("cr_H2_coef", [2.0, 2.3, 1.5], "Eq. eq:H2_cr: zeta_cr,H2 = 2 xi (2.3 x_H2 + 1.5 x_H)")
    add("cr_H2_destr_factor", 1.65, "Eq. e:HH: factor 1.65 on zeta_cr,H2")
    add("zeta_pd_ISRF", 5.7e-11, "Eq. eq:H2_pd: 5.7e-11 s^-1")
    add("sigma_pi_H2", 4.6e-18, "Eq. eq:H2_pi / Table t:sb99 row 9")
    add("sigma_pi_H", 3.1e-18, "Eq. e:H_pi / Table t:sb99 row 8")
    add("hnu_LyC_eV", 19.4, "Sec. 3.1.1 / Table t:sb99 row 10")
    # carbon / oxygen (Sec. 3.2)
    add("zeta_pi_C_ISRF", 3.43e-10, "Sec. 3.2.1 text (Table t:param prints 3.5e-10; the equation's 3.43e-10 is used)")
    add("zeta_pi_C_cr_factor", 520.0, "Sec. 3.2.1: CR-induced C photoionisation 520 x 2 x_H2 xi")
    add("zeta_cr_C_factor", 3.85, "Sec. 3.2.1: zeta_cr,C = 3.85 xi")
    add("co_fit", [4.0e3, 50.0, 1.4], "Eq. e:CO_fit: (4e3 Z'_d xi16^-2)^(chi^1/3) (50 xi16 / Z'_d^1.4)")
    add("xe_T_switch", 2.0e4, "Sec. 3.3: cold / hot electron closure at T = 2e4 K")
    # radiation normalisation (Sec. 2.2)
    add("J_PE_Draine", 1.8e-4, "Sec. 2.2: J^Draine_PE = 1.8e-4 erg cm^-2 s^-1 sr^-1")
    add("J_LW_Draine", 3.0e-5, "Sec. 2.2: J^Draine_LW = 3.0e-5 erg cm^-2 s^-1 sr^-1")
    add("J_FUV_norm", 2.1e-4, "Eq. e:chi_FUV: 2.1e-4 erg cm^-2 s^-1 sr^-1")
    add("G0_per_chiFUV", 1.7, "Sec. 4.2: G0 = 1.7 chi_FUV")
    # photoelectric heating (Sec. 4.2)
    add("pe_prefactor", 1.0e-26, "Eq. eq:photoel_heat: 1e-26 G0 eps Z'_d erg s^-1")
    add("pe_C", [5.22, 2.25, 0.04996, 0.00430, 0.147, 0.431, 0.692], "Eq. e:PE_efficiency: C0..C6")
    add("psi_offset", 50.0, "Sec. 4.2: 50 K^1/2 cm^3 added to psi")
    # photoionisation heating (Sec. 4.4)
    add("q_pi_H_eV", 3.4, "Sec. 4.4 / Table t:sb99 row 11")
    add("q_pi_H2_eV", 4.4, "Sec. 4.4 / Table t:sb99 row 12")
    # H2 heating (Sec. 4.5)
    add("h2form_heat_eV", [0.2, 4.2], "Eq. e:Gamma_H2form: 0.2 eV + 4.2 eV / (1 + n_crit/n)")
    add("f_pump", 8.0, "Eq. e:Gamma_H2pump: f_pump = 8")
    add("pump_heat_eV", 2.0, "Eq. e:Gamma_H2pump: 2 eV")
    add("pd_heat_eV", 0.4, "Eq. e:Gamma_H2diss: 0.4 eV")
    add("A_eff", 2.0e-7, "Sec. 4.5: A_eff = 2e-7 s^-1")
    # cooling assembly (Sec. 4.6)
    add("sigmoid", [10.0, 2.0e4, 3.5e4], "Eq. eq:cooling_fnct: a = 10, T_t1 = 2e4, T_t2 = 3.5e4")
    add("lya_k12", [5.31e-8, 0.15, 5.0, 0.65, 11.84], "Eq. e:k_lya")
    add("lya_E21_K", 1.184e5, "Sec. 4.6.1: E21 / k_B = 1.184e5 K")
    add("ci_H_eV", 13.6, "Eq. e:Lambda_ci_H: 13.6 eV per ionisation")
    add("cd_H2_eV", 4.48, "Eq. e:Lambda_cd_H2: 4.48 eV per dissociation")
    add("neb", [3.68e-23, 3.86, 0.12, 0.38, 0.12], "Eq. e:Lambda_neb prefactor, exponent, 0.12 n_e2^(0.38 - 0.12 ln T4)")
    add("neb_a", [6.92e-1, -5.86e-1, 8.16e-1, -5.05e-1, 1.18e-1, 7.66e-3, -5.08e-3], "Eq. e:Lambda_neb: log10 f_neb coefficients a0..a6")
    add("alpha_gd", 3.2e-34, "Eq. eq:gas-dust: 3.2e-34 erg cm^3 s^-1 K^-3/2")
    add("sigma_IR_10K", 2.0e-25, "Sec. 4.6.4: sigma_IR = 2e-25 Z'_d (T_d/10 K)^2 cm^2 H^-1")
    add("a_rad", 7.57e-15, "Sec. 4.6.4: a = 7.57e-15 erg cm^-3 K^-4")
    add("cp_ncrit_e", 53.0, "Sec. 4.6.2: C II 158um n_e,crit = 53 T4^1/2 cm^-3")
    add("cp_ncrit_H", [3.0e3, 0.1281, 0.0087], "Sec. 4.6.2: C II 158um n_H,crit = 3e3 T2^(-0.1281 - 0.0087 ln T2)")
    add("o_ncrit_H", [2.5e5, 4.9e4], "Sec. 4.6.2: O I 63um n_H,crit at T = 10 K and 5000 K")
    add("c_ncrit_H", [620.0, 150.0], "Sec. 4.6.2: C I 610um n_H,crit at T = 10 K and 5000 K")
    # dust cross sections (Sec. 2.3, Sec. 5.3)
    add("sigma_d_abs", [1.9e-21, 1.5e-21, 0.9e-21, 0.3e-21], "Sec. 2.3: absorption per H / Z'_d for LyC, LW, PE, OPT")
    add("sigma_d_Neff", 1.0e-21, "Eq. e:tau_eff: N_eff = tau_PE,eff / (1e-21 Z'_d)")
    add("N0_cr", 9.35e20, "Eq. e:cratt: N_0 = 9.35e20 cm^-2")
    # shielding (Sec. 5.1)
    add("fshld_H2", [0.965, 0.035, 8.5e-4, 5.0e14], "Eq. e:fshld_H2_DB")
    add("b5", 3.0, "Sec. 5.1: b5 = 3")
    # update (Sec. 6.1)
    add("eps_sub", 0.1, "Sec. 6.1: factor 0.1 in the substep size")
    # test settings (Sec. 7.1.2)
    add("T_bb", 6.0, "Sec. 7.1.2: grains bathed in a 6 K blackbody")
    add("tau_opt_ratio", 1.87, "Sec. 7.1.2: tau_OPT = tau_PE / 1.87; equal FUV and OPT dust heating unattenuated")
    add("dvdr_kms_pc", 1.0, "Sec. 7.1.2: |dv/dr| = 1 km s^-1 pc^-1")
    return P


def standin():
    """Stand-ins for cited-but-absent microphysics (none is paper-pinned)."""
    S = {}

    def add(name, value, provenance):
        S[name] = {"value": value, "provenance": provenance, "paper_pinned": False}

    add("alpha_B", [2.54e-13, -0.8163, -0.0208],
        "case-B H recombination 2.54e-13 T4^(-0.8163 - 0.0208 ln T4) (Draine 2011 fit, recalled, unverified); "
        "stands in for Glover+2010")
    add("k_ci_H", [5.85e-11, 157809.1, 1.0e5],
        "H collisional ionisation 5.85e-11 T^1/2 exp(-157809.1/T) / (1 + (T/1e5)^1/2) (Cen 1992 form, recalled); "
        "stands in for Janev+1987")
    add("k_cd_H", [6.67e-12, 63590.0],
        "H2 + H dissociation 6.67e-12 T^1/2 exp(-(1 + 63590/T)) (low-density form, recalled); stands in for Glover+2007")
    add("k_cd_H2", [5.996e-30, 4.1881, 6.761e-6, 5.6881, 54657.4],
        "H2 + H2 dissociation 5.996e-30 T^4.1881 (1 + 6.761e-6 T)^-5.6881 exp(-54657.4/T) (low-density form, "
        "recalled); stands in for Glover+2007")
    add("alpha_gr_Hp", [12.25, 8.074e-6, 1.378, 5.087e2, 1.586e-2, 0.4723, 1.102e-5],
        "grain-assisted H+ recombination 1e-14 C0 / (1 + C1 psi^C2 (1 + C3 T^C4 psi^(-C5 - C6 ln T))) Z'_d "
        "(Weingartner & Draine 2001c form, coefficients recalled, unverified)")
    add("alpha_gr_Cp", [45.58, 6.089e-3, 1.128, 4.331e2, 4.845e-2, 0.8120, 1.333e-4],
        "grain-assisted C+ recombination, same form (Weingartner & Draine 2001c, recalled, unverified)")
    add("alpha_rrdr_Cp", [4.67e-12, 300.0, -0.6],
        "C+ radiative + dielectronic recombination 4.67e-12 (T/300)^-0.6 (simple power law, recalled); "
        "stands in for the Gong+2017 Table 1 fit")
    add("k_CpH2", [2.31e-13, -1.3, 23.0],
        "C+ + H2 -> CH2+ 2.31e-13 T^-1.3 exp(-23/T) (recalled); stands in for Gong+2017 Table 1")
    add("x_MH", [2.0, 1.0e-7, 300.0, -0.5],
        "molecular ions x_MH+ = 2 x_H2 (c xi / (alpha_dr n))^1/2 with alpha_dr = 1e-7 (T/300)^-0.5 "
        "(dense-limit dissociative-recombination balance, made up); stands in for Draine 2011 Eq. 16.25")
    add("q_cr_H", [6.5, 26.4, 0.07],
        "CR heating per ionisation in H: 6.5 + 26.4 (x_e / (x_e + 0.07))^1/2 eV (recalled); "
        "stands in for Draine 2011 Ch. 30")
    add("q_cr_H2", [10.0, 13.0, 17.0, 18.0, 2.0, 4.0, 7.0, 10.0],
        "CR heating per ionisation in H2: piecewise linear in log10 n through (2,10), (4,13), (7,17), (10,18) eV, "
        "flat outside (recalled); stands in for Glassgold+2012 Table 6")
    add("k_H2_H", [1.0e-12, 1000.0],
        "H2* de-excitation by H 1e-12 T^1/2 exp(-1000/T) (recalled); stands in for Visser+2018 App. A")
    add("k_H2_H2", [1.4e-12, 18100.0, 1200.0],
        "H2* de-excitation by H2 1.4e-12 T^1/2 exp(-18100/(T + 1200)) (recalled); stands in for Visser+2018 App. A")
    add("ff", [1.42e-27, 1.3],
        "H free-free 1.42e-27 g_ff T^1/2 x_e x_H+ with g_ff = 1.3 (recalled); stands in for Draine 2011 Eq. 10.12")
    add("rr_energy", [0.684, -0.0416],
        "case-B recombination energy loss (0.684 - 0.0416 ln T4) k T per recombination (recalled); "
        "stands in for Draine 2011 Eqs. 27.14/27.23")
    add("grrec", [4.65e-30, 0.94, 0.74, 0.068],
        "grain recombination cooling 4.65e-30 T^0.94 psi^(0.74 T^-0.068) x_e Z'_d (Bakes & Tielens form, recalled); "
        "stands in for Weingartner & Draine 2001b Table 3")
    add("rovib_lte", [9.5e-22, 3.76, 0.12, 2.1, 0.13, 3.0e-24, 0.51, 6.7e-19, 5.86, 1.6e-18, 11.7],
        "H2 ro-vibrational LTE rate per molecule (rotational + vibrational, Hollenbach & McKee 1979 form, recalled); "
        "stands in for Moseley+2021")
    add("rovib_low", [-103.0, 97.59, -48.05, 10.80, -0.9032, 1.0, 4.0],
        "H2 low-density rate coefficient log10 L0 = poly4(log10 T), log10 T clamped to [1, 4] (Galli & Palla 1998 "
        "form, recalled); stands in for Moseley+2021")
    # fine structure: atomic data (recalled) and collision-rate shapes
    add("cp_levels", [2.0, 4.0, 91.25, 2.3e-6],
        "C+ 2-level: g0, g1, E10/k [K], A10 [s^-1] (atomic data, recalled)")
    add("cp_h2_over_h", 0.5, "C+ de-excitation by H2 relative to H (made up); stands in for Gong+2017 Table 3")
    add("c_levels", [1.0, 3.0, 5.0, 23.6, 62.4, 7.93e-8, 1.71e-14, 2.65e-7],
        "C 3-level: g0, g1, g2, E1/k, E2/k [K], A10, A20, A21 [s^-1] (atomic data, recalled)")
    add("c_coll", [0.5, 1.5, 0.5, 3.0e-9, 0.4],
        "C collision shapes: k20,H/k10,H, k21,H/k10,H, H2/H ratio, k10,e at 1e4 K, e-rate T4 exponent (made up); "
        "stands in for Gong+2017 Table 3")
    add("o_levels", [5.0, 3.0, 1.0, 227.7, 326.6, 8.91e-5, 1.34e-10, 1.75e-5],
        "O 3-level: g0, g1, g2, E1/k, E2/k [K], A10, A20, A21 [s^-1] (atomic data, recalled)")
    add("o_coll", [0.4, 0.05, 0.5, 1.4e-8, 0.39],
        "O collision shapes: k20,H/k10,H, k21,H/k10,H, H2/H ratio, k10,e at 1e4 K, e-rate T4 exponent (made up); "
        "stands in for Gong+2017 Table 3")
    add("sigma_C_pi", 1.6e-17, "C continuum self-shielding cross section used to build the C-shielding stand-in table")
    return S


def interp_grid(x0, dx, n):
    return x0 + dx * np.arange(n)


def tables():
    T = {}
    # --- CIE (stands in for Gnat & Ferland 2012 ion-by-ion tables) ---------
    lgT = interp_grid(4.0, 0.05, 101)

    def bump(x, c, w, a):
        return a * np.exp(-0.5 * ((x - c) / w) ** 2)

    lam_he = bump(lgT, 5.0, 0.22, 1.0e-22) + bump(lgT, 4.4, 0.08, 1.5e-23) + 1.0e-26 * 10 ** (0.5 * (lgT - 6.0))
    lam_met = (bump(lgT, 5.35, 0.28, 4.0e-22) + bump(lgT, 5.95, 0.35, 9.0e-23) + bump(lgT, 7.2, 0.45, 1.0e-23)
               + 1.0e-27)
    f1 = 1.0 / (1.0 + np.exp(-(lgT - 4.45) / 0.06))
    f2 = 1.0 / (1.0 + np.exp(-(lgT - 4.95) / 0.06))
    xe_he = 0.1 * (f1 + f2)
    xe_met = 1.2e-3 * (1.0 / (1.0 + np.exp(-(lgT - 5.3) / 0.25)) + 1.0 / (1.0 + np.exp(-(lgT - 6.6) / 0.3)))
    T["cie"] = {
        "axes": [{"name": "log10_T", "x0": 4.0, "dx": 0.05, "n": 101}],
        "columns": ["log10_lambda_He", "log10_lambda_metal", "xe_He", "xe_metal"],
        "interp": ["linear in column vs log10 T; log10 T clamped to the grid"],
        "values": np.stack([np.log10(lam_he), np.log10(lam_met), xe_he, xe_met], axis=1).ravel().tolist(),
        "provenance": "stand-in for Gnat & Ferland 2012 CIE (He, metals at Asplund09 ratios): smooth bumps shaped "
                      "so the total with hydrogen peaks near 5e-22 erg cm^3 s^-1 at a few 1e5 K (made up)",
        "paper_pinned": False,
    }
    # --- CO LVG cooling (stands in for Omukai+2010) -------------------------
    lT = interp_grid(0.5, 0.25, 13)
    lN = interp_grid(14.0, 0.5, 15)
    TT, NN = np.meshgrid(10 ** lT, 10 ** lN, indexing="ij")
    L0 = 4.0e-26 * (TT / 10.0) ** 2 / (1.0 + (NN / 1.0e17) ** 0.5)
    nhalf = 2.0e3 * (TT / 10.0) ** 0.5 * (1.0 + NN / 1.0e16) ** -0.2
    T["co"] = {
        "axes": [{"name": "log10_T", "x0": 0.5, "dx": 0.25, "n": 13},
                 {"name": "log10_Ntilde", "x0": 14.0, "dx": 0.5, "n": 15}],
        "columns": ["log10_L0", "log10_nhalf"],
        "interp": ["bilinear in column vs (log10 T, log10 Ntilde); both clamped to the grid"],
        "values": np.stack([np.log10(L0), np.log10(nhalf)], axis=2).ravel().tolist(),
        "provenance": "stand-in for the Omukai+2010 LVG CO table: per-molecule rate n L0 / (1 + n/n_half) (made up)",
        "paper_pinned": False,
    }
    # --- C shielding (stands in for Tielens & Hollenbach 1985) --------------
    lC = interp_grid(10.0, 0.5, 23)
    lH = interp_grid(10.0, 0.5, 29)
    CC, HH = np.meshgrid(10 ** lC, 10 ** lH, indexing="ij")
    log10f = (-1.6e-17 * CC - 0.5 * np.log(1.0 + HH / 1.0e21) - 0.3 * np.log(1.0 + HH / 3.0e22)) / math.log(10.0)
    T["cshield"] = {
        "axes": [{"name": "log10_N_C", "x0": 10.0, "dx": 0.5, "n": 23},
                 {"name": "log10_N_H2", "x0": 10.0, "dx": 0.5, "n": 29}],
        "columns": ["log10_f_shld_C"],
        "interp": ["bilinear in log10 f vs (log10 N_C, log10 N_H2); both clamped to the grid"],
        "values": log10f.ravel().tolist(),
        "provenance": "stand-in for the Tielens & Hollenbach 1985 C self- and H2 cross-shielding: "
                      "exp(-1.6e-17 N_C) (1 + N_H2/1e21)^-0.5 (1 + N_H2/3e22)^-0.3 (made up)",
        "paper_pinned": False,
    }
    return T


def main():
    doc = {
        "schema": "ism-coefficients/1",
        "about": "Coefficients of the ISM photochemistry + heating/cooling source step of arXiv:2210.08024. "
                 "'printed' values carry their citation; 'standin' and 'tables' replace cited-but-absent data.",
        "printed": printed(),
        "standin": standin(),
        "tables": tables(),
    }
    out = os.path.join(HERE, "ism_coefficients.json")
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
