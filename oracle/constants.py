"""Physical constants and the paper's printed coefficients (own transcription).

The printed values below are typed in from the paper, independently of the
shared coefficient file; ``tests/test_oracle_pins.py`` checks that the file's
``printed`` section agrees with this transcription.  Stand-in coefficients and
tables (processes the paper only cites) come from the coefficient file.
"""
import json
import os
from dataclasses import dataclass

import numpy as np

# --- physical constants (CODATA 2018, cgs) -----------------------------------
K_B = 1.380649e-16          # erg / K
EV = 1.602176634e-12        # erg
C_LIGHT = 2.99792458e10     # cm / s
M_H = 1.67262192369e-24 + 9.1093837015e-28  # g: hydrogen atom, proton + electron
PC = 3.0856775814913673e18  # cm
YR = 3.15576e7              # s (Julian year)

# --- printed coefficients ----------------------------------------------------
# Sec. 3.2, Table t:param
XC_TOT = 1.6e-4
XO_TOT = 3.2e-4
# Sec. 2.1
MUH0, MUH_SLOPE = 1.40, 0.02
GAMMA = 5.0 / 3.0
# Eq. e:H2form
KGR0 = 3.0e-17
# Eq. eq:H2_pd
ZETA_PD_ISRF = 5.7e-11
# Eqs. eq:H2_pi, e:H_pi and Table t:sb99
SIGMA_PI_H2 = 4.6e-18
SIGMA_PI_H = 3.1e-18
HNU_LYC = 19.4 * EV
# Sec. 3.2.1
ZETA_PI_C_ISRF = 3.43e-10
ZETA_PI_C_CR = 520.0
ZETA_CR_C = 3.85
# Sec. 3.3
XE_T_SWITCH = 2.0e4
# Sec. 2.2 and Eq. e:chi_FUV
J_PE = 1.8e-4
J_LW = 3.0e-5
J_FUV = 2.1e-4
G0_PER_CHI = 1.7
# Eq. e:PE_efficiency
PE_C = (5.22, 2.25, 0.04996, 0.00430, 0.147, 0.431, 0.692)
PSI_OFFSET = 50.0
# Sec. 4.4
Q_PI_H = 3.4 * EV
Q_PI_H2 = 4.4 * EV
# Sec. 4.5
A_EFF = 2.0e-7
F_PUMP = 8.0
# Eq. eq:cooling_fnct
SIG_A, SIG_T1, SIG_T2 = 10.0, 2.0e4, 3.5e4
# Eq. e:k_lya
E21_K = 1.184e5
# Eqs. e:Lambda_ci_H, e:Lambda_cd_H2
E_CI = 13.6 * EV
E_CD = 4.48 * EV
# Eq. e:Lambda_neb
NEB_A = (6.92e-1, -5.86e-1, 8.16e-1, -5.05e-1, 1.18e-1, 7.66e-3, -5.08e-3)
# Eq. eq:gas-dust, Sec. 4.6.4
ALPHA_GD = 3.2e-34
SIGMA_IR10 = 2.0e-25
A_RAD = 7.57e-15
# Sec. 2.3: absorption cross sections per H (times Z'_d)
SIG_D_LYC, SIG_D_LW, SIG_D_PE, SIG_D_OPT = 1.9e-21, 1.5e-21, 0.9e-21, 0.3e-21
# Eq. e:tau_eff
SIG_D_NEFF = 1.0e-21
# Eq. e:cratt
N0_CR = 9.35e20
# Eq. e:fshld_H2_DB
B5 = 3.0
# Sec. 4.6.2 critical densities
CP_NCRIT_E = 53.0
CP_NCRIT_H = (3.0e3, 0.1281, 0.0087)
O_NCRIT_H = (2.5e5, 4.9e4)
C_NCRIT_H = (620.0, 150.0)
# Sec. 7.1.2
T_BB = 6.0
TAU_OPT_RATIO = 1.87
DVDR = 1.0

PRINTED_TRANSCRIPTION = {
    "xC_tot_per_Zg": XC_TOT, "xO_tot_per_Zg": XO_TOT, "muH_0": MUH0, "muH_slope": MUH_SLOPE,
    "gamma": GAMMA, "kgr_0": KGR0, "kgr_shape": [2.0, 0.4, 0.2, 0.08], "cr_H2_coef": [2.0, 2.3, 1.5],
    "cr_H2_destr_factor": 1.65, "zeta_pd_ISRF": ZETA_PD_ISRF, "sigma_pi_H2": SIGMA_PI_H2,
    "sigma_pi_H": SIGMA_PI_H, "hnu_LyC_eV": 19.4, "zeta_pi_C_ISRF": ZETA_PI_C_ISRF,
    "zeta_pi_C_cr_factor": ZETA_PI_C_CR, "zeta_cr_C_factor": ZETA_CR_C, "co_fit": [4.0e3, 50.0, 1.4],
    "xe_T_switch": XE_T_SWITCH, "J_PE_Draine": J_PE, "J_LW_Draine": J_LW, "J_FUV_norm": J_FUV,
    "G0_per_chiFUV": G0_PER_CHI, "pe_prefactor": 1.0e-26, "pe_C": list(PE_C), "psi_offset": PSI_OFFSET,
    "q_pi_H_eV": 3.4, "q_pi_H2_eV": 4.4, "h2form_heat_eV": [0.2, 4.2], "f_pump": F_PUMP,
    "pump_heat_eV": 2.0, "pd_heat_eV": 0.4, "A_eff": A_EFF, "sigmoid": [SIG_A, SIG_T1, SIG_T2],
    "lya_k12": [5.31e-8, 0.15, 5.0, 0.65, 11.84], "lya_E21_K": E21_K, "ci_H_eV": 13.6, "cd_H2_eV": 4.48,
    "neb": [3.68e-23, 3.86, 0.12, 0.38, 0.12], "neb_a": list(NEB_A), "alpha_gd": ALPHA_GD,
    "sigma_IR_10K": SIGMA_IR10, "a_rad": A_RAD, "cp_ncrit_e": CP_NCRIT_E, "cp_ncrit_H": list(CP_NCRIT_H),
    "o_ncrit_H": list(O_NCRIT_H), "c_ncrit_H": list(C_NCRIT_H),
    "sigma_d_abs": [SIG_D_LYC, SIG_D_LW, SIG_D_PE, SIG_D_OPT], "sigma_d_Neff": SIG_D_NEFF,
    "N0_cr": N0_CR, "fshld_H2": [0.965, 0.035, 8.5e-4, 5.0e14], "b5": B5, "eps_sub": 0.1,
    "T_bb": T_BB, "tau_opt_ratio": TAU_OPT_RATIO, "dvdr_kms_pc": DVDR, "x_He_tot": 0.1,
}

COEFF_PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                          "data", "ism_coefficients.json")


class Standins:
    """Stand-in coefficients and tables, read from the coefficient file."""

    def __init__(self, path=COEFF_PATH):
        with open(path) as f:
            doc = json.load(f)
        self.doc = doc
        self.v = {k: np.asarray(e["value"], dtype=np.float64) for k, e in doc["standin"].items()}
        self.tables = {}
        for name, t in doc["tables"].items():
            shape = [a["n"] for a in t["axes"]] + [len(t["columns"])]
            self.tables[name] = (t["axes"], np.asarray(t["values"], dtype=np.float64).reshape(shape))

    def __getitem__(self, k):
        return self.v[k]


_STANDINS = None


def standins():
    global _STANDINS
    if _STANDINS is None:
        _STANDINS = Standins()
    return _STANDINS


@dataclass
class Params:
    """Per-call parameters of the source step (Table t:param, Sec. 6.1, Sec. 7.1.2)."""
    Zg: float = 1.0
    Zd: float = 1.0
    chi0: float = 1.0            # six-ray boundary FUV in Draine units (Sec. 5.2)
    xi_cr0: float = 2.0e-16      # unattenuated primary CR rate (Sec. 2.4)
    cr_mode: int = 0             # 0 constant, 1 attenuate by N_eff (Eq. e:cratt), 2 caller array
    dvdr_kms_pc: float = DVDR
    eps_sub: float = 0.1
    fd_rel: float = 1.0e-3
    kgr_const: int = 0           # 1: k_gr = 3e-17 Z'_d (as in the paper's tests, Sec. 7)
    h2_rovib: int = 1
    max_substeps: int = 100000
    T_floor: float = 1.0
    T_bb: float = T_BB
    tau_opt_ratio: float = TAU_OPT_RATIO

    @property
    def xCtot(self):
        return XC_TOT * self.Zg

    @property
    def xOtot(self):
        return XO_TOT * self.Zg

    @property
    def muH(self):
        return MUH0 - MUH_SLOPE * (self.Zg - 1.0)
