"""Local shielding-length radiation and the shielded one-zone equilibrium (Sec. 7.1.2; test
infrastructure).

A cell of density n sees the background field through a shielding column N_shld = n L_shld:
chi_PE/LW = chi0 exp(-sigma_d,PE/LW Z'_d N_shld); the CR rate follows Eq. e:cratt with
N_eff = N_shld; H2 and C shield themselves through N_H2 = 0.5 x_H2 n L_shld and
N_C = 0.5 x_C n L_shld from the current abundances.  The equilibrium alternates long steps of
the source step with re-evaluation of that radiation until the state stops changing.
"""
import numpy as np

from . import constants as C
from . import step
from .columns import cr_attenuation, f_shld_C, f_shld_H2

PC = C.PC


def shielding_length(n, L0_pc=5.0, n0=100.0, a=0.7):
    """L_shld = L0 (n / n0)^-a in cm (Sec. 7.1.2: L0 = 5 pc, n0 = 100 cm^-3, a = 0.7)."""
    return L0_pc * PC * (np.asarray(n, dtype=np.float64) / n0) ** (-a)


def local_shielding(n, xH2, xC, L, par):
    """Radiation dict (chi_PE, chi_LW, chi_H2, chi_C, phi, xi, Neff) of cells shielded by the
    local column n L."""
    n = np.asarray(n, dtype=np.float64)
    N = n * L
    Zd = par.Zd
    chiPE = par.chi0 * np.exp(-C.SIG_D_PE * Zd * N)
    chiLW = par.chi0 * np.exp(-C.SIG_D_LW * Zd * N)
    NH2 = 0.5 * xH2 * n * L
    NC = 0.5 * (np.zeros_like(n) if xC is None else xC) * n * L
    xi = cr_attenuation(N, par.xi_cr0) if par.cr_mode == 1 else np.full_like(n, par.xi_cr0)
    return dict(chi_PE=chiPE, chi_LW=chiLW, chi_H2=chiLW * f_shld_H2(NH2), chi_C=chiLW * f_shld_C(NC, NH2),
                phi=np.zeros_like(n), xi=xi, Neff=N)


def shielded_equilibrium(n, par, T0=100.0, xH2_0=0.1, xHp_0=1e-3, dt_yr=1e7, outer=30, tol=1e-7):
    """Steady state of the shielded one-zone model at densities n: returns the final step
    output (T, xH2, xHp, xCp, xCO, xe, ...) and the final radiation.  tol = 0 runs all
    `outer` rounds."""
    n = np.asarray(n, dtype=np.float64)
    N = n.size
    L = shielding_length(n)
    T, xH2, xHp = np.full(N, T0), np.full(N, xH2_0), np.full(N, xHp_0)
    xC = np.zeros(N)
    out = rad = None
    for _ in range(outer):
        rad = local_shielding(n, xH2, xC, L, par)
        out = step.chem_cool_step(n, T, xH2, xHp, rad, dt_yr * C.YR, par)
        change = max(np.max(np.abs(out["T"] / T - 1.0)), np.max(np.abs(out["xH2"] - xH2)))
        T, xH2, xHp = out["T"], out["xH2"], out["xHp"]
        xC = np.maximum(par.xCtot - out["xCp"] - out["xCO"], 0.0)
        if change < tol:
            break
    return out, rad
