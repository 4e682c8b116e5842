"""Plane-parallel H I -> H2 transition (Sec. 7.3; test infrastructure).

A uniform slab along x, lit by a beam of surface intensity chi0 through x = 0, with a constant
H2 formation coefficient and no cosmic rays, evolved by alternating the beamed columns and long
steps of the source step until steady; the transition column is the total hydrogen column
from the surface to the point where 2 x_H2 = 1/2.  The analytic approximation of Bialy &
Sternberg quoted in Sec. 7.3 (Eqs. e:NH_trans, e:alpha, e:G) gives the same column for the
beamed, CR-free case.
"""
import numpy as np

from . import constants as C
from . import step
from .columns import columns_beam


def analytic_ntrans(n, chi0, kgr=3.0e-17, sigma_d=None, beta=0.7):
    """Eq. e:NH_trans with alpha of Eq. e:alpha and G of Eq. e:G; sigma_d = 1.9e-21 sigma~ is
    the LW dust cross section (sigma~ = sigma_d / 1.9e-21)."""
    sigma_d = C.SIG_D_LW if sigma_d is None else sigma_d
    st = sigma_d / 1.9e-21
    alpha = 3.8e4 * chi0 * (3.0e-17 / kgr) * (1.0e2 / n)
    G = 3.0e-5 * st * (9.9 / (1.0 + 8.9 * st)) ** 0.37
    return beta / sigma_d * np.log(1.0 + (alpha * G / 2.0) ** (1.0 / beta))


def transition_column(n, xH2, dx):
    """Total H column from the surface (x = 0) to where 2 x_H2 crosses 1/2 (linear in the
    column between cell centres)."""
    f = 2.0 * np.asarray(xH2, dtype=np.float64)
    Nc = (np.arange(f.size) + 0.5) * n * dx
    k = np.nonzero((f[:-1] < 0.5) & (f[1:] >= 0.5))[0]
    if k.size == 0:
        return np.nan
    k = k[0]
    return Nc[k] + (0.5 - f[k]) * (Nc[k + 1] - Nc[k]) / (f[k + 1] - f[k])


def slab_steady(n, chi0, nx, dx, dt_yr=1e6, steps=200, par=None):
    """Steady slab: returns (x_H2 profile, step output) after `steps` rounds of (beamed columns,
    step of dt_yr), starting atomic at 100 K."""
    from .constants import Params
    par = par or Params(chi0=chi0, xi_cr0=0.0, kgr_const=1, cr_mode=0)
    shape = (1, 1, nx)
    nn = np.full(shape, float(n))
    T, xH2, xHp = np.full(nx, 100.0), np.full(nx, 1e-6), np.full(nx, 1e-4)
    xC = np.zeros(shape)
    out = None
    for _ in range(steps):
        r = columns_beam(nn, xH2.reshape(shape), xC, dx, par)
        rad = dict(chi_PE=r["chi_PE"].ravel(), chi_LW=r["chi_LW"].ravel(), chi_H2=r["chi_H2"].ravel(),
                   chi_C=r["chi_C"].ravel(), phi=np.zeros(nx), xi=r["xi"].ravel(), Neff=r["N_eff"].ravel())
        out = step.chem_cool_step(nn.ravel(), T, xH2, xHp, rad, dt_yr * C.YR, par)
        T, xH2, xHp = out["T"], out["xH2"], out["xHp"]
        xC = np.maximum(par.xCtot - out["xCp"] - out["xCO"], 0.0).reshape(shape)
    return xH2, out
