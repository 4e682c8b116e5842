"""Six-ray diffuse-UV transfer, shielding, effective column and CR attenuation (Secs. 5.1-5.3), FP64.

For a uniform cubic grid of cell size dx, rays enter from the six domain
faces along +-x, +-y, +-z with luminosity c E_0 dx^2, E_0 = chi0 E^Draine / 6
(Sec. 5.2).  With Eq. e:Erad and Delta s = dx, a cell's energy density in band
b is the sum over the six rays of

    (chi0 / 6) exp(-sigma_b N_in) (1 - exp(-dtau)) / dtau,   dtau = sigma_b n dx,

where N_in is the hydrogen column from the face to the cell's entry face.
chi_H2 additionally weights each ray by f_shld,H2(N_H2,in + n x_H2 dx / 2)
(Eq. e:Erad_H2, Eq. e:fshld_H2_DB; half the cell's own column, reading of the
footnote on the shielding column), chi_C by the C shielding function of
(N_C, N_H2) at the same mid-cell columns.  N_eff = -ln(chi_PE / chi0) /
(1e-21 Z'_d) (Eq. e:tau_eff); xi_cr follows Eq. e:cratt.

All six faces are open (no periodic wrap).  Arrays are indexed [k, j, i]
(x fastest in memory, linear index i + nx (j + ny k)).
"""
import numpy as np

from . import constants as C
from . import micro


def f_shld_H2(N_H2, b5=C.B5):
    """Eq. e:fshld_H2_DB."""
    x = N_H2 / 5.0e14
    s = np.sqrt(1.0 + x)
    return 0.965 / (1.0 + x / b5) ** 2 + 0.035 / s * np.exp(-8.5e-4 * s)


def f_shld_C(N_C, N_H2):
    """C self- and H2 cross-shielding -- stand-in table (Sec. 5.1)."""
    lc = np.log10(np.maximum(N_C, 1.0e-300))
    lh = np.log10(np.maximum(N_H2, 1.0e-300))
    return np.exp(micro.LN10 * micro.table2d("cshield", lc, lh, 0))


def g_slab(y):
    """(1 - exp(-y)) / y, the cell average of exp(-tau) over a cell of optical depth y."""
    small = y < 1.0e-4
    ys = np.where(small, 1.0, y)
    return np.where(small, 1.0 - y / 2.0 + y * y / 6.0, -np.expm1(-ys) / ys)


def upstream_columns(q, axis, forward):
    """Exclusive running sum of q along axis, starting from the face the ray enters.

    Accumulated cell by cell (no inclusive-minus-self subtraction), so a small
    upstream column next to a very dense cell keeps its relative precision.
    """
    qq = np.moveaxis(q, axis, 0)
    if not forward:
        qq = qq[::-1]
    out = np.empty_like(qq)
    run = np.zeros_like(qq[0])
    for k in range(qq.shape[0]):
        out[k] = run
        run = run + qq[k]
    if not forward:
        out = out[::-1]
    return np.moveaxis(out, 0, axis)


def columns6(n, xH2, xC, dx, par, xi_in=None):
    """Returns dict chi_PE, chi_LW, chi_H2, chi_C, N_eff, xi (arrays shaped like n [nz, ny, nx]).

    par.cr_mode: 0 -> xi = xi_cr0; 1 -> Eq. e:cratt on N_eff; 2 -> xi_in returned unchanged.
    """
    n = np.asarray(n, dtype=np.float64)
    xH2 = np.asarray(xH2, dtype=np.float64)
    xC = np.zeros_like(n) if xC is None else np.asarray(xC, dtype=np.float64)
    Zd, chi0 = par.Zd, par.chi0
    sPE, sLW = C.SIG_D_PE * Zd, C.SIG_D_LW * Zd
    qH, qH2, qC = n * dx, n * xH2 * dx, n * xC * dx
    gPE, gLW = g_slab(sPE * qH), g_slab(sLW * qH)
    chiPE = np.zeros_like(n)
    chiLW = np.zeros_like(n)
    chiH2 = np.zeros_like(n)
    chiC = np.zeros_like(n)
    for axis in (2, 1, 0):          # x, y, z
        for fwd in (True, False):   # + then - direction
            NH = upstream_columns(qH, axis, fwd)
            NH2m = upstream_columns(qH2, axis, fwd) + 0.5 * qH2
            NCm = upstream_columns(qC, axis, fwd) + 0.5 * qC
            wPE = np.exp(-sPE * NH) * gPE
            wLW = np.exp(-sLW * NH) * gLW
            chiPE += wPE
            chiLW += wLW
            chiH2 += wLW * f_shld_H2(NH2m)
            chiC += wLW * f_shld_C(NCm, NH2m)
    f = chi0 / 6.0
    chiPE, chiLW, chiH2, chiC = f * chiPE, f * chiLW, f * chiH2, f * chiC
    if chi0 > 0.0:
        Neff = -np.log(chiPE / chi0) / (C.SIG_D_NEFF * Zd)
    else:
        Neff = np.zeros_like(n)
    if par.cr_mode == 0:
        xi = np.full_like(n, par.xi_cr0)
    elif par.cr_mode == 1:
        xi = cr_attenuation(Neff, par.xi_cr0)
    else:
        xi = np.asarray(xi_in, dtype=np.float64)
    return dict(chi_PE=chiPE, chi_LW=chiLW, chi_H2=chiH2, chi_C=chiC, N_eff=Neff, xi=xi)


def columns_beam(n, xH2, xC, dx, par):
    """Radiation of a beam of surface intensity chi0 entering through the x = 0 face along +x
    (the plane-parallel slab of Sec. 7.3): the +x ray of columns6 with weight chi0 instead of
    chi0 / 6.  Same cell average and mid-cell shielding columns; N_eff and xi as in columns6."""
    n = np.asarray(n, dtype=np.float64)
    xH2 = np.asarray(xH2, dtype=np.float64)
    xC = np.zeros_like(n) if xC is None else np.asarray(xC, dtype=np.float64)
    Zd, chi0 = par.Zd, par.chi0
    sPE, sLW = C.SIG_D_PE * Zd, C.SIG_D_LW * Zd
    qH, qH2, qC = n * dx, n * xH2 * dx, n * xC * dx
    NH = upstream_columns(qH, 2, True)
    NH2m = upstream_columns(qH2, 2, True) + 0.5 * qH2
    NCm = upstream_columns(qC, 2, True) + 0.5 * qC
    chiPE = chi0 * np.exp(-sPE * NH) * g_slab(sPE * qH)
    chiLW = chi0 * np.exp(-sLW * NH) * g_slab(sLW * qH)
    Neff = -np.log(chiPE / chi0) / (C.SIG_D_NEFF * Zd) if chi0 > 0.0 else np.zeros_like(n)
    if par.cr_mode == 0:
        xi = np.full_like(n, par.xi_cr0)
    else:
        xi = cr_attenuation(Neff, par.xi_cr0)
    return dict(chi_PE=chiPE, chi_LW=chiLW, chi_H2=chiLW * f_shld_H2(NH2m), chi_C=chiLW * f_shld_C(NCm, NH2m),
                N_eff=Neff, xi=xi)


def cr_attenuation(Neff, xi0):
    """Eq. e:cratt: xi0 for N_eff <= N0, xi0 (N_eff / N0)^-1 beyond."""
    return np.where(Neff <= C.N0_CR, xi0, xi0 * C.N0_CR / np.maximum(Neff, C.N0_CR))


def columns6_cells(n, xH2, xC, dx, par, cells):
    """The six-ray result for selected cells only, by direct summation along each ray.

    cells: int array [m, 3] of (k, j, i).  Same definition as columns6, evaluated
    one cell at a time (used to check full-size grids on samples).
    """
    n = np.asarray(n, dtype=np.float64)
    xH2 = np.asarray(xH2, dtype=np.float64)
    xC = np.zeros_like(n) if xC is None else np.asarray(xC, dtype=np.float64)
    Zd, chi0 = par.Zd, par.chi0
    sPE, sLW = C.SIG_D_PE * Zd, C.SIG_D_LW * Zd
    out = {k: np.zeros(len(cells)) for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "N_eff", "xi")}
    for m, (k, j, i) in enumerate(np.asarray(cells)):
        lines = ((n[k, j, :], xH2[k, j, :], xC[k, j, :], i), (n[k, :, i], xH2[k, :, i], xC[k, :, i], j),
                 (n[:, j, i], xH2[:, j, i], xC[:, j, i], k))
        acc = np.zeros(4)
        qH = n[k, j, i] * dx
        qH2 = n[k, j, i] * xH2[k, j, i] * dx
        qC = n[k, j, i] * xC[k, j, i] * dx
        for ln, lx, lc, p in lines:
            for up in (slice(0, p), slice(p + 1, None)):
                NH = np.sum(ln[up] * dx)
                NH2 = np.sum(ln[up] * lx[up] * dx)
                NC = np.sum(ln[up] * lc[up] * dx)
                wPE = np.exp(-sPE * NH) * g_slab(np.array([sPE * qH]))[0]
                wLW = np.exp(-sLW * NH) * g_slab(np.array([sLW * qH]))[0]
                mH2 = NH2 + 0.5 * qH2
                mC = NC + 0.5 * qC
                acc += (wPE, wLW, wLW * f_shld_H2(np.array([mH2]))[0],
                        wLW * f_shld_C(np.array([mC]), np.array([mH2]))[0])
        f = chi0 / 6.0
        out["chi_PE"][m], out["chi_LW"][m], out["chi_H2"][m], out["chi_C"][m] = f * acc
        out["N_eff"][m] = -np.log(out["chi_PE"][m] / chi0) / (C.SIG_D_NEFF * Zd) if chi0 > 0 else 0.0
    if par.cr_mode == 0:
        out["xi"][:] = par.xi_cr0
    elif par.cr_mode == 1:
        out["xi"] = cr_attenuation(out["N_eff"], par.xi_cr0)
    return out
