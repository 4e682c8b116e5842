"""Point-source radiation by long characteristics (test infrastructure).

The ray tracing of Sec. 5.1 deposits, in every cell a ray crosses, the packet's absorbed
luminosity (Eq. e:Erad); with many rays per cell this converges to the radiation of a point
source attenuated along the straight line to the cell.  This module computes that limit at cell
centres, one source and one cell at a time:

* columns N_H, N_H2, N_C from the source to the cell centre: exact integrals of the
  piecewise-constant cell fields along the segment (every crossing of a grid plane found and
  sorted; each interval lies in one cell),
* chi_PE and chi_LW from J = L_FUV / (16 pi^2 r^2) in units of J^D_FUV (Eq. e:chi_FUV), with
  the luminosity split between the bands so that the two normalised intensities are equal,
  attenuated by exp(-sigma_band Z'_d N_H),
* chi_H2 = chi_LW f_shld,H2(N_H2) and chi_C = chi_LW f_shld,C(N_C, N_H2) (Eqs. e:chi_H2,
  e:fshld_H2_DB; shielding columns to the cell centre),
* the LyC photon flux phi = Q exp(-sigma_LyC Z'_d N_H) / (4 pi r^2) inside the Stromgren
  radius R_St = (3 Q / (4 pi alpha_B(1e4 K) nbar^2))^(1/3) of each source, 0 beyond.

Readings (not fixed by the paper): distances below half a cell are raised to half a cell; the
band split and the Stromgren cut follow the point-source workload's recipe.  Positions are in
cm from the grid corner; fields are indexed [k, j, i] (z, y, x), cell (i, j, k) spans
[i dx, (i + 1) dx) and so on.
"""
import numpy as np

from . import constants as C
from . import micro
from .columns import f_shld_C, f_shld_H2

L_SUN = 3.828e33  # erg s^-1, nominal solar luminosity


def segment_columns(fields, dx, p0, p1):
    """Integrals of the cell fields along p0 -> p1 (cm): every crossing with a grid plane,
    sorted; each interval between consecutive crossings lies in one cell, found from its
    midpoint, and contributes field x length."""
    p0 = np.asarray(p0, dtype=np.float64)
    p1 = np.asarray(p1, dtype=np.float64)
    d = p1 - p0
    L = float(np.sqrt(np.sum(d * d)))
    nz, ny, nx = fields[0].shape
    dims = (nx, ny, nz)
    ts = [0.0, 1.0]
    for a in range(3):
        if d[a] == 0.0:
            continue
        lo, hi = sorted((p0[a], p1[a]))
        for m in range(int(np.floor(lo / dx)) + 1, int(np.ceil(hi / dx))):
            t = (m * dx - p0[a]) / d[a]
            if 0.0 < t < 1.0:
                ts.append(t)
    ts = np.unique(np.array(ts))
    out = np.zeros(len(fields))
    for ta, tb in zip(ts[:-1], ts[1:]):
        if tb <= ta:
            continue
        mid = p0 + d * (0.5 * (ta + tb))
        idx = [min(max(int(np.floor(mid[a] / dx)), 0), dims[a] - 1) for a in range(3)]
        seg = (tb - ta) * L
        for f, field in enumerate(fields):
            out[f] += field[idx[2], idx[1], idx[0]] * seg
    return out


def stromgren_radius(Q, nbar=1.0):
    """Radius of the ionised sphere of a source of Q ionising photons per second in gas of mean
    density nbar, case-B recombination at 1e4 K."""
    return (3.0 * Q / (4.0 * np.pi * micro.alpha_B(1.0e4) * nbar * nbar)) ** (1.0 / 3.0)


def point_source_cells(n, xH2, xC, dx, sources, par, cells):
    """Radiation from the sources at the centres of the given cells.

    sources: array [m, 5] of (x, y, z, Q, L_FUV) in cm, s^-1, erg s^-1.
    cells: int array [k, 3] of (k, j, i).  Returns dict chi_PE, chi_LW, chi_H2, chi_C, phi."""
    n = np.asarray(n, dtype=np.float64)
    xH2 = np.asarray(xH2, dtype=np.float64)
    xC = np.zeros_like(n) if xC is None else np.asarray(xC, dtype=np.float64)
    fields = (n, n * xH2, n * xC)
    Zd = par.Zd
    out = {k: np.zeros(len(cells)) for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "phi")}
    for s in np.asarray(sources, dtype=np.float64):
        pos, Q, L = s[:3], s[3], s[4]
        Rst = stromgren_radius(Q)
        for m, (k, j, i) in enumerate(np.asarray(cells)):
            c = np.array([(i + 0.5) * dx, (j + 0.5) * dx, (k + 0.5) * dx])
            r = max(float(np.sqrt(np.sum((c - pos) ** 2))), 0.5 * dx)
            NH, NH2, NC = segment_columns(fields, dx, pos, c)
            chi = L / (16.0 * np.pi ** 2 * r * r * C.J_FUV)
            wPE = chi * np.exp(-C.SIG_D_PE * Zd * NH)
            wLW = chi * np.exp(-C.SIG_D_LW * Zd * NH)
            out["chi_PE"][m] += wPE
            out["chi_LW"][m] += wLW
            out["chi_H2"][m] += wLW * f_shld_H2(NH2)
            out["chi_C"][m] += wLW * f_shld_C(NC, NH2)
            if r < Rst:
                out["phi"][m] += Q * np.exp(-C.SIG_D_LYC * Zd * NH) / (4.0 * np.pi * r * r)
    return out


def point_source_maps(n, xH2, xC, dx, sources, par):
    """point_source_cells for every cell of the grid; arrays shaped like n."""
    shape = np.shape(n)
    cells = np.stack(np.unravel_index(np.arange(np.size(n)), shape), 1)
    r = point_source_cells(n, xH2, xC, dx, sources, par, cells)
    return {k: v.reshape(shape) for k, v in r.items()}
