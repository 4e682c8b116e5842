"""Adaptive ray tracing of point-source radiation (Sec. 5.1), FP64 -- test infrastructure.

Each source emits 12 x 4^l0 photon packets along the HEALPix directions of level l0 (Gorski
et al. 2005; nested numbering, so the four children of pixel p at level l are 4p .. 4p+3 at
level l+1).  A packet walks cell by cell.  In a cell crossed over a length ds, band j has the
opacity alpha_j and the packet deposits the absorbed luminosity

    dL_j = L_in,j (1 - exp(-alpha_j ds)),   L_in,j = L_src,j exp(-tau_j) / N_ray(l),

tau_j the optical depth from the source to the entry face; the cell's energy density is the
sum of dL_j / (alpha_j dV c) over packets (Eq. e:Erad), so J_j = sum dL_j / alpha_j / (4 pi dV).
The LW band also carries the weight f_shld,H2(N_H2) and f_shld,C(N_C, N_H2) with the columns
from the source to the middle of the segment (Eq. e:Erad_H2 and the text around it).  Before a
packet enters a cell at distance r it is

* dropped if tau_j > tau_max in every band (default 30),
* split into its four children, which start at the same distance r along their own directions
  and carry the parent's columns, if N_ray(l) dx^2 / (4 pi r^2) < Phi_c (rays per cell per
  source; default 4),

and it is lost through the domain boundary (all six faces open).  A piece that would start
within 1e-10 cells of the boundary is not entered: where a plane crossing meets the domain
exit (up to rounding) the packet leaves rather than splitting on the boundary.

Bands and opacities (Sec. 5.1): PE and LW by dust only, alpha = n sigma_d Z'_d; LyC by H, H2
and dust, alpha = n (x_HI sigma_pi,H + x_H2 sigma_pi,H2 + Z'_d sigma_d,LyC), x_HI = 1 - 2 x_H2
- x_H+.  PE and LW packets carry L_FUV each and are normalised by J^D_FUV, so both bands see
the same unattenuated intensity (the point-source recipe of the long-characteristics module);
LyC packets carry Q photons s^-1 and give the photon flux phi = sum dQ / alpha_LyC / dV.

With flux=True the trace also returns the flux vector of each band, the same sums with every
deposit times the packet's direction n (Eq. e:Frad): F_j = sum dL_j n / alpha_j / dV.  PE and
LW are given as band energy fluxes (erg cm^-2 s^-1): a packet's FUV luminosity is shared
between them as J^D_PE : J^D_LW, the shares of the Draine field, so that F_PE + F_LW is the
FUV flux; LyC as a photon flux (photons cm^-2 s^-1).  radiation_force turns them into the
force per volume on the gas-dust mixture (Sec. 6.2) with the grain-destruction switch.

The HEALPix pixel centres are taken from the continuous inverse HEALPix projection
(Calabretta & Roukema 2007) evaluated at the centre of each base-pixel sub-square, not from
the ring-index formulas.

A packet's path is cut at every grid-plane crossing between its start and the domain exit;
each piece lies in one cell, found from its midpoint.  The crossings are sorted per packet.
Positions are in cm from the grid corner; arrays are indexed [k, j, i] (z, y, x).
"""
import numpy as np

from . import constants as C
from .columns import f_shld_C, f_shld_H2


def _deinterleave(ipf, nbits):
    """Split the interleaved bits of the in-face index: x from the even bits, y from the odd."""
    ix = np.zeros_like(ipf)
    iy = np.zeros_like(ipf)
    for b in range(nbits):
        ix |= ((ipf >> (2 * b)) & 1) << b
        iy |= ((ipf >> (2 * b + 1)) & 1) << b
    return ix, iy


def healpix_dirs(level, pix=None):
    """Unit vectors [len(pix), 3] of the HEALPix pixel centres of a level (nested numbering;
    all 12 4^level pixels when pix is None).

    Base pixel f is a square turned by 45 degrees in the projection plane (x_s, y_s), centred
    at (pi/4 + f pi/2, pi/4) for f < 4, ((f - 4) pi/2, 0) for 4 <= f < 8 and
    (pi/4 + (f - 8) pi/2, -pi/4) beyond, with half-diagonal pi/4; sub-pixel (ix, iy) has its
    centre at u = (ix + 1/2)/nside, v = (iy + 1/2)/nside along the two sides, x growing to the
    east and y to the west of the north corner.  The inverse projection: z = 8 y_s / (3 pi),
    phi = x_s where |y_s| <= pi/4; otherwise sigma = 2 - 4 |y_s| / pi,
    z = sign(y_s) (1 - sigma^2 / 3), phi = x_f + (x_s - x_f) / sigma with x_f the centre of the
    polar facet (a multiple of pi/2 plus pi/4) that holds x_s."""
    ns = 1 << level
    p = np.arange(12 * ns * ns, dtype=np.int64) if pix is None else np.atleast_1d(np.asarray(pix, dtype=np.int64))
    f = p // (ns * ns)
    ix, iy = _deinterleave(p % (ns * ns), level)
    q = np.pi / 4.0
    xc = np.where(f < 4, q + f * 2 * q, np.where(f < 8, (f - 4) * 2 * q, q + (f - 8) * 2 * q))
    yc = np.where(f < 4, q, np.where(f < 8, 0.0, -q))
    u = (ix + 0.5) / ns
    v = (iy + 0.5) / ns
    xs = xc + (u - v) * q
    ys = yc + (u + v - 1.0) * q
    eq = np.abs(ys) <= q
    sig = np.where(eq, 1.0, 2.0 - np.abs(ys) / q)
    z = np.where(eq, ys / (3.0 * np.pi / 8.0), np.sign(ys) * (1.0 - sig * sig / 3.0))
    xf = (np.floor(xs / (2 * q)) + 0.5) * 2 * q
    phi = np.where(eq, xs, xf + (xs - xf) / sig)
    s = np.sqrt(np.maximum(1.0 - z * z, 0.0))
    u = np.stack([s * np.cos(phi), s * np.sin(phi), z], 1)
    # components that vanish exactly (directions in a coordinate plane) are zero, not the
    # 1e-17 left by cos(pi/2); the smallest true component at level 13 is about 1e-9
    u[np.abs(u) < 1e-12] = 0.0
    return u


def _g(y):
    """(1 - exp(-y)) / y, 1 at y = 0."""
    y = np.asarray(y, dtype=np.float64)
    out = np.ones_like(y)
    m = y > 0.0
    out[m] = -np.expm1(-y[m]) / y[m]
    return out


class _Grid:
    """Opacities and the per-cell quantities a packet needs, flattened (x fastest)."""

    def __init__(self, n, xH2, xHp, xC, dx, par):
        n = np.asarray(n, dtype=np.float64)
        self.shape = n.shape
        nz, ny, nx = n.shape
        self.nx, self.ny = nx, ny
        xH2 = np.asarray(xH2, dtype=np.float64)
        xHp = np.asarray(xHp, dtype=np.float64)
        xC = np.zeros_like(n) if xC is None else np.asarray(xC, dtype=np.float64)
        Zd = par.Zd
        self.sPE, self.sLW = C.SIG_D_PE * Zd, C.SIG_D_LW * Zd
        xHI = np.maximum(1.0 - 2.0 * xH2 - xHp, 0.0)
        self.aPE, self.aLW = (self.sPE * n).ravel(), (self.sLW * n).ravel()
        self.aLyC = (n * (xHI * C.SIGMA_PI_H + xH2 * C.SIGMA_PI_H2 + Zd * C.SIG_D_LYC)).ravel()
        self.nH2, self.nC, self.nf = (n * xH2).ravel(), (n * xC).ravel(), n.ravel()
        self.dx = dx
        self.dV = dx ** 3
        self.fuv_norm = 1.0 / (4.0 * np.pi * self.dV * C.J_FUV)
        self.box = np.array([nx * dx, ny * dx, nz * dx])
        self.dims = np.array([nx, ny, nz])


EXIT_TOL = 1e-10  # cells


def _walk(G, s, lev, pix, state, rays_per_cell, tau_max, max_level):
    """One packet from its start to where it ends or splits.

    state: (r0, N_H, N_H2, N_C, tau_LyC) at the start.  Returns (reason, segs, end) with reason
    'exit', 'drop' or 'split'; segs the pieces it deposits in (cell, ds, columns at the entry
    face); end the state where it stopped (for 'split': where its children start)."""
    r0, NH, NH2, NC, tLyC = state
    u = healpix_dirs(lev, pix)[0]
    nray = 12.0 * 4.0 ** lev
    dx, box = G.dx, G.box
    with np.errstate(divide="ignore"):
        bound = np.where(u > 0, box, 0.0)
        rb = np.where(u != 0, (bound - s) / np.where(u != 0, u, 1.0), np.inf)
    r_exit = float(np.min(rb))
    p0 = s + r0 * u
    if np.any(p0 < 0.0) or np.any(p0 >= box) or r0 >= r_exit - EXIT_TOL * dx:
        return "exit", None, state
    cuts = [r0, r_exit]
    for a in range(3):
        if u[a] == 0.0:
            continue
        lo, hi = sorted((p0[a], s[a] + r_exit * u[a]))
        m = np.arange(int(np.floor(lo / dx)) + 1, int(np.ceil(hi / dx)))
        rm = (m * dx - s[a]) / u[a]
        cuts.extend(rm[(rm > r0) & (rm < r_exit)].tolist())
    cuts = np.unique(np.array(cuts))
    ra, rbnd = cuts[:-1], cuts[1:]
    # a piece that would start within EXIT_TOL cells of the exit is not entered: the packet
    # has left (a plane crossing that meets the exit up to rounding is not a cell entry)
    keep = ra < r_exit - EXIT_TOL * dx
    ra, rbnd = ra[keep], rbnd[keep]
    mid = s[None, :] + (0.5 * (ra + rbnd))[:, None] * u[None, :]
    ijk = np.clip(np.floor(mid / dx).astype(np.int64), 0, G.dims - 1)
    cell = ijk[:, 0] + G.nx * (ijk[:, 1] + G.ny * ijk[:, 2])
    ds = rbnd - ra
    # columns at each entry face (running sums from the packet's start)
    NH_in = NH + np.concatenate(([0.0], np.cumsum(G.nf[cell] * ds)))
    NH2_in = NH2 + np.concatenate(([0.0], np.cumsum(G.nH2[cell] * ds)))
    NC_in = NC + np.concatenate(([0.0], np.cumsum(G.nC[cell] * ds)))
    tL_in = tLyC + np.concatenate(([0.0], np.cumsum(G.aLyC[cell] * ds)))
    drop = (G.sPE * NH_in[:-1] > tau_max) & (G.sLW * NH_in[:-1] > tau_max) & (tL_in[:-1] > tau_max)
    if lev < max_level:
        with np.errstate(divide="ignore"):
            split = nray * dx * dx / (4.0 * np.pi * ra * ra) < rays_per_cell
    else:
        split = np.zeros(len(ra), dtype=bool)
    stop = np.nonzero(drop | split)[0]
    k = int(stop[0]) if stop.size else len(ra)
    segs = (cell[:k], ds[:k], NH_in[:k], NH2_in[:k], NC_in[:k], tL_in[:k])
    reason = "exit" if k == len(ra) else ("drop" if drop[k] else "split")
    r_end = r_exit if k == len(ra) else float(ra[k])
    end = (r_end, float(NH_in[k]), float(NH2_in[k]), float(NC_in[k]), float(tL_in[k]))
    return reason, segs, end


def _deposits(G, segs, lev, Lband):
    """Per-piece additions to chi_PE, chi_LW, chi_H2, chi_C and phi."""
    c, d, NH, NH2, NC, tL = segs
    nray = 12.0 * 4.0 ** lev
    att = np.exp(-np.stack([G.sPE * NH, G.sLW * NH, tL], 1))
    Lin = Lband[None, :] * att / nray
    wPE = Lin[:, 0] * d * _g(G.aPE[c] * d) * G.fuv_norm
    wLW = Lin[:, 1] * d * _g(G.aLW[c] * d) * G.fuv_norm
    wLyC = Lin[:, 2] * d * _g(G.aLyC[c] * d) / G.dV
    mH2 = NH2 + 0.5 * G.nH2[c] * d
    mC = NC + 0.5 * G.nC[c] * d
    return c, (wPE, wLW, wLW * f_shld_H2(mH2), wLW * f_shld_C(mC, mH2), wLyC)


FIELDS = ("chi_PE", "chi_LW", "chi_H2", "chi_C", "phi")
# flux components, in the order of the 'flux' output: band-major, then x, y, z
FLUX = ("F_PE_x", "F_PE_y", "F_PE_z", "F_LW_x", "F_LW_y", "F_LW_z", "F_LyC_x", "F_LyC_y", "F_LyC_z")


def _flux_deposits(w, u):
    """Flux additions [9, pieces] of one packet with direction u from its chi_PE, chi_LW and
    phi additions w (Eq. e:Frad): chi deposits carry 1 / (4 pi J^D_FUV), so 4 pi J^D_PE and
    4 pi J^D_LW turn them into the bands' energy fluxes; phi is already a photon flux."""
    wPE, wLW, _, _, wLyC = w
    out = []
    for wb, k in ((wPE, 4.0 * np.pi * C.J_PE), (wLW, 4.0 * np.pi * C.J_LW), (wLyC, 1.0)):
        out.extend(k * wb * u[a] for a in range(3))
    return out


def ray_trace(n, xH2, xHp, xC, dx, sources, par, level0=4, rays_per_cell=4.0, tau_max=30.0,
              max_level=13, flux=False):
    """Radiation of the point sources on the grid.

    n, xH2, xHp, xC: arrays [nz, ny, nx] (xC may be None = 0).  sources: [m, 5] of
    (x, y, z, Q, L_FUV) in cm, s^-1, erg s^-1.  Returns dict chi_PE, chi_LW, chi_H2, chi_C, phi
    (arrays shaped like n) and budget [m, 6]: luminosity lost through the boundary in PE, LW,
    LyC, then luminosity dropped at tau > tau_max in the same bands (erg s^-1, erg s^-1,
    photons s^-1); with flux=True also 'flux' [9, nz, ny, nx] in the order of FLUX."""
    G = _Grid(n, xH2, xHp, xC, dx, par)
    keys = FIELDS + (FLUX if flux else ())
    acc = {k: np.zeros(int(np.prod(G.shape))) for k in keys}
    srcs = np.atleast_2d(np.asarray(sources, dtype=np.float64))
    budget = np.zeros((len(srcs), 6))
    for si, (sx, sy, sz, Q, L) in enumerate(srcs):
        s = np.array([sx, sy, sz])
        Lband = np.array([L, L, Q])
        stack = [(level0, p, (0.0, 0.0, 0.0, 0.0, 0.0)) for p in range(12 * 4 ** level0)]
        while stack:
            lev, pix, state = stack.pop()
            reason, segs, end = _walk(G, s, lev, pix, state, rays_per_cell, tau_max, max_level)
            if segs is not None:
                c, w = _deposits(G, segs, lev, Lband)
                if flux:
                    w = tuple(w) + tuple(_flux_deposits(w, healpix_dirs(lev, pix)[0]))
                for k, v in zip(keys, w):
                    np.add.at(acc[k], c, v)
            if reason == "split":
                stack.extend((lev + 1, 4 * pix + ch, end) for ch in range(4))
            else:
                _, NH, _, _, tL = end
                att = np.exp(-np.array([G.sPE * NH, G.sLW * NH, tL]))
                o = 0 if reason == "exit" else 3
                budget[si, o:o + 3] += Lband * att / (12.0 * 4.0 ** lev)
    out = {k: acc[k].reshape(G.shape) for k in FIELDS}
    if flux:
        out["flux"] = np.stack([acc[k].reshape(G.shape) for k in FLUX])
    out["budget"] = budget
    return out


# Largest angle between a pixel centre and the centre of any of its descendants, in units of
# the pixel's mean size sqrt(4 pi / N_pix): about 0.97 measured over levels 0-5 and four
# levels of descendants; 2 leaves a wide margin (a larger bound only adds candidates).
DESC_RADIUS = 2.0


def ray_trace_cells(n, xH2, xHp, xC, dx, sources, par, cells, level0=4, rays_per_cell=4.0,
                    tau_max=30.0, max_level=13, flux=False):
    """ray_trace at selected cells only: dict of arrays [len(cells)] (and 'flux' [9, len(cells)]
    with flux=True).

    Packet trees of different level-l0 pixels are independent, so a cell's value is the sum
    over the packets whose lines cross it.  For each cell and source the candidates are the
    (level, pixel) pairs whose direction passes within the cell's circumscribed sphere and
    whose level can be active at the cell's distance (a packet of level l lives between
    R_(l-1) and R_l + sqrt(3) cells, R_l^2 = N_pix(l) / (4 pi Phi_c)); the pixel tree is
    searched from level l0 down, pruning with DESC_RADIUS.  Each candidate is reached by
    walking its chain of ancestors from the source (memoised), and only its pieces inside the
    cell are kept.  cells: int array [k, 3] of (k, j, i)."""
    G = _Grid(n, xH2, xHp, xC, dx, par)
    cells = np.atleast_2d(np.asarray(cells, dtype=np.int64))
    keys = FIELDS + (FLUX if flux else ())
    out = {k: np.zeros(len(cells)) for k in keys}
    srcs = np.atleast_2d(np.asarray(sources, dtype=np.float64))
    rho = 0.5 * np.sqrt(3.0)  # circumscribed radius of a cell, cell units
    R = [np.sqrt(12.0 * 4.0 ** l / (4.0 * np.pi * rays_per_cell)) for l in range(max_level + 2)]
    lo = [0.0 if l == level0 else R[l - 1] for l in range(max_level + 1)]
    hi = [np.inf if l == max_level else R[l] + np.sqrt(3.0) for l in range(max_level + 1)]
    for si, (sx, sy, sz, Q, L) in enumerate(srcs):
        s = np.array([sx, sy, sz])
        Lband = np.array([L, L, Q])
        memo = {}

        def chain(lev, pix):
            """Walk result of packet (lev, pix), or None if it never exists."""
            key = (lev, pix)
            if key not in memo:
                if lev == level0:
                    start = (0.0, 0.0, 0.0, 0.0, 0.0)
                else:
                    parent = chain(lev - 1, pix >> 2)
                    if parent is None or parent[0] != "split":
                        memo[key] = None
                        return None
                    start = parent[2]
                memo[key] = _walk(G, s, lev, pix, start, rays_per_cell, tau_max, max_level)
            return memo[key]

        for ci, (k, j, i) in enumerate(cells):
            cen = (np.array([i, j, k], dtype=np.float64) + 0.5) * dx
            v = cen - s
            d = float(np.sqrt(np.sum(v * v))) / dx
            vhat = v / (d * dx) if d > 0 else np.array([0.0, 0.0, 1.0])
            half = np.arcsin(rho / d) if d > rho else np.pi
            target = int(i + G.nx * (j + G.ny * k))
            pix = np.arange(12 * 4 ** level0, dtype=np.int64)
            lev = level0
            while pix.size:
                ang = np.arccos(np.clip(healpix_dirs(lev, pix) @ vhat, -1.0, 1.0))
                keep = ang <= half + DESC_RADIUS * np.sqrt(4.0 * np.pi / (12.0 * 4.0 ** lev))
                pix, ang = pix[keep], ang[keep]
                if lo[lev] <= d + rho and hi[lev] >= d - rho:
                    for p in pix[ang <= half]:
                        w = chain(lev, int(p))
                        if w is not None and w[1] is not None:
                            c, dep = _deposits(G, w[1], lev, Lband)
                            m = c == target
                            if m.any():
                                if flux:
                                    dep = tuple(dep) + tuple(_flux_deposits(dep, healpix_dirs(lev, int(p))[0]))
                                for key, val in zip(keys, dep):
                                    out[key][ci] += float(np.sum(val[m]))
                if lev >= max_level or R[lev] > d + rho:
                    break
                pix = (4 * pix[:, None] + np.arange(4)[None, :]).ravel()
                lev += 1
    if flux:
        out["flux"] = np.stack([out.pop(k) for k in FLUX])
    return out


def absorbed(out, n, xH2, xHp, dx, par):
    """Luminosity absorbed in the grid per band (PE, LW in erg s^-1, LyC in photons s^-1),
    recovered from the output fields: alpha_j J_j 4 pi dV summed over cells."""
    n = np.asarray(n, dtype=np.float64)
    Zd = par.Zd
    xHI = np.maximum(1.0 - 2.0 * np.asarray(xH2) - np.asarray(xHp), 0.0)
    aLyC = n * (xHI * C.SIGMA_PI_H + np.asarray(xH2) * C.SIGMA_PI_H2 + Zd * C.SIG_D_LYC)
    dV = dx ** 3
    k = 4.0 * np.pi * dV * C.J_FUV
    return np.array([np.sum(C.SIG_D_PE * Zd * n * out["chi_PE"]) * k,
                     np.sum(C.SIG_D_LW * Zd * n * out["chi_LW"]) * k,
                     np.sum(aLyC * out["phi"]) * dV])


# Grain destruction (appendix on grain destruction): grains are taken as destroyed, and the
# radiation force on them omitted, where T exceeds 1e6 K (thermal sputtering) or where the
# radiation pressure exceeds 50 times the gas pressure (non-thermal sputtering: the terminal
# drift then lies on the branch s ~ sqrt(P_rad / P) >~ sqrt(50)); P_rad = |F| / c with F the
# total flux of the traced bands and P = 2 n k_B T.
T_DESTROY = 1.0e6
PRAD_RATIO_MAX = 50.0


def radiation_force(n, T, xH2, xHp, flux, par, T_destroy=T_DESTROY, prad_ratio_max=PRAD_RATIO_MAX,
                    dt=0.0, mom=None, etot=None):
    """Radiation force per volume on the gas-dust mixture (Sec. 6.2): the sum over bands of
    alpha_j F_j / c, alpha_j the band's opacity (PE, LW: dust; LyC: dust, H and H2; the same
    opacities as the trace), with the LyC photon flux carrying h nu_LyC per photon.  Where the
    grains are destroyed the dust part of every band is dropped and only the photoionisation
    part of LyC remains.

    n, T, xH2, xHp: arrays of any shape; flux: [9, *shape] as ray_trace returns it.  Returns
    dict f [3, *shape] (dyn cm^-3) and dust_off (bool).  With mom ([3, *shape] momentum
    density, g cm^-2 s^-1) the source-term update of Sec. 6.2 is also made on copies: mom + f dt
    and, with etot (total energy density, erg cm^-3), etot plus the change of rho v^2 / 2 at
    fixed rho = mu_H m_H n; returned as 'mom' and 'etot'."""
    n = np.asarray(n, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    xH2 = np.asarray(xH2, dtype=np.float64)
    xHp = np.asarray(xHp, dtype=np.float64)
    F = np.asarray(flux, dtype=np.float64).reshape((3, 3) + n.shape)
    F_PE, F_LW, F_LyC = F[0], F[1], C.HNU_LYC * F[2]  # energy fluxes
    Ftot = F_PE + F_LW + F_LyC
    prad = np.sqrt(np.sum(Ftot * Ftot, 0)) / C.C_LIGHT
    P = 2.0 * n * C.K_B * T
    off = (T > T_destroy) | (prad > prad_ratio_max * P)
    keep = np.where(off, 0.0, 1.0)
    Zd = par.Zd
    xHI = np.maximum(1.0 - 2.0 * xH2 - xHp, 0.0)
    a_gas = n * (xHI * C.SIGMA_PI_H + xH2 * C.SIGMA_PI_H2)
    f = (keep * n * Zd * (C.SIG_D_PE * F_PE + C.SIG_D_LW * F_LW + C.SIG_D_LYC * F_LyC)
         + a_gas * F_LyC) / C.C_LIGHT
    out = {"f": f, "dust_off": off}
    if mom is not None:
        p0 = np.asarray(mom, dtype=np.float64)
        p1 = p0 + f * dt
        out["mom"] = p1
        if etot is not None:
            rho = par.muH * C.M_H * n
            with np.errstate(divide="ignore", invalid="ignore"):
                dk = np.where(rho > 0.0, (np.sum(p1 * p1, 0) - np.sum(p0 * p0, 0)) / (2.0 * rho), 0.0)
            out["etot"] = np.asarray(etot, dtype=np.float64) + dk
    return out
