"""Pins of the adaptive ray-tracing oracle (Sec. 5.1) against facts it does not compute itself:
the HEALPix ring formulas of Gorski et al. (2005), photon conservation, the exact mean path
to the domain boundary in an empty box, the invariance of the result under the injection
level in a uniform medium, and the long-characteristics limit (itself pinned elsewhere)."""
import numpy as np
import pytest
from scipy import integrate

from oracle import art, sources
from oracle import constants as C
from oracle.constants import Params

pytestmark = [pytest.mark.slow, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

DX = C.PC


def _ring_table(level):
    """(z, phi) of every pixel centre from the ring formulas: polar ring j < nside holds 4j
    pixels at z = 1 - j^2 / (3 nside^2), phi = (k - 1/2) pi / (2j); belt ring j in
    [nside, 3 nside] holds 4 nside pixels at z = (4 nside - 2j) / (3 nside),
    phi = (k - s/2) pi / (2 nside) with s = (j - nside + 1) mod 2; the south mirrors the north."""
    ns = 1 << level
    out = []
    for j in range(1, 4 * ns):
        if j < ns or j > 3 * ns:
            jj = j if j < ns else 4 * ns - j
            z = 1.0 - jj * jj / (3.0 * ns * ns)
            z = z if j < ns else -z
            out += [(z, (k - 0.5) * np.pi / (2 * jj)) for k in range(1, 4 * jj + 1)]
        else:
            s = (j - ns + 1) % 2
            out += [((4 * ns - 2 * j) / (3.0 * ns), (k - 0.5 * s) * np.pi / (2 * ns)) for k in range(1, 4 * ns + 1)]
    return np.array(out)


def test_healpix_base_pixels():
    u = art.healpix_dirs(0)
    q = np.pi / 4
    phi = [q + f * 2 * q for f in range(4)] + [f * 2 * q for f in range(4)] + [q + f * 2 * q for f in range(4)]
    z = [2 / 3] * 4 + [0.0] * 4 + [-2 / 3] * 4
    s = np.sqrt(1 - np.array(z) ** 2)
    ref = np.stack([s * np.cos(phi), s * np.sin(phi), z], 1)
    np.testing.assert_allclose(u, ref, atol=1e-15)


@pytest.mark.parametrize("level", [1, 2, 3, 4])
def test_healpix_centres_follow_the_ring_formulas(level):
    u = art.healpix_dirs(level)
    assert u.shape == (12 * 4 ** level, 3)
    np.testing.assert_allclose(np.sum(u * u, 1), 1.0, atol=1e-14)
    got = np.stack([u[:, 2], np.mod(np.arctan2(u[:, 1], u[:, 0]), 2 * np.pi)], 1)
    ref = _ring_table(level)
    ref[:, 1] = np.mod(ref[:, 1], 2 * np.pi)
    # the same set of points: sort both by (z, phi)
    g = got[np.lexsort((np.round(got[:, 1], 9), np.round(got[:, 0], 9)))]
    r = ref[np.lexsort((np.round(ref[:, 1], 9), np.round(ref[:, 0], 9)))]
    np.testing.assert_allclose(g, r, atol=1e-11)
    # equal areas: a quantile of z matches the area fraction above it
    ns = 1 << level
    for z0 in (-0.9, -0.3, 0.2, 0.7):
        frac = np.mean(u[:, 2] > z0)
        assert abs(frac - (1 - z0) / 2) < 1.0 / ns


def test_healpix_descendants_stay_near_their_ancestor():
    """The nesting (children of p are 4p .. 4p+3) and the search radius of the per-cell mode."""
    worst = 0.0
    for level in range(0, 5):
        P = art.healpix_dirs(level)
        size = np.sqrt(4 * np.pi / len(P))
        for k in (1, 2, 3):
            D = art.healpix_dirs(level + k)
            anc = np.arange(len(D)) >> (2 * k)
            ang = np.arccos(np.clip(np.sum(D * P[anc], 1), -1, 1))
            worst = max(worst, ang.max() / size)
            # a child is closer to its own parent's centre than the pixel size
            assert ang.max() < size
    assert worst < art.DESC_RADIUS / 1.5


def _medium(shape, seed, dense=True):
    rng = np.random.default_rng(seed)
    n = 10 ** rng.uniform(-1, 1.5, shape)
    if dense:
        n[:, :, shape[2] * 2 // 3:] *= 300.0
    xH2 = 0.5 * rng.uniform(0, 0.8, shape)
    xHp = rng.uniform(0, 1, shape) * (1 - 2 * xH2)
    xC = rng.uniform(0, 1e-4, shape)
    return n, xH2, xHp, xC


SRC = np.array([[5.3 * DX, 6.1 * DX, 5.7 * DX, 1e49, 1e5 * sources.L_SUN],
                [0.2 * DX, 9.9 * DX, 3.4 * DX, 1e48, 3e4 * sources.L_SUN]])


@pytest.mark.parametrize("kw", [dict(), dict(level0=1, tau_max=3.0, max_level=4)])
def test_photon_conservation(kw):
    """Every packet's luminosity ends absorbed in a cell, lost through a face or dropped: the
    absorbed part recovered from the fields (alpha J 4 pi dV), plus the budget, is the
    sources' total in each band."""
    par = Params()
    n, xH2, xHp, xC = _medium((10, 11, 12), 1)
    out = art.ray_trace(n, xH2, xHp, xC, DX, SRC, par, **kw)
    ab = art.absorbed(out, n, xH2, xHp, DX, par)
    L = np.array([SRC[:, 4].sum(), SRC[:, 4].sum(), SRC[:, 3].sum()])
    b = out["budget"]
    np.testing.assert_allclose(ab + b[:, :3].sum(0) + b[:, 3:].sum(0), L, rtol=1e-12)
    assert np.all(ab > 0) and np.all(b[:, :3].sum(0) > 0)
    if kw:
        assert b[:, 3].sum() > 0  # tau_max = 3 drops packets in the dense part


def _mean_exit(s, box):
    """Mean over directions of the distance from s to the boundary of [0, box]: each face seen
    from s contributes (1/4 pi) int h / rho^2 dA (h the distance to its plane)."""
    tot = 0.0
    for a in range(3):
        b, c = [q for q in range(3) if q != a]
        for h in (s[a], box[a] - s[a]):
            v, _ = integrate.dblquad(lambda y, x: h / (h * h + x * x + y * y), -s[b], box[b] - s[b],
                                     -s[c], box[c] - s[c], epsabs=1e-13, epsrel=1e-11)
            tot += v
    return tot / (4 * np.pi)


@pytest.mark.parametrize("level0,pos,tol", [(4, [3.3, 7.1, 4.6], 1e-3), (4, [0.4, 0.7, 9.2], 2e-3),
                                            (2, [3.3, 7.1, 4.6], 1e-3), (2, [0.4, 0.7, 9.2], 1e-2)])
def test_empty_box_mean_path(level0, pos, tol):
    """With no opacity every packet deposits L ds / N_ray; split packets hand their path on to
    their children, so the total is L times the HEALPix average of the distance to the
    boundary over the finest directions -- a quadrature of the exact mean."""
    shape = (10, 12, 11)
    box = np.array([11.0, 12.0, 10.0])
    s = np.array(pos)
    z = np.zeros(shape)
    out = art.ray_trace(z, z, z, None, DX, [[*(s * DX), 1e49, 1e38]], Params(), level0=level0)
    tot = out["chi_PE"].sum() * 4 * np.pi * DX ** 3 * C.J_FUV / 1e38 / DX
    totq = out["phi"].sum() * DX ** 3 / 1e49 / DX
    ref = _mean_exit(s, box)
    assert abs(tot / ref - 1) < tol and abs(totq / ref - 1) < tol
    np.testing.assert_allclose(out["budget"][0, :3], [1e38, 1e38, 1e49], rtol=1e-12)


def test_injection_level_invariance_in_a_uniform_medium():
    """Packets lie on radial lines and columns in a uniform medium depend on distance only, so
    beyond the level-4 split radius injecting at level 2 or 4 gives the same packets."""
    par = Params()
    shape = (14, 14, 14)
    n, xH2, xHp = np.full(shape, 4.0), np.full(shape, 0.2), np.full(shape, 0.1)
    xC = np.full(shape, 5e-5)
    s = np.array([6.6, 7.3, 6.9])
    src = [[*(s * DX), 1e49, 1e5 * sources.L_SUN]]
    a = art.ray_trace(n, xH2, xHp, xC, DX, src, par, level0=2)
    b = art.ray_trace(n, xH2, xHp, xC, DX, src, par, level0=4)
    kk, jj, ii = np.indices(shape)
    lo = [np.clip(s[q], g, g + 1) for q, g in enumerate((ii, jj, kk))]
    dmin = np.sqrt((lo[0] - s[0]) ** 2 + (lo[1] - s[1]) ** 2 + (lo[2] - s[2]) ** 2)
    R4 = np.sqrt(12 * 4 ** 4 / (4 * np.pi * 4.0))
    m = dmin > R4 + 0.01
    assert m.sum() > 100
    for k in art.FIELDS:
        np.testing.assert_allclose(a[k][m], b[k][m], rtol=1e-11, atol=0)
    np.testing.assert_allclose(a["budget"], b["budget"], rtol=1e-11)


def test_long_characteristics_limit():
    """Averaged over shells the packets reproduce the attenuated, shielded radiation of the
    source at cell centres (the long-characteristics oracle): rays per cell make a cell's
    own value noisy (about 10%), a shell's sum is within 1-2% beyond three cells."""
    par = Params()
    shape = (16, 16, 16)
    n, xH2, xHp = np.full(shape, 30.0), np.full(shape, 0.2), np.zeros(shape)
    s = np.array([8.3, 7.6, 8.1]) * DX
    src = [[*s, 0.0, 1e38]]
    out = art.ray_trace(n, xH2, xHp, None, DX, src, par, level0=2)
    lc = sources.point_source_maps(n, xH2, None, DX, src, par)
    kk, jj, ii = np.indices(shape)
    r = np.sqrt(((ii + 0.5) * DX - s[0]) ** 2 + ((jj + 0.5) * DX - s[1]) ** 2 + ((kk + 0.5) * DX - s[2]) ** 2) / DX
    for lo, hi, tol in ((1.5, 3, 0.06), (3, 5, 0.02), (5, 7, 0.02), (7, 9, 0.02)):
        m = (r >= lo) & (r < hi)
        for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C"):
            assert abs(out[k][m].sum() / lc[k][m].sum() - 1) < tol, (k, lo, hi)
    assert np.all(out["phi"] == 0.0)


def test_cells_mode_matches_the_full_trace():
    par = Params()
    shape = (10, 11, 12)
    n, xH2, xHp, xC = _medium(shape, 2)
    rng = np.random.default_rng(3)
    cells = np.stack(np.unravel_index(rng.choice(n.size, 30, replace=False), shape), 1)
    cells = np.concatenate([cells, [[5, 6, 5], [3, 9, 0], [0, 0, 0], [9, 10, 11]]])
    for kw in (dict(), dict(level0=1, tau_max=3.0, max_level=4)):
        full = art.ray_trace(n, xH2, xHp, xC, DX, SRC, par, **kw)
        got = art.ray_trace_cells(n, xH2, xHp, xC, DX, SRC, par, cells, **kw)
        for k in art.FIELDS:
            ref = full[k][cells[:, 0], cells[:, 1], cells[:, 2]]
            np.testing.assert_allclose(got[k], ref, rtol=1e-12, atol=0)


# ---- flux (Eq. e:Frad) and radiation force (Sec. 6.2) ---------------------------------

def _energy_fluxes(out):
    """c E_j per band in the flux's units: 4 pi J^D_j chi_j for PE and LW, phi for LyC."""
    return (4 * np.pi * C.J_PE * out["chi_PE"], 4 * np.pi * C.J_LW * out["chi_LW"], out["phi"])


@pytest.mark.parametrize("kw", [dict(), dict(level0=1, tau_max=3.0, max_level=4)])
def test_flux_bounded_by_the_energy_density(kw):
    """|F_j| <= c E_j in every cell (a sum of unit vectors times the deposits), with equality
    where one packet alone deposits."""
    par = Params()
    n, xH2, xHp, xC = _medium((10, 11, 12), 1)
    out = art.ray_trace(n, xH2, xHp, xC, DX, SRC, par, flux=True, **kw)
    F = out["flux"]
    for b, cE in enumerate(_energy_fluxes(out)):
        mag = np.sqrt(np.sum(F[3 * b:3 * b + 3] ** 2, 0))
        assert np.all(mag <= cE * (1 + 1e-12)), b
        assert mag.max() > 0


def _cone(shape, s):
    """Per cell: distance d from s to the centre (cm), unit vector to the centre, and cos of
    the half-angle of the cell's circumscribed sphere seen from s (0 where s is inside it)."""
    kk, jj, ii = np.indices(shape)
    v = np.stack([(ii + 0.5) * DX - s[0], (jj + 0.5) * DX - s[1], (kk + 0.5) * DX - s[2]])
    d = np.sqrt(np.sum(v * v, 0))
    rho = 0.5 * np.sqrt(3) * DX
    cosmax = np.where(d > rho, np.sqrt(np.maximum(1 - (rho / np.maximum(d, rho)) ** 2, 0)), 0.0)
    return d, v / np.maximum(d, 1e-300), cosmax


def test_flux_points_away_from_the_source():
    """Packets travel on straight lines from the source, so every packet crossing a cell is
    within the cone of the cell's circumscribed sphere: F_j . r_hat >= cos(theta_max) c E_j
    in every cell (exact; a wrong sign or a swapped component fails it)."""
    par = Params()
    shape = (12, 13, 14)
    n, xH2, xHp, xC = _medium(shape, 5, dense=False)
    s = np.array([6.3, 5.2, 7.9]) * DX
    out = art.ray_trace(n, xH2, xHp, xC, DX, [[*s, 1e49, 1e5 * sources.L_SUN]], par, flux=True)
    d, rhat, cosmax = _cone(shape, s)
    F = out["flux"]
    m = cosmax > 0.5
    assert m.sum() > 1000
    for b, cE in enumerate(_energy_fluxes(out)):
        along = np.sum(F[3 * b:3 * b + 3] * rhat, 0)
        assert np.all(along[m] >= cosmax[m] * cE[m] * (1 - 1e-12)), b
        assert np.all(along[m] > 0)


def test_flux_mirror_antisymmetry():
    """A source at a cell centre in a medium symmetric under x -> -x about it: F_x changes sign
    under the mirror, F_y and F_z do not (the HEALPix directions are mirror-symmetric)."""
    par = Params()
    shape = (9, 10, 11)
    n, xH2, xHp, xC = _medium(shape, 6, dense=False)
    n, xH2, xHp, xC = (0.5 * (a + a[:, :, ::-1]) for a in (n, xH2, xHp, xC))
    s = np.array([5.5, 4.7, 4.2]) * DX
    out = art.ray_trace(n, xH2, xHp, xC, DX, [[*s, 1e49, 1e5 * sources.L_SUN]], par, flux=True)
    F = out["flux"]
    for b in range(3):
        sc = np.abs(F[3 * b:3 * b + 3]).max()
        np.testing.assert_allclose(F[3 * b], -F[3 * b][:, :, ::-1], rtol=0, atol=1e-10 * sc)
        for a in (1, 2):
            np.testing.assert_allclose(F[3 * b + a], F[3 * b + a][:, :, ::-1], rtol=0, atol=1e-10 * sc)


def test_force_matches_the_absorbed_luminosity():
    """Every packet's absorbed luminosity dL_j brings the momentum dL_j n / c, so in each cell
    f . r_hat c dV lies between cos(theta_max) and 1 times the cell's absorbed luminosity
    alpha_j c E_j dV summed over bands (with h nu_LyC per LyC photon)."""
    par = Params()
    shape = (12, 13, 14)
    n, xH2, xHp, xC = _medium(shape, 7, dense=False)
    s = np.array([6.3, 5.2, 7.9]) * DX
    out = art.ray_trace(n, xH2, xHp, xC, DX, [[*s, 1e49, 1e5 * sources.L_SUN]], par, flux=True)
    T = np.full(shape, 50.0)
    fr = art.radiation_force(n, T, xH2, xHp, out["flux"], par, prad_ratio_max=np.inf)
    assert not fr["dust_off"].any()
    xHI = 1 - 2 * xH2 - xHp
    aLyC = n * (xHI * C.SIGMA_PI_H + xH2 * C.SIGMA_PI_H2 + par.Zd * C.SIG_D_LYC)
    cE = _energy_fluxes(out)
    absorbed = (C.SIG_D_PE * par.Zd * n * cE[0] + C.SIG_D_LW * par.Zd * n * cE[1]
                + aLyC * C.HNU_LYC * cE[2]) * DX ** 3
    d, rhat, cosmax = _cone(shape, s)
    along = np.sum(fr["f"] * rhat, 0) * C.C_LIGHT * DX ** 3
    m = cosmax > 0.5
    assert np.all(along[m] >= cosmax[m] * absorbed[m] * (1 - 1e-12))
    assert np.all(along[m] <= absorbed[m] * (1 + 1e-12))


def test_force_grain_destruction_switch():
    """Dust force off above 1e6 K and where P_rad = |F| / c exceeds 50 times 2 n k_B T; the
    photoionisation part of LyC stays; with no neutral hydrogen and the grains destroyed the
    force vanishes."""
    par = Params()
    n = np.array([1.0, 1.0, 1.0, 1.0, 10.0, 10.0, 10.0])
    T = np.array([1e4, 1.01e6, 1e4, 1e4, 100.0, 100.0, 2e6])
    xH2 = np.zeros(7)
    xHp = np.array([0.5, 0.5, 0.5, 0.5, 1.0, 1.0, 1.0])
    F = np.zeros((9, 7))
    F[0] = [1e-3, 1e-3, 0, 0, 0, 0, 0]          # PE energy flux along x
    P = 2 * n * C.K_B * T
    # cells 2 and 3: a LyC photon flux along -y whose pressure is 50 P times (1 -+ 1e-6)
    F[7, 2] = -50 * P[2] * C.C_LIGHT / C.HNU_LYC * (1 - 1e-6)
    F[7, 3] = -50 * P[3] * C.C_LIGHT / C.HNU_LYC * (1 + 1e-6)
    F[6, 4] = 1e6                                  # weak LyC in an ionised cell
    F[6, 5] = 50 * P[5] * C.C_LIGHT / C.HNU_LYC * 2  # strong LyC in an ionised cell
    F[6, 6] = 1e6
    fr = art.radiation_force(n, T, xH2, xHp, F, par)
    off = fr["dust_off"]
    assert off.tolist() == [False, True, False, True, False, True, True]
    f = fr["f"]
    assert f[0, 0] > 0 and f[0, 1] == 0.0
    # below the threshold the dust and the gas push; above it only the neutral hydrogen
    gas = n[2] * 0.5 * C.SIGMA_PI_H
    dust = n[2] * par.Zd * C.SIG_D_LYC
    np.testing.assert_allclose(f[1, 2] / F[7, 2], (gas + dust) * C.HNU_LYC / C.C_LIGHT, rtol=1e-14)
    np.testing.assert_allclose(f[1, 3] / F[7, 3], gas * C.HNU_LYC / C.C_LIGHT, rtol=1e-14)
    assert f[0, 4] > 0 and np.all(f[:, 5] == 0) and np.all(f[:, 6] == 0)


def test_force_momentum_update():
    """The source-term update of Sec. 6.2: from rest the energy gains the kinetic energy of the
    acquired momentum, (f dt)^2 / (2 rho); a force that reverses the momentum (f dt = -2 p)
    leaves the energy as it was; n = 0 is left alone."""
    par = Params(Zg=1.0)
    n = np.array([2.0, 3.0, 0.0])
    z = np.zeros(3)
    F = np.zeros((9, 3))
    F[0] = [1e-2, 1e-2, 1e-2]
    F[4] = [3e-3, -2e-3, 0.0]
    dt = 1e11
    f = art.radiation_force(n, np.full(3, 100.0), z, z, F, par, prad_ratio_max=np.inf)["f"]
    rho = 1.4 * C.M_H * n
    mom0 = np.zeros((3, 3))
    mom0[:, 1] = -0.5 * f[:, 1] * dt
    e0 = np.array([3e-22, 2e-10, 3e-10])
    out = art.radiation_force(n, np.full(3, 100.0), z, z, F, par, prad_ratio_max=np.inf,
                              dt=dt, mom=mom0, etot=e0)
    np.testing.assert_allclose(out["mom"], mom0 + f * dt, rtol=1e-15)
    np.testing.assert_allclose(out["etot"][0] - e0[0], np.sum((f[:, 0] * dt) ** 2) / (2 * rho[0]), rtol=1e-12)
    np.testing.assert_allclose(out["etot"][1], e0[1], rtol=1e-12)
    assert np.all(f[:, 2] == 0) and out["etot"][2] == e0[2]


def test_cells_mode_flux_matches_the_full_trace():
    par = Params()
    shape = (10, 11, 12)
    n, xH2, xHp, xC = _medium(shape, 2)
    rng = np.random.default_rng(8)
    cells = np.stack(np.unravel_index(rng.choice(n.size, 20, replace=False), shape), 1)
    full = art.ray_trace(n, xH2, xHp, xC, DX, SRC, par, flux=True)
    got = art.ray_trace_cells(n, xH2, xHp, xC, DX, SRC, par, cells, flux=True)
    ref = full["flux"][:, cells[:, 0], cells[:, 1], cells[:, 2]]
    sc = np.abs(full["flux"]).max(axis=(1, 2, 3))[:, None]
    np.testing.assert_allclose(got["flux"], ref, rtol=1e-12, atol=1e-14 * sc.max())
