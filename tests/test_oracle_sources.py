"""Pins of the point-source oracle (oracle/sources.py) against closed forms, brute-force
quadrature and symmetry."""
import numpy as np
import pytest

from oracle import constants as C
from oracle import micro, sources
from oracle.columns import f_shld_H2
from oracle.constants import Params

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")
DX = 3.0e18


def test_uniform_field_column_is_density_times_length():
    rng = np.random.default_rng(0)
    n = np.full((6, 7, 8), 2.5)
    for _ in range(50):
        p0 = rng.uniform(0, 1, 3) * np.array([8, 7, 6]) * DX
        p1 = rng.uniform(0, 1, 3) * np.array([8, 7, 6]) * DX
        (N,) = sources.segment_columns((n,), DX, p0, p1)
        assert N == pytest.approx(2.5 * np.linalg.norm(p1 - p0), rel=1e-13)


def test_axis_ray_through_slabs():
    """Along x through cells of densities 1, 2, 3, ...: partial first and last cells."""
    nx = 6
    n = np.broadcast_to(np.arange(1.0, nx + 1)[None, None, :], (2, 2, nx)).copy()
    p0 = np.array([0.25 * DX, 0.5 * DX, 0.5 * DX])
    p1 = np.array([4.75 * DX, 0.5 * DX, 0.5 * DX])
    (N,) = sources.segment_columns((n,), DX, p0, p1)
    expect = (0.75 * 1 + 2 + 3 + 4 + 0.75 * 5) * DX
    assert N == pytest.approx(expect, rel=1e-14)


def test_segment_columns_against_fine_quadrature():
    rng = np.random.default_rng(1)
    n = 10.0 ** rng.uniform(-1, 2, (5, 6, 7))
    x2 = rng.uniform(0, 0.5, n.shape)
    for _ in range(20):
        p0 = rng.uniform(0, 1, 3) * np.array([7, 6, 5]) * DX
        p1 = rng.uniform(0, 1, 3) * np.array([7, 6, 5]) * DX
        N, N2 = sources.segment_columns((n, n * x2), DX, p0, p1)
        M = 200000
        t = (np.arange(M) + 0.5) / M
        pts = p0[None, :] + t[:, None] * (p1 - p0)[None, :]
        idx = np.minimum(np.floor(pts / DX).astype(int), np.array([7, 6, 5]) - 1)
        L = np.linalg.norm(p1 - p0)
        Nq = n[idx[:, 2], idx[:, 1], idx[:, 0]].sum() * L / M
        N2q = (n * x2)[idx[:, 2], idx[:, 1], idx[:, 0]].sum() * L / M
        # the midpoint rule is exact inside cells; each of the <= 18 crossings errs by < one sample
        tol = 18 * L / M * n.max()
        assert abs(N - Nq) <= tol and abs(N2 - N2q) <= tol


def test_segment_columns_symmetric_in_direction():
    rng = np.random.default_rng(2)
    n = rng.uniform(0, 5, (4, 4, 4))
    for _ in range(20):
        p0, p1 = rng.uniform(0, 4 * DX, 3), rng.uniform(0, 4 * DX, 3)
        a = sources.segment_columns((n,), DX, p0, p1)
        b = sources.segment_columns((n,), DX, p1, p0)
        assert a[0] == pytest.approx(b[0], rel=1e-13)


def test_vacuum_inverse_square_and_band_split():
    """No gas: chi_PE = chi_LW = chi_H2 = L / (16 pi^2 r^2 J^D_FUV), and J_PE + J_LW carries
    the whole mean intensity L / (16 pi^2 r^2)."""
    n = np.zeros((8, 8, 8))
    L = 1.36e6 * sources.L_SUN
    src = np.array([[0.5 * DX, 0.5 * DX, 0.5 * DX, 1e49, L]])
    cells = np.array([[0, 0, 4], [0, 0, 7], [3, 0, 4]])
    r = sources.point_source_cells(n, n, None, DX, src, Params(), cells)
    for m, (k, j, i) in enumerate(cells):
        d = np.linalg.norm(np.array([i, j, k]) * DX)
        chi = L / (16 * np.pi ** 2 * d * d * C.J_FUV)
        assert r["chi_PE"][m] == pytest.approx(chi, rel=1e-13)
        assert r["chi_LW"][m] == pytest.approx(chi, rel=1e-13)
        assert r["chi_H2"][m] == pytest.approx(chi * f_shld_H2(0.0), rel=1e-13)
        J = C.J_PE * r["chi_PE"][m] + C.J_LW * r["chi_LW"][m]
        assert J == pytest.approx(L / (16 * np.pi ** 2 * d * d), rel=1e-13)
    # doubling the distance quarters the field
    assert r["chi_PE"][0] / r["chi_PE"][2] == pytest.approx((3 ** 2 + 4 ** 2) / 4 ** 2, rel=1e-13)


def test_lyc_inside_and_outside_the_stromgren_radius():
    n = np.full((1, 1, 64), 1.0)
    Q = 1e47
    Rst = sources.stromgren_radius(Q)
    # closed form: 3 Q = 4 pi alpha_B R^3
    assert 4 * np.pi * micro.alpha_B(1e4) * Rst ** 3 / 3 == pytest.approx(Q, rel=1e-12)
    dx = Rst / 20.0
    src = np.array([[0.5 * dx, 0.5 * dx, 0.5 * dx, Q, 0.0]])
    cells = np.array([[0, 0, 10], [0, 0, 30]])
    r = sources.point_source_cells(n, np.zeros_like(n), None, dx, src, Params(), cells)
    d = 10 * dx
    assert r["phi"][0] == pytest.approx(Q * np.exp(-C.SIG_D_LYC * d) / (4 * np.pi * d * d), rel=1e-12)
    assert r["phi"][1] == 0.0


def test_dust_attenuation_and_shielding_columns():
    """A uniform slab between source and cell: exp(-sigma N) per band and f_shld at the
    full H2 column."""
    n = np.full((1, 1, 40), 50.0)
    xH2 = np.full_like(n, 0.3)
    L = 1e5 * sources.L_SUN
    src = np.array([[0.5 * DX, 0.5 * DX, 0.5 * DX, 0.0, L]])
    par = Params(Zd=2.0)
    r = sources.point_source_cells(n, xH2, None, DX, src, par, np.array([[0, 0, 20]]))
    d = 20 * DX
    N = 50.0 * d
    chi = L / (16 * np.pi ** 2 * d * d * C.J_FUV)
    assert r["chi_PE"][0] == pytest.approx(chi * np.exp(-C.SIG_D_PE * 2.0 * N), rel=1e-12)
    assert r["chi_H2"][0] == pytest.approx(chi * np.exp(-C.SIG_D_LW * 2.0 * N) * f_shld_H2(0.3 * N), rel=1e-12)
