"""The plane-parallel H I -> H2 transition (Sec. 7.3) against the analytic transition column
the paper quotes (Eqs. e:NH_trans, e:alpha, e:G): a beamed, CR-free slab with k_gr = 3e-17
evolved to steady state.  The formula is sharp in the strong- and weak-field limits and
approximate in between (alpha G / 2 ~ 0.5), where it is checked to 30%; the transition is
resolved by more than 3 cells in every case (the paper's convergence condition).  With CR
ionisation (attenuated as in Eq. e:cratt) the text of Sec. 7.3 fixes two facts without
printed values: the transition column grows with xi_cr,0, and deep in the slab the H I
fraction is linear in xi / (k_gr n) with the constant that Eqs. e:HH and eq:H2_cr give."""
import numpy as np
import pytest

from oracle import slab
from oracle.constants import PC

pytestmark = [pytest.mark.filterwarnings("ignore::RuntimeWarning"), pytest.mark.slow]


def test_analytic_formula_limits():
    """Eq. e:NH_trans reduces to ln(alpha G)/sigma for alpha G >> 1 and to
    (beta / sigma) (alpha G / 2)^(1/beta) for alpha G << 1."""
    s = slab.analytic_ntrans(1.0, 1.0, sigma_d=1.9e-21)
    st = 1.0
    G = 3.0e-5 * st * (9.9 / (1 + 8.9 * st)) ** 0.37
    for n, chi in ((1e-3, 1e5), (1e6, 1e-3)):
        a = 3.8e4 * chi * (1e2 / n)
        N = slab.analytic_ntrans(n, chi, sigma_d=1.9e-21)
        if a * G > 1e6:
            assert N == pytest.approx(np.log(a * G / 2) / 1.9e-21, rel=0.01)
        else:
            assert N == pytest.approx(0.7 / 1.9e-21 * (a * G / 2) ** (1 / 0.7), rel=0.01)
    assert s > 0


@pytest.mark.parametrize("n,chi0,dx_pc,nx,tol", [(1e3, 1.0, 1e-4, 128, 0.15), (1e2, 1.0, 0.02, 128, 0.30),
                                                 (1e2, 1e3, 0.1, 256, 0.10)])
def test_transition_column_matches_the_analytic_approximation(n, chi0, dx_pc, nx, tol):
    xH2, out = slab.slab_steady(n, chi0, nx, dx_pc * PC, dt_yr=1e6, steps=100)
    Nt = slab.transition_column(n, xH2, dx_pc * PC)
    assert Nt / (n * dx_pc * PC) > 3.0                     # resolved
    assert Nt == pytest.approx(slab.analytic_ntrans(n, chi0), rel=tol)
    assert 2 * xH2[-1] > 0.75                               # mostly molecular at depth


def _cr_par(chi0, xi0):
    from oracle.constants import Params
    return Params(chi0=chi0, xi_cr0=xi0, kgr_const=1, cr_mode=1 if xi0 > 0 else 0)


def test_cosmic_rays_raise_the_transition_column():
    """Sec. 7.3 with CR ionisation attenuated by Eq. e:cratt: CRs destroy H2, so the transition
    column grows with xi_cr,0, and tends to the CR-free column as xi_cr,0 -> 0."""
    n, chi0, dx, nx = 1e2, 1.0, 0.02 * PC, 192
    N = []
    for xi0 in (0.0, 2e-18, 2e-17, 2e-16, 1e-15):
        xH2, _ = slab.slab_steady(n, chi0, nx, dx, dt_yr=1e6, steps=100, par=_cr_par(chi0, xi0))
        N.append(slab.transition_column(n, xH2, dx))
    N = np.array(N)
    assert np.all(N / (n * dx) > 3.0)                       # every transition resolved
    assert N[1] == pytest.approx(N[0], rel=0.03)
    assert np.all(np.diff(N[1:]) > 0), N
    assert N[-1] > 1.2 * N[0]


def test_deep_hi_fraction_follows_the_cosmic_ray_balance():
    """Deep in a thick slab (photodissociation shielded away, cold gas) Eq. e:HH reduces to the
    balance of grain formation and CR destruction, k_gr n x_H = 1.65 zeta_cr,H2 x_H2 with
    zeta_cr,H2 = 2 xi (2.3 x_H2 + 1.5 x_HI) (Eq. eq:H2_cr): the H I fraction is linear in
    xi / (k_gr n), x_HI k_gr n / xi -> 1.65 x 2.3 / 2 for x_H2 -> 1/2 (the text of Sec. 7.3).
    Checked with the local, attenuated xi of every cell beyond N_H = 5e21 cm^-2."""
    from oracle.columns import columns_beam
    n, chi0, xi0, dx, nx = 1e2, 1.0, 2e-16, 0.25 * PC, 160
    par = _cr_par(chi0, xi0)
    xH2, out = slab.slab_steady(n, chi0, nx, dx, dt_yr=1e6, steps=100, par=par)
    shape = (1, 1, nx)
    xC = np.maximum(par.xCtot - out["xCp"] - out["xCO"], 0.0).reshape(shape)
    r = columns_beam(np.full(shape, n), xH2.reshape(shape), xC, dx, par)
    xi = r["xi"].ravel()
    kgr = 3.0e-17 * par.Zd
    xHp = out["xHp"]
    xH = 1.0 - 2.0 * xH2 - xHp
    Ncol = (np.arange(nx) + 0.5) * n * dx
    deep = Ncol > 5e21
    assert deep.sum() > 50
    # the balance with each cell's own abundances
    destroy = 1.65 * 2.0 * xi * (2.3 * xH2 + 1.5 * xH) * xH2
    np.testing.assert_allclose(kgr * n * xH[deep], destroy[deep], rtol=0.02)
    # and its limit: linear in xi / (k_gr n)
    ratio = xH * kgr * n / xi
    np.testing.assert_allclose(ratio[deep], 1.65 * 2.3 / 2.0, rtol=0.03)
    # the regime of the limit: x_HI small, x_H+ negligible beside it
    assert np.all(xH[deep] < 0.05) and np.all(xHp[deep] < 1e-4 * xH[deep])
