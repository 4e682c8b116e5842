"""The plane-parallel H I -> H2 transition (Sec. 7.2) against the analytic transition column
the paper quotes (Eqs. e:NH_trans, e:alpha, e:G): a beamed, CR-free slab with k_gr = 3e-17
evolved to steady state.  The formula is sharp in the strong- and weak-field limits and
approximate in between (alpha G / 2 ~ 0.5), where it is checked to 30%; the transition is
resolved by more than 3 cells in every case (the paper's convergence condition)."""
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
