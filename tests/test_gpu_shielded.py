"""Local shielding-length radiation (ism_local_shielding) and the shielded one-zone
equilibrium computed with the GPU step, against the oracle."""
import numpy as np
import pytest

import helpers as H
from oracle import constants as OC
from oracle import shield
from oracle.constants import Params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ism():
    import torch
    from paper_2210_08024_amd import ism as m
    torch.cuda.set_device(0)
    m.init(0)
    return m


@pytest.mark.parametrize("prec,cr_mode", [(0, 1), (1, 1), (0, 0)])
def test_local_shielding_matches_oracle(ism, prec, cr_mode):
    import torch
    rng = np.random.default_rng(3)
    N = 777
    n = 10 ** rng.uniform(-1, 6, N)
    xH2 = rng.uniform(0, 0.5, N)
    xC = rng.uniform(0, 1.6e-4, N)
    L = shield.shielding_length(n)
    par = Params(cr_mode=cr_mode, Zd=0.7)
    ref = shield.local_shielding(n, xH2, xC, L, par)
    out = ism.local_shielding(H.to_dev(n), H.to_dev(xH2), H.to_dev(xC), H.to_dev(L), H.ism_params_from(par), prec)
    tol = 1e-12 if prec == 0 else 2e-5
    for k, rk in (("chi_PE", "chi_PE"), ("chi_LW", "chi_LW"), ("chi_H2", "chi_H2"), ("chi_C", "chi_C"),
                  ("N_eff", "Neff"), ("xi", "xi")):
        g = out[k].cpu().numpy().astype(np.float64)
        err = np.abs(g - ref[rk]) / np.maximum(np.abs(ref[rk]), 1e-300)
        ok = np.abs(ref[rk]) > 1e-300
        assert err[ok].max() < tol, (k, err[ok].max())


def test_shielded_equilibrium_on_the_gpu(ism):
    """Thirty rounds of (local shielding, FP64 step of 1e7 yr) on a density sweep, as the
    oracle does them: T, x_H2, x_CO within 1e-9."""
    import torch
    par = Params(cr_mode=1)
    ip = H.ism_params_from(par)
    n = 10 ** np.linspace(0.0, 6.5, 53)
    ref, _ = shield.shielded_equilibrium(n, par, outer=30, tol=0.0)
    N = n.size
    nd, L = H.to_dev(n), H.to_dev(shield.shielding_length(n))
    T = torch.full((N,), 100.0, dtype=torch.float64, device="cuda")
    xH2 = torch.full((N,), 0.1, dtype=torch.float64, device="cuda")
    xHp = torch.full((N,), 1e-3, dtype=torch.float64, device="cuda")
    xC = torch.zeros(N, dtype=torch.float64, device="cuda")
    for _ in range(30):
        rad = ism.local_shielding(nd, xH2, xC, L, ip, ism.F64)
        rad["phi"] = None
        out = ism.chem_cool_step(nd, T, xH2, xHp, rad, 1e7 * OC.YR, ip, ism.F64)
        xC = (par.xCtot - out["xCp"] - out["xCO"]).clamp_min(0.0)
    g = dict(T=T.cpu().numpy(), xH2=xH2.cpu().numpy(), xHp=xHp.cpu().numpy(), xCO=out["xCO"].cpu().numpy(),
             xCp=out["xCp"].cpu().numpy(), xe=out["xe"].cpu().numpy())
    H.check_fields(g, ref, 1e-9, H.FLOORS_F64, par.xCtot, label="shielded equilibrium")
