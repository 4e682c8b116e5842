"""The 128^3 GRF configuration across its metallicities and step lengths: Z' in {0.1, 1, 3} x
dt in {1e3, 1e4, 1e5} yr (Z' = 1, dt = 1e4 yr also runs in test_gpu_parity with more fields).
GPU columns6 + step over the whole grid, the oracle on 1,024 sampled cells computed one by one.

Bars: FP64 within 1e-9 relative; the mixed path within a flat 1e-3 relative in T and every
abundance on every sampled cell.  A cell may be exempt only if it is named in ILL_CONDITIONED
with the reason: the FP64 scheme itself moves its end state by S >= 1e-4 when the input T,
x_H2, x_H+ change by a relative 1e-6 (about ten FP32 ulps), so no float evaluation of it can be
held to 1e-3; such a cell is still held to 10 S."""
import numpy as np
import pytest

import helpers as H
from oracle import columns as ocol
from oracle import constants as OC
from oracle.constants import Params

pytestmark = pytest.mark.gpu

# (Z', dt in yr) -> {cell index: reason}
ILL_CONDITIONED = {}


@pytest.fixture(scope="module")
def ism():
    import torch
    from paper_2210_08024_amd import ism as m
    torch.cuda.set_device(0)
    m.init(0)
    return m


@pytest.fixture(scope="module")
def grf128():
    from paper_2210_08024_amd import workloads
    return workloads.make("grf128")


PAIRS = [(0.1, 1e3), (0.1, 1e4), (0.1, 1e5), (1.0, 1e3), (1.0, 1e5), (3.0, 1e3), (3.0, 1e4), (3.0, 1e5)]


@pytest.mark.parametrize("Zg,dt_yr", PAIRS)
def test_grf128_metallicity_and_step_length(ism, grf128, Zg, dt_yr):
    import torch
    s, cfg = grf128
    print(f"grf128 Z'={Zg} dt={dt_yr:g} yr", flush=True)
    shape = s["n"].shape
    par = Params(Zg=Zg, Zd=Zg, cr_mode=1)
    ipar = H.ism_params_from(par)
    dx = cfg["dx_pc"] * OC.PC
    dt = dt_yr * OC.YR
    N = s["n"].size
    rng = np.random.default_rng(int(Zg * 10 + np.log10(dt_yr)))
    idx = rng.choice(N, 1024, replace=False)
    cells = np.stack(np.unravel_index(idx, shape), 1)
    rc = ocol.columns6_cells(s["n"], s["xH2"], None, dx, par, cells)
    radi = dict(chi_PE=rc["chi_PE"], chi_LW=rc["chi_LW"], chi_H2=rc["chi_H2"], chi_C=rc["chi_C"],
                phi=np.zeros(len(idx)), xi=rc["xi"], Neff=rc["N_eff"])
    ref = H.oracle_step(s, radi, dt, par, idx=idx)
    sens = H.oracle_sensitivity(s, radi, dt, par, idx, ref)
    tid = torch.from_numpy(idx).cuda()
    for prec in (0, 1):
        n = H.to_dev(s["n"])
        T, xH2, xHp = H.to_dev(s["T"]), H.to_dev(s["xH2"]), H.to_dev(s["xHp"])
        rad = ism.columns6(n.view(shape), xH2.view(shape), None, dx, ipar, prec)
        radf = {k: v.view(-1) for k, v in rad.items()}
        radf["phi"] = None
        out = ism.chem_cool_step(n, T, xH2, xHp, radf, dt, ipar, prec)
        g = dict(T=T[tid].cpu().numpy(), xH2=xH2[tid].cpu().numpy(), xHp=xHp[tid].cpu().numpy())
        for k in ("xCp", "xCO", "xe"):
            g[k] = out[k][tid].cpu().numpy().astype(np.float64)
        assert int((out["status"].cpu().numpy() & 0xEF).sum()) == 0
        if prec == 0:
            H.check_fields(g, ref, 1e-9, H.FLOORS_F64, par.xCtot, label=f"F64 Z'={Zg} dt={dt_yr:g}")
            continue
        H.check_mixed_flat(g, ref, idx, par.xCtot, named=ILL_CONDITIONED.get((Zg, dt_yr)), sens=sens,
                           label=f"mixed Z'={Zg} dt={dt_yr:g}")
