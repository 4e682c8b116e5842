"""The 512^3 point-source configuration (134,217,728 cells, 2 pc, 16 sources, one step of
1e4 yr) on all three paths at full size.  Checked against the oracle on sampled cells: the
FP64 six-ray columns and straight-line source maps at a few cells, then the step of every
path on the 64^3 subsample (every 8th cell along each axis, 262,144 cells) against the FP64
oracle step fed the GPU's FP64 radiation at those cells.

Bars: F64 1e-9; mixed and surrogate a flat 1e-3 in T and every abundance on every subsample
cell (a cell may be exempt only when named in ILL_CONDITIONED, see helpers.check_mixed_flat);
accepted surrogate cells are certified to 1e-3 and fall under the same bar."""
import numpy as np
import pytest

import helpers as H
from oracle import columns as ocol
from oracle import constants as OC
from oracle import sources as osrc
from oracle.constants import Params

pytestmark = pytest.mark.gpu
FIELDS = ("T", "xH2", "xHp", "xe", "xCp", "xCO")
RAD = ("chi_PE", "chi_LW", "chi_H2", "chi_C", "N_eff", "xi")


@pytest.fixture(scope="module")
def ism():
    import torch
    from paper_2210_08024_amd import ism as m
    torch.cuda.set_device(0)
    m.init(0)
    return m


# cell index -> reason: cells where the FP64 scheme itself cannot be held to 1e-3 by a float
# evaluation (see helpers.check_mixed_flat and helpers.oracle_sensitivity)
ILL_CONDITIONED = {
    81940480: "(k, j, i) = (312, 296, 0), n = 16.8, T 133 -> 31.5 K in 21 substeps as x_H+ recombines "
              "from 0.29 to 0.011: near thermal balance the derivative dH/dT_mu is a small difference of "
              "two evaluations of H, and one float rounding (1e-7 of the larger term) of the second one "
              "moves the end T by 1.9e-3 in the oracle itself (a 1e-6 input change: 1.2e-4)",
}


def test_c4_full_size_all_paths(ism):
    import torch
    from paper_2210_08024_amd import surrogate_train, workloads
    print("pts512: generating the 512^3 inputs", flush=True)
    s, cfg = workloads.make("pts512")
    shape = s["n"].shape
    N = s["n"].size
    dx = cfg["dx_pc"] * OC.PC
    dt = cfg["dt_yr"] * OC.YR
    par_o = Params(Zg=1.0, Zd=1.0, cr_mode=2)
    par = H.ism_params_from(par_o)
    dev = lambda a, dt_=None: H.to_dev(a, dt_)
    n = dev(s["n"])
    T0, xH2_0, xHp_0 = dev(s["T"]), dev(s["xH2"]), dev(s["xHp"])
    xi = dev(s["xi"])
    print("pts512: point-source maps (F64)", flush=True)
    maps = {k: torch.zeros(N, dtype=torch.float64, device="cuda") for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "phi")}
    ism.point_sources(n.view(shape), xH2_0.view(shape), None, dx, par, 0, cfg["sources"],
                      {k: v.view(shape) for k, v in maps.items()})
    # radiation checks at a few cells
    rng = np.random.default_rng(44)
    few = rng.choice(N, 24, replace=False)
    cells = np.stack(np.unravel_index(few, shape), 1)
    tf = torch.from_numpy(few).cuda()
    ref_maps = osrc.point_source_cells(s["n"], s["xH2"], None, dx, cfg["sources"], par_o, cells[:6])
    for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "phi"):
        g = maps[k][tf[:6]].cpu().numpy()
        err = np.abs(g - ref_maps[k]) / np.maximum(np.abs(ref_maps[k]), 1e-300)
        assert err.max() < 1e-9, ("maps", k, err.max())
    # the step comparison on the 64^3 subsample: every 8th cell along each axis (262,144 cells)
    st = 8
    kk, jj, ii = np.meshgrid(*(np.arange(0, m, st) for m in shape), indexing="ij")
    idx = (ii + shape[2] * (jj + shape[1] * kk)).ravel()
    tid = torch.from_numpy(idx).cuda()
    sur = surrogate_train.load()
    nfb = torch.zeros(1, dtype=torch.int64, device="cuda")
    got, rad_sample = {}, None
    for path in ("f64", "mixed", "surrogate"):
        print(f"pts512: path {path}", flush=True)
        f64 = path == "f64"
        rd = torch.float64 if f64 else torch.float32
        rad = {k: torch.empty(N, dtype=rd, device="cuda") for k in RAD}
        rad["xi"].copy_(xi)
        ism.columns6(n.view(shape), xH2_0.view(shape), None, dx, par, 0 if f64 else 1,
                     out={k: v.view(shape) for k, v in rad.items()})
        if f64:
            rc = ocol.columns6_cells(s["n"], s["xH2"], None, dx, par_o, cells)
            for k, ko in (("chi_PE", "chi_PE"), ("chi_LW", "chi_LW"), ("chi_H2", "chi_H2"), ("chi_C", "chi_C"),
                          ("N_eff", "N_eff")):
                g = rad[k][tf].cpu().numpy()
                err = np.abs(g - rc[ko]) / np.maximum(np.abs(rc[ko]), 1e-300)
                assert err.max() < 1e-9, ("columns", k, err.max())
        for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C"):
            rad[k].add_(maps[k].to(rd))
        r = dict(rad)
        r["phi"] = maps["phi"].to(rd)
        T, xH2, xHp = T0.clone(), xH2_0.clone(), xHp_0.clone()
        if path == "surrogate":
            out = ism.chem_cool_step_surrogate(sur, n, T, xH2, xHp, r, dt, par, n_fallback=nfb)
            print(f"  fallback fraction {nfb.item() / N:.4f}", flush=True)
        else:
            out = ism.chem_cool_step(n, T, xH2, xHp, r, dt, par, 0 if f64 else 1)
        assert int((out["status"] & 0xEF).sum().item()) == 0
        if f64:
            rad_sample = {k: r[k][tid].cpu().numpy() for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "phi", "xi")}
            rad_sample["Neff"] = r["N_eff"][tid].cpu().numpy()
        g = dict(T=T[tid].cpu().numpy(), xH2=xH2[tid].cpu().numpy(), xHp=xHp[tid].cpu().numpy())
        for k in ("xCp", "xCO", "xe"):
            g[k] = out[k][tid].cpu().numpy().astype(np.float64)
        got[path] = g
        del rad, r, out
        torch.cuda.empty_cache()
    print(f"pts512: oracle on {len(idx)} cells", flush=True)
    ref = H.oracle_step(s, rad_sample, dt, par_o, idx=idx)
    H.check_fields(got["f64"], ref, 1e-9, H.FLOORS_F64, par_o.xCtot, label="pts512 F64")
    worst = np.zeros(len(idx))
    for path in ("mixed", "surrogate"):
        for k in FIELDS:
            worst = np.maximum(worst, H.mixed_rel(got[path][k], ref[k], k, par_o.xCtot))
    sens = None
    over = np.nonzero(worst > 1e-3)[0]
    if over.size:
        # the oracle's own conditioning, at the cells over the bar only (for the report)
        sens = np.zeros(len(idx))
        sens[over] = H.oracle_sensitivity(s, {k: v[over] for k, v in rad_sample.items()}, dt, par_o, idx[over],
                                          {k: v[over] for k, v in ref.items()})
    for path in ("mixed", "surrogate"):
        H.check_mixed_flat(got[path], ref, idx, par_o.xCtot, named=ILL_CONDITIONED, sens=sens,
                           label=f"pts512 {path}")
