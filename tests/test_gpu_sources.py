"""Point-source radiation (ism_point_sources) against the long-characteristics oracle, and
the 256^3 point-source configuration (ten successive steps) on sampled cells."""
import numpy as np
import pytest

import helpers as H
from oracle import art
from oracle import columns as ocol
from oracle import constants as OC
from oracle import sources as osrc
from oracle.constants import Params

pytestmark = pytest.mark.gpu
KEYS = ("chi_PE", "chi_LW", "chi_H2", "chi_C", "phi")


@pytest.fixture(scope="module")
def ism():
    import torch
    from paper_2210_08024_amd import ism as m
    torch.cuda.set_device(0)
    m.init(0)
    return m


def _zeros(torch, shape, rd):
    return {k: torch.zeros(shape, dtype=rd, device="cuda") for k in KEYS}


def _small_case(seed):
    rng = np.random.default_rng(seed)
    shape = (8, 10, 12)  # nz, ny, nx
    n = 10.0 ** rng.uniform(-1.0, 2.5, shape)
    xH2 = rng.uniform(0.0, 0.5, shape)
    xC = rng.uniform(0.0, 1e-4, shape)
    dx = 2.0 * OC.PC
    box = np.array([12, 10, 8]) * dx
    src = np.concatenate([rng.uniform(0, 1, (3, 3)) * box, np.full((3, 1), 1e49),
                          np.full((3, 1), 1e5 * osrc.L_SUN)], axis=1)
    src[0, :3] = [5.5 * dx, 4.5 * dx, 3.5 * dx]   # exactly at a cell centre (r < dx/2 there)
    src[1, :3] = [3.0 * dx, 7.0 * dx, 2.0 * dx]   # on a cell corner
    return n, xH2, xC, dx, src


@pytest.mark.parametrize("prec", [0, 1])
def test_point_sources_match_oracle_full_grid(ism, prec):
    import torch
    n, xH2, xC, dx, src = _small_case(5)
    par = Params(Zd=1.5)
    ref = osrc.point_source_maps(n, xH2, xC, dx, src, par)
    rd = torch.float64 if prec == 0 else torch.float32
    out = _zeros(torch, n.shape, rd)
    ism.point_sources(H.to_dev(n).view(n.shape), H.to_dev(xH2).view(n.shape), H.to_dev(xC).view(n.shape), dx,
                      H.ism_params_from(par), prec, src, out)
    tol = 1e-11 if prec == 0 else 2e-5
    for k in KEYS:
        g = out[k].cpu().numpy().astype(np.float64)
        scale = np.abs(ref[k]).max()
        err = np.abs(g - ref[k]) / np.maximum(np.abs(ref[k]), 1e-30 * scale + 1e-300)
        assert err.max() < tol, (k, err.max())


def test_point_sources_add_to_existing_fields_and_edge_cases(ism):
    import torch
    n, xH2, xC, dx, src = _small_case(6)
    par = H.ism_params_from(Params())
    out = _zeros(torch, n.shape, torch.float64)
    for v in out.values():
        v.fill_(1.0)
    ism.point_sources(H.to_dev(n).view(n.shape), H.to_dev(xH2).view(n.shape), None, dx, par, 0, src, out)
    ref = osrc.point_source_maps(n, xH2, None, dx, src, Params())
    for k in KEYS:
        np.testing.assert_allclose(out[k].cpu().numpy(), 1.0 + ref[k], rtol=1e-11)
    # no sources: no change
    before = {k: v.clone() for k, v in out.items()}
    ism.point_sources(H.to_dev(n).view(n.shape), H.to_dev(xH2).view(n.shape), None, dx, par, 0, [], out)
    for k in KEYS:
        assert torch.equal(before[k], out[k])
    # a source outside the grid is rejected before launch
    bad = src.copy()
    bad[0, 0] = 100 * dx
    with pytest.raises(ism.IsmError):
        ism.point_sources(H.to_dev(n).view(n.shape), H.to_dev(xH2).view(n.shape), None, dx, par, 0, bad, out)


@pytest.fixture(scope="module")
def pts256():
    from paper_2210_08024_amd import workloads
    return workloads.make("pts256")


@pytest.mark.parametrize("maps_kind", ["art", "lc"])
def test_c2_ten_steps_sampled(ism, pts256, maps_kind):
    """256^3, 2 pc, 16 sources, CR map: six-ray columns every step, source maps once (from the
    initial state; adaptive ray tracing as in the benchmark, or long characteristics), ten
    mixed steps of 1e4 yr with x_C fed back.  Sampled cells: the maps against the oracle on 48
    cells, and the first and last steps on 4,096 cells against the oracle step from the GPU's
    state and radiation of that step (a flat 1e-3 in T and abundances, floors as elsewhere)."""
    import torch
    s, cfg = pts256
    shape = s["n"].shape
    N = s["n"].size
    dx = cfg["dx_pc"] * OC.PC
    dt = cfg["dt_yr"] * OC.YR
    par_o = Params(Zg=1.0, Zd=1.0, cr_mode=2)
    par = H.ism_params_from(par_o)
    n = H.to_dev(s["n"]).view(shape)
    T, xH2, xHp = H.to_dev(s["T"]), H.to_dev(s["xH2"]), H.to_dev(s["xHp"])
    xi = H.to_dev(s["xi"], torch.float32)
    maps = _zeros(torch, shape, torch.float32)
    rng = np.random.default_rng(11)
    # the maps' oracle walks every source per cell: 48 cells; the step's oracle takes the GPU's
    # radiation at the cell: 4,096 cells
    idx_maps = np.sort(rng.choice(N, 48, replace=False))
    idx = np.sort(rng.choice(N, 4096, replace=False))
    tmaps = torch.from_numpy(idx_maps).cuda()
    tid = torch.from_numpy(idx).cuda()
    cells = np.stack(np.unravel_index(idx_maps, shape), 1)
    print(f"pts256 ten steps, maps by {maps_kind}", flush=True)
    if maps_kind == "art":
        ism.ray_trace(n, xH2.view(shape), xHp.view(shape), None, dx, par, 1, cfg["sources"], maps)
        ref_maps = art.ray_trace_cells(s["n"], s["xH2"], s["xHp"], None, dx, cfg["sources"], par_o, cells)
        tol, fl = 1e-4, 1e-6   # float deposits, atomically summed (the ray-tracing bars)
    else:
        ism.point_sources(n, xH2.view(shape), None, dx, par, 1, cfg["sources"], maps)
        ref_maps = osrc.point_source_cells(s["n"], s["xH2"], None, dx, cfg["sources"], par_o, cells)
        tol, fl = 2e-5, 0.0
    for k in KEYS:
        g = maps[k].view(-1)[tmaps].cpu().numpy().astype(np.float64)
        err = np.abs(g - ref_maps[k]) / np.maximum(np.abs(ref_maps[k]), max(1e-30, fl * np.abs(ref_maps[k]).max()))
        assert err.max() < tol, (k, err.max())
    xC = None
    xCt = par_o.xCtot
    for step in range(cfg["steps"]):
        rad = {k: torch.empty(N, dtype=torch.float32, device="cuda") for k in
               ("chi_PE", "chi_LW", "chi_H2", "chi_C", "N_eff")}
        rad["xi"] = xi.clone()
        ism.columns6(n, xH2.view(shape), xC, dx, par, 1, out={k: v.view(shape) for k, v in rad.items()})
        for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C"):
            rad[k] += maps[k].view(-1)
        rad["phi"] = maps["phi"].view(-1)
        state0 = {k: v[tid].cpu().numpy() for k, v in (("T", T), ("xH2", xH2), ("xHp", xHp))}
        out = ism.chem_cool_step(n.view(-1), T, xH2, xHp, rad, dt, par, 1)
        if step in (0, cfg["steps"] - 1):
            radi = {k: rad[k][tid].cpu().numpy().astype(np.float64) for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C")}
            radi.update(phi=rad["phi"][tid].cpu().numpy().astype(np.float64),
                        xi=rad["xi"][tid].cpu().numpy().astype(np.float64),
                        Neff=rad["N_eff"][tid].cpu().numpy().astype(np.float64))
            st = dict(n=s["n"].ravel()[idx], **state0)
            ref = H.oracle_step(st, radi, dt, par_o)
            g = dict(T=T[tid].cpu().numpy(), xH2=xH2[tid].cpu().numpy(), xHp=xHp[tid].cpu().numpy())
            for k in ("xCp", "xCO", "xe"):
                g[k] = out[k][tid].cpu().numpy().astype(np.float64)
            H.check_mixed_flat(g, ref, idx, xCt, label=f"pts256 ({maps_kind} maps) step {step}")
        xC = (xCt - out["xCp"].double() - out["xCO"].double()).clamp_min(0.0).view(shape)
    assert int((out["status"] & 0xEF).sum().item()) == 0
