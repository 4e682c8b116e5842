"""ism_chem_cool_step_noalloc against ism_chem_cool_step: the same inputs through both entry
points give bitwise the same cell state and outputs, on two calls in a row (the whole 128^3 grid,
then a smaller, ragged set of cells that reuses the first call's scratch), in both precisions and
ordering modes; and a call beyond the ordered-cell limit is rejected before any work."""
import ctypes

import numpy as np
import pytest

import helpers as H
from oracle import constants as OC
from oracle.constants import Params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ism():
    import torch
    from paper_2210_08024_amd import ism as m
    torch.cuda.set_device(0)
    m.init(0)
    return m


def _outs(torch, N, prec):
    rd = torch.float64 if prec == 0 else torch.float32
    return {"xCp": torch.empty(N, dtype=rd, device="cuda"), "xCO": torch.empty(N, dtype=rd, device="cuda"),
            "xe": torch.empty(N, dtype=rd, device="cuda"), "nsub": torch.zeros(N, dtype=torch.int32, device="cuda"),
            "status": torch.empty(N, dtype=torch.uint8, device="cuda")}


@pytest.mark.parametrize("prec,order", [(0, 1), (1, 1), (1, 0)])
def test_noalloc_matches_the_allocating_step(ism, prec, order):
    import torch
    from paper_2210_08024_amd import workloads
    s, cfg = workloads.make("grf128")
    shape = s["n"].shape
    N = s["n"].size
    par = H.ism_params_from(Params(cr_mode=1))
    par.order_cells = order
    dx = cfg["dx_pc"] * OC.PC
    dt = cfg["dt_yr"] * OC.YR
    n = H.to_dev(s["n"])
    rad = {k: v.view(-1) for k, v in ism.columns6(n.view(shape), H.to_dev(s["xH2"]).view(shape), None, dx, par,
                                                   prec).items()}
    rad["phi"] = None
    init = {k: H.to_dev(s[k]) for k in ("T", "xH2", "xHp")}
    rng = np.random.default_rng(9)
    small = torch.from_numpy(np.sort(rng.choice(N, 100_003, replace=False))).cuda()
    for label, sel in (("whole grid", None), ("100,003 cells", small)):
        print(f"noalloc prec {prec} order {order}: {label}", flush=True)
        pick = (lambda a: a.clone()) if sel is None else (lambda a: a[sel].contiguous())
        nn = pick(n)
        rd = {k: (None if v is None else pick(v)) for k, v in rad.items()}
        res = {}
        for fn in (ism.chem_cool_step, ism.chem_cool_step_noalloc):
            T, a, b = (pick(init[k]) for k in ("T", "xH2", "xHp"))
            out = _outs(torch, nn.numel(), prec)
            fn(nn, T, a, b, rd, dt, par, prec, out=out)
            torch.cuda.synchronize()
            out.update(T=T, xH2=a, xHp=b)
            res[fn.__name__] = out
        ref, got = res["chem_cool_step"], res["chem_cool_step_noalloc"]
        for k in ref:
            assert bool((ref[k] == got[k]).all()), f"{label}: {k} differs"
        assert int((got["status"] & 0xEF).sum()) == 0


def test_noalloc_rejects_more_ordered_cells_than_its_scratch_holds(ism):
    import torch
    from paper_2210_08024_amd.ism import _Params, lib
    M = (1 << 23) + 1
    # real buffers of M cells, so that nothing could read out of bounds even if the check failed
    d = [torch.ones(M, dtype=torch.float64, device="cuda") for _ in range(11)]
    o = [torch.empty(M, dtype=torch.float64, device="cuda") for _ in range(3)]
    ns = torch.zeros(M, dtype=torch.int32, device="cuda")
    st = torch.empty(M, dtype=torch.uint8, device="cuda")
    p = H.ism_params_from(Params())
    p.order_cells = 1
    c = p._c()
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = lib().ism_chem_cool_step_noalloc(ctypes.byref(c), 0, M, ctypes.c_double(3.15576e11), *[vp(t) for t in d],
                                          *[vp(t) for t in o], vp(ns), vp(st),
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -1
    assert b"at most" in lib().ism_last_error()
