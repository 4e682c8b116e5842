"""Concurrent calls on two streams.  Library scratch belongs to the (device, stream) a call is
enqueued on, so calls on different streams may overlap; each must give exactly the result it
gives alone.  On the 128^3 GRF grid: the six-ray columns of the lower and upper halves (along z,
as two grids), then the source step of the two halves of the cells (every ordering mode, both
precisions) and the surrogate step, each pair launched on two streams without waiting in
between, against the same calls made one after the other on one stream.  Bitwise."""
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


@pytest.fixture(scope="module")
def grf128():
    from paper_2210_08024_amd import workloads
    return workloads.make("grf128")


def _pairs(torch, fn, concurrent):
    """Run fn(0, stream) and fn(1, stream) on two streams (concurrent) or on one stream in turn."""
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    outs = []
    for h, st in enumerate((s1, s2) if concurrent else (s1, s1)):
        with torch.cuda.stream(st):
            outs.append(fn(h, st))
    torch.cuda.synchronize()
    return outs


def _eq(a, b, label):
    for k in a:
        if a[k] is None:
            continue
        assert a[k].shape == b[k].shape and bool((a[k] == b[k]).all()), f"{label}: {k} differs"


@pytest.mark.parametrize("prec", [0, 1])
def test_columns_on_two_streams(ism, grf128, prec):
    import torch
    s, cfg = grf128
    print(f"columns6 on two streams, prec {prec}", flush=True)
    nz = s["n"].shape[0]
    par = H.ism_params_from(Params(cr_mode=1))
    dx = cfg["dx_pc"] * OC.PC
    halves = [slice(0, nz // 2), slice(nz // 2, nz)]
    n = [H.to_dev(s["n"][h]).view(s["n"][h].shape) for h in halves]
    x2 = [H.to_dev(s["xH2"][h]).view(s["n"][h].shape) for h in halves]

    def fn(h, st):
        out = ism.columns6(n[h], x2[h], None, dx, par, prec, stream=st)
        return {k: v.clone() for k, v in out.items()}

    ser = _pairs(torch, fn, False)
    con = _pairs(torch, fn, True)
    for h in (0, 1):
        _eq(ser[h], con[h], f"columns6 half {h}")


@pytest.mark.parametrize("prec,order", [(0, 1), (1, 1), (1, 2), (1, 0)])
def test_step_on_two_streams(ism, grf128, prec, order):
    import torch
    s, cfg = grf128
    print(f"step on two streams, prec {prec}, order_cells {order}", flush=True)
    shape = s["n"].shape
    N = s["n"].size
    par = H.ism_params_from(Params(cr_mode=1))
    par.order_cells = order
    dx = cfg["dx_pc"] * OC.PC
    dt = cfg["dt_yr"] * OC.YR
    n = H.to_dev(s["n"])
    xH2 = H.to_dev(s["xH2"])
    rad = {k: v.view(-1) for k, v in ism.columns6(n.view(shape), xH2.view(shape), None, dx, par, prec).items()}
    rad["phi"] = None
    halves = [slice(0, N // 2), slice(N // 2, N)]
    init = {k: H.to_dev(s[k]) for k in ("T", "xH2", "xHp")}
    # order_cells 2 reads the counts of a previous step from nsub: give each half some
    nsub0 = torch.randint(1, 40, (N,), dtype=torch.int32, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    torch.cuda.synchronize()

    rdt = torch.float64 if prec == 0 else torch.float32

    def outputs(sl):
        m = sl.stop - sl.start
        return {"xCp": torch.empty(m, dtype=rdt, device="cuda"), "xCO": torch.empty(m, dtype=rdt, device="cuda"),
                "xe": torch.empty(m, dtype=rdt, device="cuda"), "nsub": nsub0[sl].clone(),
                "status": torch.empty(m, dtype=torch.uint8, device="cuda")}

    def fn(h, st):
        sl = halves[h]
        T, a, b = (init[k][sl].clone() for k in ("T", "xH2", "xHp"))
        rd = {k: (None if v is None else v[sl]) for k, v in rad.items()}
        res = ism.chem_cool_step(n[sl], T, a, b, rd, dt, par, prec, out=outputs(sl), stream=st)
        res.update(T=T, xH2=a, xHp=b)
        return res

    ser = _pairs(torch, fn, False)
    con = _pairs(torch, fn, True)
    for h in (0, 1):
        _eq(ser[h], con[h], f"step half {h}")
    # and the halves together equal the whole grid in one call (results do not depend on order)
    T, a, b = (init[k].clone() for k in ("T", "xH2", "xHp"))
    whole = ism.chem_cool_step(n, T, a, b, rad, dt, par, prec, out=outputs(slice(0, N)))
    torch.cuda.synchronize()
    for k, v in (("T", T), ("xH2", a), ("xHp", b), ("xe", whole["xe"])):
        joined = torch.cat([ser[0][k], ser[1][k]])
        assert bool((joined == v).all()), f"halves vs whole grid: {k}"


def test_surrogate_step_on_two_streams(ism, grf128):
    import torch
    from paper_2210_08024_amd import surrogate_train
    s, cfg = grf128
    print("surrogate step on two streams", flush=True)
    shape = s["n"].shape
    N = s["n"].size
    par = H.ism_params_from(Params(cr_mode=1))
    dx = cfg["dx_pc"] * OC.PC
    dt = cfg["dt_yr"] * OC.YR
    n = H.to_dev(s["n"])
    xH2 = H.to_dev(s["xH2"])
    rad = {k: v.view(-1) for k, v in ism.columns6(n.view(shape), xH2.view(shape), None, dx, par, 1).items()}
    rad["phi"] = None
    halves = [slice(0, N // 2), slice(N // 2, N)]
    init = {k: H.to_dev(s[k]) for k in ("T", "xH2", "xHp")}
    sur = surrogate_train.load()
    torch.cuda.synchronize()

    def fn(h, st):
        sl = halves[h]
        T, a, b = (init[k][sl].clone() for k in ("T", "xH2", "xHp"))
        rd = {k: (None if v is None else v[sl]) for k, v in rad.items()}
        nfb = torch.zeros(1, dtype=torch.int64, device="cuda")
        res = ism.chem_cool_step_surrogate(sur, n[sl], T, a, b, rd, dt, par, n_fallback=nfb, stream=st)
        res.update(T=T, xH2=a, xHp=b, nfb=nfb)
        return res

    ser = _pairs(torch, fn, False)
    con = _pairs(torch, fn, True)
    for h in (0, 1):
        _eq(ser[h], con[h], f"surrogate step half {h}")
