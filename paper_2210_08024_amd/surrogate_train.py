"""Training of the source-step surrogate on pairs that the plain FP64 GPU step generates.

Data: for each workload recipe (i.i.d. cells of the small configuration, the lognormal GRF
cube, optically thin cells, the 256^3 grid with point sources and a CR map), metallicity and step
length, the plain FP64 step advances the cells on the GPU; ``ism_surrogate_pairs`` turns
(pre-step state, radiation, Z', dt) and the post-step state into network inputs and targets; the
training set is drawn from all pairs stratified in (log n, log T).  Training: standardised inputs
(spreads floored at 0.1) and targets, MSE, Adam with a cosine learning-rate decay, all on the GPU
through ``ism_surrogate_train_step``.

    python -m paper_2210_08024_amd.surrogate_train [--samples 16777216] [--steps 20000]
        [--batch 65536] [--out data/surrogate.npy]
"""
import argparse
import math
import os
import sys
import time

import numpy as np
import torch

from . import ism, workloads

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CKPT_PATH = os.path.join(ROOT, "data", "surrogate.npy")
YR = workloads.YR
PC = workloads.PC

# (recipe, grid or cell count, metallicities, step lengths in yr)
DEFAULT_SPECS = (
    ("tiny16", 16, (0.1, 1.0, 3.0), (1e3, 1e4, 1e5)),
    ("grf128", 128, (0.1, 1.0, 3.0), (1e3, 1e4, 1e5)),
    ("thin", 1 << 20, (1.0,), (1e4, 1e5, 1e6)),
    # the 256^3 grid with 16 point sources (EUV near the sources) and the per-cell CR map: the
    # first two steps of 1e4 yr, so that the 512^3 configuration's inputs are covered
    ("pts256", 256, (1.0,), (1e4,)),
)
# standardisation: a feature's spread is floored (log features in dex, abundances linear), so a
# feature that barely varies in the data cannot blow up inputs outside it
SD_FLOOR = 0.1
# stratification of the pairs in (log10 n, log10 T): bins of 0.5 dex over these ranges
STRAT_N = (-3.0, 6.0)
STRAT_T = (0.0, 8.0)


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a).ravel()).to(device="cuda", dtype=dtype)


def _grid_radiation(state, dx_cm, par):
    shape = state["n"].shape
    N = state["n"].size
    n = _dev(state["n"]).view(shape)
    xH2 = _dev(state["xH2"]).view(shape)
    rad = {k: torch.empty(N, dtype=torch.float64, device="cuda") for k in
           ("chi_PE", "chi_LW", "chi_H2", "chi_C", "N_eff", "xi")}
    ism.columns6(n, xH2, None, dx_cm, par, ism.F64, out={k: v.view(shape) for k, v in rad.items()})
    return rad


_STATES = {}


def _state(recipe, size, salt):
    key = (recipe, size, salt)
    if key not in _STATES:
        if recipe == "thin":
            _STATES[key] = workloads.thin(size, salt=2 + salt)
        elif recipe.startswith("tiny"):
            s = workloads.tiny(size ** 3, salt=salt)
            _STATES[key] = ({k: v.reshape(size, size, size) for k, v in s.items()}, None)
        else:
            _STATES[key] = (workloads.grf_cube(size, 4.0, salt=1 + salt), None)
    return _STATES[key]


def pairs_pts256(dt_yr, steps=2):
    """(X, Y) from the first `steps` plain FP64 steps of the 256^3 point-source grid: straight-line
    source maps from the initial state (the configuration's recipe), six-ray columns every step
    with x_C fed back, per-cell CR map."""
    s, cfg = workloads.make("pts256")
    shape = s["n"].shape
    N = s["n"].size
    dx = cfg["dx_pc"] * PC
    par = ism.Params(Zg=1.0, Zd=1.0, cr_mode=2)
    n = _dev(s["n"])
    T, xH2, xHp = _dev(s["T"]), _dev(s["xH2"]), _dev(s["xHp"])
    maps = {k: torch.zeros(N, dtype=torch.float64, device="cuda") for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "phi")}
    ism.point_sources(n.view(shape), xH2.view(shape), None, dx, par, ism.F64, cfg["sources"],
                      {k: v.view(shape) for k, v in maps.items()})
    xi = _dev(s["xi"])
    xC = None
    Xs, Ys = [], []
    xCt = 1.6e-4
    for _ in range(steps):
        rad = {k: torch.empty(N, dtype=torch.float64, device="cuda") for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C", "N_eff")}
        rad["xi"] = xi.clone()
        ism.columns6(n.view(shape), xH2.view(shape), xC, dx, par, ism.F64, out={k: v.view(shape) for k, v in rad.items()})
        for k in ("chi_PE", "chi_LW", "chi_H2", "chi_C"):
            rad[k] += maps[k]
        rad["phi"] = maps["phi"]
        T1, x21, xp1 = T.clone(), xH2.clone(), xHp.clone()
        out = ism.chem_cool_step(n, T1, x21, xp1, rad, dt_yr * YR, par, ism.F64, want=("xCp", "xCO"))
        X, Y = ism.surrogate_pairs(n, T, xH2, xHp, rad, dt_yr * YR, par, ism.F64, post=dict(T=T1, xH2=x21, xHp=xp1))
        Xs.append(X)
        Ys.append(Y)
        T, xH2, xHp = T1, x21, xp1
        xC = (xCt - out["xCp"] - out["xCO"]).clamp_min(0.0).view(shape)
    return torch.cat(Xs), torch.cat(Ys)


def pairs_for(recipe, size, Zg, dt_yr, salt=0):
    """(X, Y) float32 device tensors from one plain FP64 step of a seeded workload."""
    if recipe == "pts256":
        return pairs_pts256(dt_yr)
    st, r = _state(recipe, size, salt)
    if recipe == "thin":
        rad = {"chi_PE": _dev(r["chi_PE"]), "chi_LW": _dev(r["chi_LW"]), "chi_H2": _dev(r["chi_H2"]),
               "chi_C": _dev(r["chi_C"]), "phi": _dev(r["phi"]), "xi": _dev(r["xi"]), "N_eff": _dev(r["Neff"])}
        par = ism.Params(Zg=Zg, Zd=Zg, cr_mode=0)
    else:
        cr_mode, dx_pc = (0, 2.0) if recipe.startswith("tiny") else (1, 4.0)
        par = ism.Params(Zg=Zg, Zd=Zg, cr_mode=cr_mode)
        rad = _grid_radiation(st, dx_pc * PC, par)
    n = _dev(st["n"])
    T0, x20, xp0 = _dev(st["T"]), _dev(st["xH2"]), _dev(st["xHp"])
    T1, x21, xp1 = T0.clone(), x20.clone(), xp0.clone()
    ism.chem_cool_step(n, T1, x21, xp1, rad, dt_yr * YR, par, ism.F64, want=())
    X, Y = ism.surrogate_pairs(n, T0, x20, xp0, rad, dt_yr * YR, par, ism.F64,
                               post=dict(T=T1, xH2=x21, xHp=xp1))
    return X, Y


def stratified(X, n_out, seed=0):
    """Indices of n_out pairs drawn stratified in (log10 n, log10 T) (input columns 0 and 1): equal
    shares of the 0.5-dex bins that hold pairs (all of a bin's pairs when it holds fewer), the
    remainder uniformly from the pairs not yet drawn."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    nb_n = int(round((STRAT_N[1] - STRAT_N[0]) / 0.5))
    nb_T = int(round((STRAT_T[1] - STRAT_T[0]) / 0.5))
    bn = ((X[:, 0] - STRAT_N[0]) / 0.5).floor().clamp(0, nb_n - 1).long()
    bT = ((X[:, 1] - STRAT_T[0]) / 0.5).floor().clamp(0, nb_T - 1).long()
    b = bn * nb_T + bT
    # random order, then a stable sort by bin: each bin's pairs in random order, contiguous
    perm = torch.randperm(X.shape[0], device="cuda", generator=g)
    order = perm[torch.sort(b[perm], stable=True).indices]
    counts = torch.bincount(b, minlength=nb_n * nb_T)
    starts = torch.cumsum(counts, 0) - counts
    filled = int((counts > 0).sum())
    quota = max(1, n_out // max(filled, 1))
    take = torch.clamp(counts, max=quota)
    rank = torch.arange(X.shape[0], device="cuda") - starts[b[order]]
    chosen = order[rank < take[b[order]]]
    if chosen.numel() < n_out:
        mask = torch.ones(X.shape[0], dtype=torch.bool, device="cuda")
        mask[chosen] = False
        rest = torch.nonzero(mask).squeeze(1)
        rest = rest[torch.randperm(rest.numel(), device="cuda", generator=g)[:n_out - chosen.numel()]]
        chosen = torch.cat([chosen, rest])
    return chosen[torch.randperm(chosen.numel(), device="cuda", generator=g)][:n_out]


def dataset(specs=DEFAULT_SPECS, samples=None, seed=0, log=print):
    """Pairs of every (recipe, Z', dt) in specs, drawn stratified in (log n, log T) down to
    `samples` (all of them, shuffled, when samples is None)."""
    Xs, Ys = [], []
    for recipe, size, Zs, dts in specs:
        for Zg in Zs:
            for dt in dts:
                t0 = time.time()
                X, Y = pairs_for(recipe, size, Zg, dt)
                ok = torch.isfinite(X).all(1) & torch.isfinite(Y).all(1)
                Xs.append(X[ok])
                Ys.append(Y[ok])
                log(f"  pairs {recipe} Z'={Zg:g} dt={dt:.0e} yr: {int(ok.sum())} ({time.time() - t0:.1f} s)")
    X = torch.cat(Xs)
    Y = torch.cat(Ys)
    del Xs, Ys
    if samples is None:
        g = torch.Generator(device="cuda").manual_seed(seed)
        idx = torch.randperm(X.shape[0], device="cuda", generator=g)
    else:
        idx = stratified(X, min(samples, X.shape[0]), seed)
    return X[idx].contiguous(), Y[idx].contiguous()


def fit(X, Y, steps=20000, batch=65536, lr0=1e-3, lr1=1e-5, seed=0, val_frac=0.1, log=print, log_every=1000):
    """Train a surrogate on (X, Y); returns (surrogate, history of (step, train loss, val loss))."""
    N = X.shape[0]
    nval = max(1, int(val_frac * N))
    Xv, Yv, Xt, Yt = X[:nval], Y[:nval], X[nval:], Y[nval:]
    mu_x, sd_x = Xt.mean(0), Xt.std(0).clamp_min(SD_FLOOR)
    mu_y, sd_y = Yt.mean(0), Yt.std(0).clamp_min(1e-6)
    s = ism.Surrogate(seed=seed)
    s.set_norm(mu_x.tolist(), sd_x.tolist(), mu_y.tolist(), sd_y.tolist())
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ntr = Xt.shape[0]
    batch = min(batch, ntr)
    nb = ntr // batch
    hist = []
    t0 = time.time()
    for k in range(steps):
        lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * k / max(steps - 1, 1)))
        b = k % nb
        s.train_step(Xt[b * batch:(b + 1) * batch], Yt[b * batch:(b + 1) * batch], lr, loss)
        if (k + 1) % log_every == 0 or k + 1 == steps:
            vl = val_loss(s, Xv, Yv, mu_y, sd_y)
            hist.append((k + 1, loss.item(), vl))
            log(f"  step {k + 1}: train {hist[-1][1]:.3e}  val {vl:.3e}  ({time.time() - t0:.1f} s)")
    return s, hist


def val_loss(s, Xv, Yv, mu_y, sd_y):
    P = s.forward(Xv)
    return float((((P - Yv) / sd_y) ** 2).mean().item())


def save(s, path=CKPT_PATH):
    np.save(path, s.get_params(), allow_pickle=False)


def load(path=CKPT_PATH, seed=0):
    s = ism.Surrogate(seed=seed)
    s.set_params(np.load(path, allow_pickle=False))
    return s


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--samples", type=int, default=1 << 24)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--out", default=CKPT_PATH)
    a = ap.parse_args(argv)
    torch.cuda.set_device(0)
    ism.init(0)
    t0 = time.time()
    X, Y = dataset(samples=a.samples)
    print(f"dataset: {X.shape[0]} pairs ({time.time() - t0:.1f} s)", flush=True)
    s, hist = fit(X, Y, steps=a.steps, batch=a.batch, log=lambda m: print(m, flush=True))
    save(s, a.out)
    print(f"saved {a.out}; final train {hist[-1][1]:.3e} val {hist[-1][2]:.3e}", flush=True)


if __name__ == "__main__":
    sys.exit(main())
