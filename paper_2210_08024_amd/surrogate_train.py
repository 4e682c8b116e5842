"""Training of the source-step surrogate on pairs that the plain FP64 GPU step generates.

Data: for each workload recipe (i.i.d. cells of the small configuration, the lognormal GRF
cube, optically thin cells), metallicity and step length, the plain FP64 step advances the
cells on the GPU; ``ism_surrogate_pairs`` turns (pre-step state, radiation, Z', dt) and the
post-step state into network inputs and targets.  Training: standardised inputs and targets,
MSE, Adam with a cosine learning-rate decay, all on the GPU through ``ism_surrogate_train_step``.

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
)


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


def pairs_for(recipe, size, Zg, dt_yr, salt=0):
    """(X, Y) float32 device tensors from one plain FP64 step of a seeded workload."""
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


def dataset(specs=DEFAULT_SPECS, samples=None, seed=0, log=print):
    """Concatenated pairs of every (recipe, Z', dt) in specs, shuffled, optionally cut to `samples`."""
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
    g = torch.Generator(device="cuda").manual_seed(seed)
    perm = torch.randperm(X.shape[0], device="cuda", generator=g)
    if samples is not None:
        perm = perm[:samples]
    return X[perm].contiguous(), Y[perm].contiguous()


def fit(X, Y, steps=20000, batch=65536, lr0=1e-3, lr1=1e-5, seed=0, val_frac=0.1, log=print, log_every=1000):
    """Train a surrogate on (X, Y); returns (surrogate, history of (step, train loss, val loss))."""
    N = X.shape[0]
    nval = max(1, int(val_frac * N))
    Xv, Yv, Xt, Yt = X[:nval], Y[:nval], X[nval:], Y[nval:]
    mu_x, sd_x = Xt.mean(0), Xt.std(0).clamp_min(1e-6)
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
