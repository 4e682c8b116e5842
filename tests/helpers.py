"""Shared test helpers: seeded inputs, oracle runs and the relative-error check."""
import numpy as np

from oracle import columns as ocol
from oracle import constants as OC
from oracle import step as ostep

YR = OC.YR

# |a - b| <= tol * max(|b|, floor): floors for near-zero abundances (x_H2, x_H+, x_e: absolute;
# C-bearing species: relative to x_C,tot).
FLOORS_F64 = dict(T=0.0, xH2=1e-10, xHp=1e-10, xe=1e-10, xCp=1e-10, xCO=1e-10)
FLOORS_MIX = dict(T=0.0, xH2=1e-7, xHp=1e-7, xe=1e-7, xCp=1e-7, xCO=1e-7)


def rel_err(a, b, floor=0.0):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def check_fields(gpu, ref, tol, floors, xCt, fields=("T", "xH2", "xHp", "xe", "xCp", "xCO"), label=""):
    report = {}
    for k in fields:
        fl = floors[k] * (xCt if k in ("xCp", "xCO") else 1.0)
        e = rel_err(gpu[k], ref[k], fl)
        report[k] = (float(e.max()), float(np.percentile(e, 99)))
        bad = np.nonzero(e > tol)[0]
        assert bad.size == 0, (f"{label} {k}: {bad.size} cells over {tol}; worst {e.max():.3e} at cell "
                               f"{int(np.argmax(e))}: gpu {np.asarray(gpu[k])[np.argmax(e)]!r} "
                               f"ref {np.asarray(ref[k])[np.argmax(e)]!r}")
    return report


def mixed_rel(a, b, k, xCt):
    """Relative error of one field on the 1e-3 comparison floors (T: none; x_H2, x_H+, x_e: 1e-7;
    C-bearing species: 1e-7 x_C,tot)."""
    fl = FLOORS_MIX[k] * (xCt if k in ("xCp", "xCO") else 1.0)
    return rel_err(a, b, fl)


def oracle_sensitivity(state, rad, dt_s, par, idx, ref, rel=1e-6, fd_noise=1e-7):
    """S per cell: the largest relative change of the oracle's end state (any field, on the 1e-3
    floors) (a) when its input T, x_H2 and x_H+ are all scaled by 1 +- rel, or (b) when, in every
    substep, H of the finite-difference partner evaluation at T (1 + fd_rel) moves by +-fd_noise
    of its larger term -- one float rounding of that evaluation, which the derivative dH/dT_mu
    divides by fd_rel."""
    sens = np.zeros(len(idx))
    for sign in (1.0, -1.0):
        sp = {"n": state["n"]}
        for k in ("T", "xH2", "xHp"):
            sp[k] = state[k] * (1.0 + sign * rel)
        for alt in (oracle_step(sp, rad, dt_s, par, idx=idx),
                    oracle_step(state, rad, dt_s, par, idx=idx, fd_noise=sign * fd_noise)):
            for k in ("T", "xH2", "xHp", "xe", "xCp", "xCO"):
                sens = np.maximum(sens, mixed_rel(alt[k], ref[k], k, par.xCtot))
    return sens


def check_mixed_flat(gpu, ref, idx, xCt, named=None, sens=None, label=""):
    """The chosen form's bar: every sampled cell within 1e-3 in T and every abundance.

    `named` maps a cell index to the reason it is exempt: a cell where the FP64 scheme itself is
    ill-conditioned (its end state moves by S >= 1e-4 for a 1e-6 relative input change or for one
    float rounding of the finite-difference partner evaluation, see oracle_sensitivity), so that a
    float evaluation cannot be held to 1e-3.  A named cell must still show that sensitivity and
    stay within 10 S.  Returns (max error, p99) over the cells and fields."""
    named = named or {}
    worst = np.zeros(len(idx))
    field = np.full(len(idx), "", dtype=object)
    for k in ("T", "xH2", "xHp", "xe", "xCp", "xCO"):
        e = mixed_rel(gpu[k], ref[k], k, xCt)
        field = np.where(e > worst, k, field)
        worst = np.maximum(worst, e)
    over = np.nonzero(worst > 1e-3)[0]
    msg = "; ".join(f"cell {int(idx[i])} {field[i]} {worst[i]:.2e}" +
                    (f" S {sens[i]:.2e}" if sens is not None else "") for i in over[:20])
    print(f"  {label}: max {worst.max():.2e}, p99 {np.percentile(worst, 99):.2e}, "
          f"cells over 1e-3: {over.size} {msg}", flush=True)
    for i in over:
        c = int(idx[i])
        assert c in named, f"{label}: cell {c} over 1e-3 ({field[i]} {worst[i]:.3e}) and not named; {msg}"
        assert sens is not None and sens[i] >= 1e-4, (label, c, "named but not ill-conditioned", sens[i])
        assert worst[i] <= 10.0 * sens[i], (label, c, worst[i], sens[i])
    return float(worst.max()), float(np.percentile(worst, 99))


def oracle_rad(state, dx_cm, par, xC=None):
    r = ocol.columns6(state["n"], state["xH2"], xC, dx_cm, par)
    N = state["n"].size
    return dict(chi_PE=r["chi_PE"].ravel(), chi_LW=r["chi_LW"].ravel(), chi_H2=r["chi_H2"].ravel(),
                chi_C=r["chi_C"].ravel(), phi=np.zeros(N), xi=r["xi"].ravel(), Neff=r["N_eff"].ravel())


def oracle_step(state, rad, dt_s, par, idx=None, fd_noise=0.0):
    sel = (lambda a: a.ravel()) if idx is None else (lambda a: a.ravel()[idx])
    N = np.size(state["n"])
    # radiation may be given for the whole grid or already for the selected cells
    radi = {k: (sel(v) if np.size(v) == N else np.asarray(v).ravel()) for k, v in rad.items()}
    return ostep.chem_cool_step(sel(state["n"]), sel(state["T"]), sel(state["xH2"]), sel(state["xHp"]), radi,
                                dt_s, par, fd_noise=fd_noise)


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a).ravel())
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_rad(rad, dtype):
    return dict(chi_PE=to_dev(rad["chi_PE"], dtype), chi_LW=to_dev(rad["chi_LW"], dtype),
                chi_H2=to_dev(rad["chi_H2"], dtype), chi_C=to_dev(rad["chi_C"], dtype),
                phi=to_dev(rad["phi"], dtype), xi=to_dev(rad["xi"], dtype), N_eff=to_dev(rad["Neff"], dtype))


def ism_params_from(par):
    from paper_2210_08024_amd import ism
    return ism.Params(Zg=par.Zg, Zd=par.Zd, chi0=par.chi0, xi_cr0=par.xi_cr0, cr_mode=par.cr_mode,
                      kgr_const=par.kgr_const, h2_rovib=par.h2_rovib, eps_sub=par.eps_sub, fd_rel=par.fd_rel,
                      max_substeps=par.max_substeps, T_floor=par.T_floor, T_bb=par.T_bb,
                      tau_opt_ratio=par.tau_opt_ratio, dvdr_kms_pc=par.dvdr_kms_pc)


def gpu_step(state, rad, dt_s, par, prec):
    import torch
    from paper_2210_08024_amd import ism
    rd = torch.float64 if prec == ism.F64 else torch.float32
    n = to_dev(state["n"])
    T = to_dev(state["T"])
    xH2 = to_dev(state["xH2"])
    xHp = to_dev(state["xHp"])
    out = ism.chem_cool_step(n, T, xH2, xHp, gpu_rad(rad, rd), dt_s, ism_params_from(par), prec)
    torch.cuda.synchronize()
    res = dict(T=T.cpu().numpy(), xH2=xH2.cpu().numpy(), xHp=xHp.cpu().numpy())
    for k, v in out.items():
        res[k] = v.cpu().numpy()
    return res
