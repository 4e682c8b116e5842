"""The subcycled heating/cooling + chemistry source step (Sec. 6.1), FP64.

Algorithm, in the paper's order, per cell and with n and radiation fixed:

1. Equilibrium C/O/e at the input (T, x_H2, x_H+); carried thermal variable
   T_mu = T / mu with mu = mu_H / (1.1 + x_e - x_H2), e = K T_mu,
   K = n mu_H k_B / (gamma - 1) (Eqs. e:ODE1, e:ODE2).
2. Until t = dt:
   a. T from T_mu with the current abundances; evaluate Gamma, Lambda,
      H = n Gamma - n^2 Lambda, C_H2, C_H+.
   b. dt_sub = min(dt - t, 0.1 e/|H|, 0.1/|C_H2|, 0.1/|C_H+|) (Sec. 6.1;
      terms with a zero denominator are skipped).
   c. dH/dT_mu by a forward difference (step fd_rel T_mu) with all
      abundances held and T_d re-solved; T_mu <- T_mu + dt_sub H / (K -
      dt_sub dH/dT_mu), which is the paper's semi-implicit update rewritten.
   d. Rate coefficients at T^{n+1} = mu^n T_mu^{n+1}, with the abundance-
      dependent factors (zeta_cr,H2, n_e, psi's n_e) frozen at step n; the
      linear system dX/dt = A X + b for X = (x_H2, x_H+) advanced by backward
      Euler.
   e. Equilibrium C/O/e recomputed at (T^{n+1}, X^{n+1}).
3. T_out from T_mu with the final abundances.

Guards that the paper does not state (substep cap, T floor, denominator
guard) set status bits and never fire on the configured workloads.
"""
import numpy as np

from . import constants as C
from . import micro

ST_CAP, ST_NAN, ST_TFLOOR, ST_DENOM, ST_FALLBACK, ST_TD = 1, 2, 4, 8, 16, 32

RAD_KEYS = ("chi_PE", "chi_LW", "chi_H2", "chi_C", "phi", "xi", "Neff")


def _sub(d, idx):
    return {k: (v[idx] if np.ndim(v) else v) for k, v in d.items()}


def be_solve(xH2, xHp, F, D, I, Rr, dt):
    """Backward Euler for dX/dt = A X + b, X = (x_H2, x_H+), with x_H = 1 - 2 x_H2 - x_H+.

    A = [[-(2F + D), -F], [-2I, -(I + Rr)]], b = (F, I); X' solves
    (1 - A dt) X' = X + b dt (Sec. 6.1).  Cramer's rule, with the numerators
    multiplied out so that no two large terms cancel:

      det  = 1 + dt (2F + D + I + Rr) + dt^2 (2F Rr + D I + D Rr)
      x_H2' = [x_H2 (1 + dt (I + Rr)) + F dt (1 - x_H+) + F dt^2 Rr] / det
      x_H+' = [x_H+ (1 + dt (2F + D)) + I dt (1 - 2 x_H2) + I dt^2 D] / det

    (expanding (x_H2 + F dt)(1 + dt (I + Rr)) - F dt (x_H+ + I dt) and
    (1 + dt (2F + D))(x_H+ + I dt) - 2 I dt (x_H2 + F dt)).
    """
    det = 1.0 + dt * (2.0 * F + D + I + Rr) + dt * dt * (2.0 * F * Rr + D * I + D * Rr)
    a = (xH2 * (1.0 + dt * (I + Rr)) + F * dt * (1.0 - xHp) + F * dt * dt * Rr) / det
    b = (xHp * (1.0 + dt * (2.0 * F + D)) + I * dt * (1.0 - 2.0 * xH2) + I * dt * dt * D) / det
    return a, b


def chem_cool_step(n, T, xH2, xHp, rad, dt, par, record=None, fd_noise=0.0):
    """Advance every cell by dt [s].  Returns a dict of T, xH2, xHp, xCp, xCO, xe, nsub, status.

    rad: dict of per-cell arrays (or scalars) chi_PE, chi_LW, chi_H2, chi_C,
    phi, xi, Neff.  All FP64.

    fd_noise (conditioning probe, 0 in every comparison): when non-zero, H of the evaluation at
    T (1 + fd_rel) is shifted by fd_noise times its larger term, max(n |Gamma|, n^2 |Lambda|), in
    every substep -- the size of one rounding of that evaluation at relative precision fd_noise.
    """
    n = np.asarray(n, dtype=np.float64).ravel()
    N = n.size
    T = np.broadcast_to(np.asarray(T, dtype=np.float64), (N,)).copy()
    xH2 = np.broadcast_to(np.asarray(xH2, dtype=np.float64), (N,)).copy()
    xHp = np.broadcast_to(np.asarray(xHp, dtype=np.float64), (N,)).copy()
    rad = {k: np.broadcast_to(np.asarray(rad[k], dtype=np.float64), (N,)) for k in RAD_KEYS}
    muH = par.muH
    K = n * muH * C.K_B / (C.GAMMA - 1.0)
    eq = micro.eq_species(T, n, xH2, xHp, rad["chi_PE"], rad["chi_LW"], rad["chi_C"], rad["xi"], par)
    Tmu = T * (1.1 + eq["xe"] - xH2) / muH
    t = np.zeros(N)
    nsub = np.zeros(N, dtype=np.int64)
    status = np.zeros(N, dtype=np.int64)
    done = np.zeros(N, dtype=bool)
    eq = {k: v.copy() for k, v in eq.items()}
    delta = par.fd_rel
    while not done.all():
        a = np.nonzero(~done)[0]
        na, xH2a, xHpa, Tmua, Ka = n[a], xH2[a], xHp[a], Tmu[a], K[a]
        eqa = _sub(eq, a)
        rada = _sub(rad, a)
        mu_den = 1.1 + eqa["xe"] - xH2a
        Ta = muH * Tmua / mu_den
        ev = micro.evaluate(Ta, na, xH2a, xHpa, eqa, rada, par)
        H = ev["H"]
        e = Ka * Tmua
        rem = dt - t[a]
        dts = rem.copy()
        for num, den in ((par.eps_sub * e, np.abs(H)), (par.eps_sub, np.abs(ev["C_H2"])),
                         (par.eps_sub, np.abs(ev["C_Hp"]))):
            nz = den > 0.0
            dts = np.where(nz, np.minimum(dts, num / np.where(nz, den, 1.0)), dts)
        ev2 = micro.evaluate(Ta * (1.0 + delta), na, xH2a, xHpa, eqa, rada, par)
        H2 = ev2["H"]
        if fd_noise:
            H2 = H2 + fd_noise * np.maximum(na * np.abs(ev2["Gamma"]), na * na * np.abs(ev2["Lambda"]))
        dH = (H2 - H) / (delta * Tmua)
        den = Ka - dts * dH
        guard = den <= 0.1 * Ka
        den = np.where(guard, Ka, den)
        st = status[a] | np.where(guard, ST_DENOM, 0) | np.where(ev["Td_bad"] | ev2["Td_bad"], ST_TD, 0)
        Tmu_new = Tmua + dts * H / den
        Tmu_min = par.T_floor * mu_den / muH
        fl = Tmu_new < Tmu_min
        Tmu_new = np.where(fl, Tmu_min, Tmu_new)
        st |= np.where(fl, ST_TFLOOR, 0)
        # abundance update at T^{n+1} = mu^n T_mu^{n+1}, abundance factors frozen at step n
        Tp = muH * Tmu_new / mu_den
        evp = micro.evaluate(Tp, na, xH2a, xHpa, eqa, rada, par, chem_only=True)
        xH2n, xHpn = be_solve(xH2a, xHpa, evp["F"], evp["D"], evp["I"], evp["Rr"], dts)
        eqn = micro.eq_species(Tp, na, xH2n, xHpn, rada["chi_PE"], rada["chi_LW"], rada["chi_C"], rada["xi"], par)
        fin = np.isfinite(Tmu_new) & np.isfinite(xH2n) & np.isfinite(xHpn)
        st |= np.where(fin, 0, ST_NAN)
        last = dts == rem
        tn = np.where(last, dt, t[a] + dts)
        ns = nsub[a] + 1
        cap = (ns >= par.max_substeps) & ~last
        st |= np.where(cap, ST_CAP, 0)
        Tmu[a], xH2[a], xHp[a], t[a], nsub[a], status[a] = Tmu_new, xH2n, xHpn, tn, ns, st
        for k in eq:
            eq[k][a] = eqn[k]
        done[a] = last | cap | ~fin
        if record is not None:
            record(a, dts)
    Tout = muH * Tmu / (1.1 + eq["xe"] - xH2)
    return dict(T=Tout, xH2=xH2, xHp=xHp, xCp=eq["xCp"], xCO=eq["xCO"], xe=eq["xe"], nsub=nsub,
                status=status, xC=eq["xC"], xO=eq["xO"], xOp=eq["xOp"])
