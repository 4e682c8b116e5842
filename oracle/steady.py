"""Independent steady states of the one-zone source terms, by brute force.

A steady state is a temperature T and abundances X = (x_H2, x_H+) with
H(T, X) = 0, C_H2 = 0 and C_H+ = 0 and the C/O/e closure consistent
(the paper finds its equilibrium curves by root finding on thermal and
ionisation balance, Secs. 4.6.6 and 7.1.1).

Method (no use of the subcycled step):
* for each T on a fine log grid, the chemical equilibrium X_eq(T) is the fixed
  point of X = -A(X)^{-1} b(X), whose closed form at frozen coefficients is
  x_H = 1 / (1 + 2F/D + I/Rr), x_H2 = F x_H / D, x_H+ = I x_H / Rr;
* sign changes of h(T) = H(T, X_eq(T)) are bisected;
* a root is stable where h goes from positive to negative with increasing T.

Only roots where h is continuous (|h| tiny relative to n Gamma at the root)
are reported: the cold/hot electron switch at 2e4 K makes h jump.
"""
import numpy as np

from . import micro


def chem_equilibrium(T, n, rad, par, tol=1e-14, maxit=500):
    T = np.asarray(T, dtype=np.float64)
    shape = T.shape
    xH2 = np.full(shape, 0.1)
    xHp = np.full(shape, 0.1)
    for _ in range(maxit):
        eq = micro.eq_species(T, n, xH2, xHp, rad["chi_PE"], rad["chi_LW"], rad["chi_C"], rad["xi"], par)
        ev = micro.evaluate(T, n, xH2, xHp, eq, rad, par, chem_only=True)
        F, D, I, Rr = ev["F"], ev["D"], ev["I"], ev["Rr"]
        xH = 1.0 / (1.0 + 2.0 * F / D + I / Rr)
        nH2 = F * xH / D
        nHp = I * xH / Rr
        # damping keeps the iteration on x_e-dependent rates from oscillating
        nH2 = 0.5 * (nH2 + xH2)
        nHp = 0.5 * (nHp + xHp)
        err = max(np.max(np.abs(nH2 - xH2) / np.maximum(nH2, 1e-300)),
                  np.max(np.abs(nHp - xHp) / np.maximum(nHp, 1e-300)))
        xH2, xHp = nH2, nHp
        if err < tol:
            break
    eq = micro.eq_species(T, n, xH2, xHp, rad["chi_PE"], rad["chi_LW"], rad["chi_C"], rad["xi"], par)
    return xH2, xHp, eq


def h_of_T(T, n, rad, par):
    xH2, xHp, eq = chem_equilibrium(T, n, rad, par)
    ev = micro.evaluate(T, n, xH2, xHp, eq, rad, par)
    return ev["H"], ev["Gamma"] * n, xH2, xHp, eq


def steady_states(n, rad, par, lo=0.0, hi=9.0, npts=4000, iters=60):
    """All continuous roots of h(T) on [10^lo, 10^hi] K.  Returns list of (T, stable, xH2, xHp, eq)."""
    Tg = np.logspace(lo, hi, npts)
    radg = {k: np.full(npts, v) for k, v in rad.items()}
    h, g, _, _, _ = h_of_T(Tg, n, radg, par)
    s = np.sign(h)
    idx = np.nonzero(s[:-1] * s[1:] < 0)[0]
    roots = []
    for i in idx:
        a, b = Tg[i], Tg[i + 1]
        ha = h[i]
        one = {k: np.array([v]) for k, v in rad.items()}
        for _ in range(iters):
            m = np.sqrt(a * b)
            hm = h_of_T(np.array([m]), n, one, par)[0][0]
            if np.sign(hm) == np.sign(ha):
                a, ha = m, hm
            else:
                b = m
        Tr = np.sqrt(a * b)
        hr, gr, xH2, xHp, eq = h_of_T(np.array([Tr]), n, one, par)
        if abs(hr[0]) <= 1e-6 * abs(gr[0]):
            roots.append((Tr, h[i] > 0, xH2[0], xHp[0], {k: v[0] for k, v in eq.items()}))
    return roots
