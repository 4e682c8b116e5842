"""Operation census of one substep of the source step, taken on the oracle.

Counts numpy ufunc applications on one-cell arrays while the oracle evaluates one
substep (Sec. 6.1): the full evaluation at T, the forward-difference evaluation
at T (1 + fd_rel), the rate coefficients at T^{n+1}, the backward-Euler update
and the equilibrium closure.  Inner iterations are counted at their minimum,
so the figure is a lower bound on the method's work per substep:

* the dust-temperature root counts one residual + derivative evaluation,
* the x_e fixed point of the C/O/e closure counts one pass.

Arithmetic (add, subtract, multiply, divide, negative, absolute, maximum,
minimum, comparisons, sqrt) counts one flop each; transcendentals (exp, log,
log10, power, cbrt, expm1) are counted separately, one per call.
"""
import numpy as np

from . import constants as C
from . import micro, step

ARITH = {"add", "subtract", "multiply", "true_divide", "divide", "negative", "absolute", "maximum", "minimum",
         "greater", "greater_equal", "less", "less_equal", "equal", "not_equal", "sqrt", "square", "fmax",
         "fmin", "floor", "reciprocal", "logical_and", "logical_or", "logical_not", "clip"}
TRANS = {"exp", "log", "log10", "power", "cbrt", "expm1", "exp2", "log2", "float_power"}


class _Counter:
    def __init__(self):
        self.arith = 0
        self.trans = 0
        self.other = {}


class Counted(np.ndarray):
    counter = None

    def __array_ufunc__(self, ufunc, method, *inputs, **kwargs):
        cnt = Counted.counter
        args = [np.asarray(x) if isinstance(x, Counted) else x for x in inputs]
        if "out" in kwargs:
            kwargs["out"] = tuple(np.asarray(o) if isinstance(o, Counted) else o for o in kwargs["out"])
        res = getattr(ufunc, method)(*args, **kwargs)
        if cnt is not None and method == "__call__":
            size = max((np.size(x) for x in args if isinstance(x, np.ndarray)), default=1)
            if ufunc.__name__ in TRANS:
                cnt.trans += size
            elif ufunc.__name__ in ARITH:
                cnt.arith += size
            else:
                cnt.other[ufunc.__name__] = cnt.other.get(ufunc.__name__, 0) + size
        if isinstance(res, np.ndarray):
            return res.view(Counted)
        if isinstance(res, tuple):
            return tuple(r.view(Counted) if isinstance(r, np.ndarray) else r for r in res)
        return res


def _one(v):
    return np.array([float(v)]).view(Counted)


def substep_census(par=None, T=300.0, n=10.0, xH2=0.1, xHp=0.01):
    """Counts (arith, transcendental) for one substep of one cell."""
    par = par or C.Params()
    rad = {k: _one(v) for k, v in dict(chi_PE=1.0, chi_LW=1.0, chi_H2=0.5, chi_C=0.8, phi=0.0, xi=2e-16,
                                          Neff=1e20).items()}
    cnt = _Counter()
    orig_dust, orig_eq = micro.dust_T, micro.eq_species

    def dust_once(T_, n_, G, par_, iters=64):
        A = C.SIGMA_IR10 / 100.0 * C.C_LIGHT * C.A_RAD
        B = n_ * C.ALPHA_GD * np.sqrt(T_)
        Td = T_ * 0.0 + 20.0
        g = A * Td * Td * (Td * Td * Td * Td - par_.T_bb ** 4) - G - B * (T_ - Td)
        dg = A * (6.0 * Td ** 5 - 2.0 * par_.T_bb ** 4 * Td) + B
        Td = Td - g / dg
        return Td, np.zeros(1, bool)

    def eq_once(*a, **k):
        k["maxit"] = 1
        return orig_eq(*a, **k)

    micro.dust_T, micro.eq_species = dust_once, eq_once
    Counted.counter = cnt
    try:
        Tc, nc, x2, xp = _one(T), _one(n), _one(xH2), _one(xHp)
        eq = micro.eq_species(Tc, nc, x2, xp, rad["chi_PE"], rad["chi_LW"], rad["chi_C"], rad["xi"], par)
        cnt.arith = cnt.trans = 0          # the entry closure is per cell, not per substep
        ev = micro.evaluate(Tc, nc, x2, xp, eq, rad, par)
        ev2 = micro.evaluate(Tc * (1.0 + par.fd_rel), nc, x2, xp, eq, rad, par)
        K = nc * par.muH * C.K_B / (C.GAMMA - 1.0)
        dts = np.minimum(1e10, par.eps_sub * K * Tc / np.abs(ev["H"]))
        dH = (ev2["H"] - ev["H"]) / (par.fd_rel * Tc)
        Tn = Tc + dts * ev["H"] / (K - dts * dH)
        evp = micro.evaluate(Tn, nc, x2, xp, eq, rad, par, chem_only=True)
        a, b = step.be_solve(x2, xp, evp["F"], evp["D"], evp["I"], evp["Rr"], dts)
        micro.eq_species(Tn, nc, a, b, rad["chi_PE"], rad["chi_LW"], rad["chi_C"], rad["xi"], par)
    finally:
        Counted.counter = None
        micro.dust_T, micro.eq_species = orig_dust, orig_eq
    return cnt.arith, cnt.trans


if __name__ == "__main__":
    a, t = substep_census()
    print(f"per substep: {a} arithmetic flops, {t} transcendentals")
