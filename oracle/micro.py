"""Microphysics of the source step, FP64, written from the paper.

Every function takes numpy arrays (broadcastable) and returns FP64 arrays.
Citations name the paper's section / equation.  Terms built from stand-in
coefficients (processes the paper only cites; see the coefficient file's
``standin`` section) are marked "stand-in": for those the oracle is
"parity unpinned" beyond agreement with the HIP path.
"""
import numpy as np

from . import constants as C

LN10 = np.log(10.0)


def _sd():
    return C.standins()


# --------------------------------------------------------------------------
# table interpolation (stand-in tables; the rule is part of the definition)
# --------------------------------------------------------------------------
def _axis_pos(ax, x):
    """Clamp x to the axis grid; return (lower index, fraction)."""
    n, x0, dx = ax["n"], ax["x0"], ax["dx"]
    u = (np.clip(x, x0, x0 + (n - 1) * dx) - x0) / dx
    i = np.minimum(np.floor(u).astype(np.int64), n - 2)
    return i, u - i


def table1d(name, x, col):
    axes, vals = _sd().tables[name]
    i, f = _axis_pos(axes[0], x)
    return vals[i, col] * (1.0 - f) + vals[i + 1, col] * f


def table2d(name, x, y, col):
    axes, vals = _sd().tables[name]
    i, f = _axis_pos(axes[0], x)
    j, g = _axis_pos(axes[1], y)
    v00, v01 = vals[i, j, col], vals[i, j + 1, col]
    v10, v11 = vals[i + 1, j, col], vals[i + 1, j + 1, col]
    return (v00 * (1.0 - g) + v01 * g) * (1.0 - f) + (v10 * (1.0 - g) + v11 * g) * f


# --------------------------------------------------------------------------
# rate coefficients (Sec. 3)
# --------------------------------------------------------------------------
def k_gr(T, Zd, kgr_const):
    """Grain H2 formation, Eq. e:H2form (or the constant 3e-17 Z'_d of Sec. 7)."""
    T = np.asarray(T, dtype=np.float64)
    if kgr_const:
        return C.KGR0 * Zd * np.ones_like(T)
    T2 = T / 100.0
    s = np.sqrt(T2)
    return C.KGR0 * Zd * 2.0 * s / (1.0 + 0.4 * s + 0.2 * T2 + 0.08 * T2 * T2)


def alpha_B(T):
    """Case-B H+ radiative recombination (Sec. 3.1.2) -- stand-in."""
    a0, a1, a2 = _sd()["alpha_B"]
    T4 = T / 1.0e4
    return a0 * T4 ** (a1 + a2 * np.log(T4))


def k_ci_H(T):
    """Collisional ionisation of H by electrons (Sec. 3.1.2) -- stand-in."""
    k0, TH, Tc = _sd()["k_ci_H"]
    return k0 * np.sqrt(T) * np.exp(-TH / T) / (1.0 + np.sqrt(T / Tc))


def k_cd_H(T):
    """H2 collisional dissociation by H (Sec. 3.1.1) -- stand-in."""
    k0, TH = _sd()["k_cd_H"]
    return k0 * np.sqrt(T) * np.exp(-(1.0 + TH / T))


def k_cd_H2(T):
    """H2 collisional dissociation by H2 (Sec. 3.1.1) -- stand-in."""
    k0, p, b, q, TH = _sd()["k_cd_H2"]
    return k0 * T ** p * (1.0 + b * T) ** (-q) * np.exp(-TH / T)


def alpha_gr(T, psi, coef, Zd):
    """Grain-assisted recombination (Secs. 3.1.2, 3.2.1) -- stand-in (WD01c form)."""
    c0, c1, c2, c3, c4, c5, c6 = coef
    return 1.0e-14 * c0 * Zd / (1.0 + c1 * psi ** c2 * (1.0 + c3 * T ** c4 * psi ** (-c5 - c6 * np.log(T))))


def alpha_rrdr_Cp(T):
    """C+ radiative + dielectronic recombination (Sec. 3.2.1) -- stand-in."""
    a0, T0, p = _sd()["alpha_rrdr_Cp"]
    return a0 * (T / T0) ** p


def k_CpH2(T):
    """C+ + H2 -> CH2+ (Sec. 3.2.1) -- stand-in."""
    k0, p, TH = _sd()["k_CpH2"]
    return k0 * T ** p * np.exp(-TH / T)


def k_H2_H(T):
    k0, TH = _sd()["k_H2_H"]
    return k0 * np.sqrt(T) * np.exp(-TH / T)


def k_H2_H2(T):
    k0, TH, Ts = _sd()["k_H2_H2"]
    return k0 * np.sqrt(T) * np.exp(-TH / (T + Ts))


def x_MH(T, n, xH2, xi):
    """Molecular-ion electrons (Eq. e:xEL term x_MH+, times 2 x_H2) -- stand-in."""
    c, a0, T0, p = _sd()["x_MH"]
    return 2.0 * xH2 * np.sqrt(c * xi / (a0 * (T / T0) ** p * n))


def chi_fuv(chi_PE, chi_LW):
    """Eq. e:chi_FUV with J_PE = J^D_PE chi_PE, J_LW = J^D_LW chi_LW."""
    return (C.J_PE * chi_PE + C.J_LW * chi_LW) / C.J_FUV


def psi_charge(T, n, xe, chi_PE, chi_LW):
    """Grain charging parameter G0 T^1/2 / n_e plus 50 (Sec. 4.2).

    n_e is floored at 1e-20 n so that psi stays finite in fully neutral,
    unirradiated gas (a guard; never active on ionised or irradiated gas).
    """
    G0 = C.G0_PER_CHI * chi_fuv(chi_PE, chi_LW)
    return G0 * np.sqrt(T) / (n * np.maximum(xe, 1.0e-20)) + C.PSI_OFFSET


# --------------------------------------------------------------------------
# equilibrium C / O / electron closure (Secs. 3.2-3.3)
# --------------------------------------------------------------------------
def eq_species(T, n, xH2, xHp, chi_PE, chi_LW, chi_C, xi, par, tol=1.0e-12, maxit=50):
    """x_C+, x_CO, x_C, x_O+, x_O, x_e in formation-destruction balance.

    O+: x_O+ / x_O,tot = x_H+ (Sec. 3.2.2).  C+: Eq. eq:C+_frac with
    n_e = n (x_e0 + x_C+) solved as the positive root of the quadratic for
    T < 2e4 K (Eq. e:xEL), iterating the psi dependence of the grain
    recombination to a fixed point in x_e; for T >= 2e4 K x_e follows
    Eq. e:xELhot and x_C+ is linear in x_C,tot.  CO: Eqs. e:CO, e:CO_fit
    with chi_CO = chi_LW.  C and O by conservation.
    """
    sd = _sd()
    T = np.asarray(T, dtype=np.float64)
    shape = np.broadcast(T, n, xH2, xHp, chi_PE, chi_LW, chi_C, xi).shape
    T, n, xH2, xHp, chi_PE, chi_LW, chi_C, xi = (np.broadcast_to(np.asarray(a, dtype=np.float64), shape)
                                                 for a in (T, n, xH2, xHp, chi_PE, chi_LW, chi_C, xi))
    xCt, xOt, Zd = par.xCtot, par.xOtot, par.Zd
    xOp = xOt * xHp
    a = C.ZETA_PI_C_ISRF * chi_C + C.ZETA_PI_C_CR * 2.0 * xH2 * xi + C.ZETA_CR_C * xi
    c = alpha_rrdr_Cp(T) * n
    kch = k_CpH2(T) * n * xH2
    hot = T >= C.XE_T_SWITCH

    xCp = np.zeros(shape)
    xe = np.zeros(shape)
    # cold branch: fixed point on x_e
    xe0 = xHp + xOp + x_MH(T, n, xH2, xi)
    xe_k = xe0 + xCt
    live = ~hot
    yk = np.zeros(shape)
    for _ in range(maxit):
        if not live.any():
            break
        psi = psi_charge(T, n, xe_k, chi_PE, chi_LW)
        B = alpha_gr(T, psi, sd["alpha_gr_Cp"], Zd) * n + kch
        p = a + B + c * xe0
        den = p + np.sqrt(p * p + 4.0 * c * xCt * a)
        y = np.where(a > 0.0, 2.0 * xCt * a / np.where(den > 0.0, den, 1.0), 0.0)
        xe_new = xe0 + y
        conv = np.abs(xe_new - xe_k) <= tol * xe_new
        yk = np.where(live, y, yk)
        xe_k = np.where(live, xe_new, xe_k)
        live = live & ~conv
    xCp = np.where(hot, 0.0, yk)
    xe = np.where(hot, 0.0, xe_k)
    # hot branch: Eq. e:xELhot, x_C+ with that x_e
    lgT = np.log10(T)
    xe_hot = xHp + table1d("cie", lgT, 2) + par.Zg * table1d("cie", lgT, 3)
    psi_h = psi_charge(T, n, xe_hot, chi_PE, chi_LW)
    Bh = alpha_gr(T, psi_h, sd["alpha_gr_Cp"], Zd) * n + kch
    dh = a + Bh + c * xe_hot
    yh = np.where(a > 0.0, xCt * a / np.where(dh > 0.0, dh, 1.0), 0.0)
    xCp = np.where(hot, yh, xCp)
    xe = np.where(hot, xe_hot, xe)
    # CO fit
    xi16 = np.maximum(xi / 1.0e-16, 1.0e-10)
    ncrit = (4.0e3 * Zd / (xi16 * xi16)) ** np.cbrt(chi_LW) * (50.0 * xi16 / Zd ** 1.4)
    frac = np.maximum(xCp / xCt, xHp)
    xCO = xCt * 2.0 * xH2 * (1.0 - frac) / (1.0 + (ncrit / n) ** 2)
    xC = xCt - xCp - xCO
    xO = xOt - xCO - xOp
    return dict(xCp=xCp, xCO=xCO, xC=xC, xOp=xOp, xO=xO, xe=xe)


# --------------------------------------------------------------------------
# dust temperature (Sec. 4.6.4, Eq. eq:dust_en, readings of Sec. 7.1.2)
# --------------------------------------------------------------------------
def dust_heating_per_Zd(chi_PE, chi_LW, phi, Neff, par):
    """UV + optical dust heating per H divided by Z'_d [erg s^-1]."""
    uv = 4.0 * np.pi * (C.SIG_D_PE * C.J_PE * chi_PE + C.SIG_D_LW * C.J_LW * chi_LW) + C.SIG_D_LYC * phi * C.HNU_LYC
    tau = C.SIG_D_NEFF * par.Zd * Neff
    opt = 4.0 * np.pi * (C.SIG_D_PE * C.J_PE + C.SIG_D_LW * C.J_LW) * par.chi0 * np.exp(-tau / par.tau_opt_ratio)
    return uv + opt


def dust_T(T, n, G, par, iters=64):
    """Equilibrium dust temperature by bisection.

    Solves sigma_IR(T_d) c a (T_d^4 - T_bb^4) = Gamma_d + n Lambda_g-d(T, T_d)
    (Eq. eq:dust_en with sigma_IR(T_d) = 2e-25 Z'_d (T_d/10)^2 and
    Eq. eq:gas-dust), divided through by Z'_d.  The residual is increasing in
    T_d above T_bb; the bracket is [min(T_bb, T), 1e4 K].  Returns (T_d,
    unbracketed flag).
    """
    A = C.SIGMA_IR10 / 100.0 * C.C_LIGHT * C.A_RAD
    B = n * C.ALPHA_GD * np.sqrt(T)
    Tbb4 = par.T_bb ** 4

    def g(Td):
        return A * Td * Td * (Td ** 4 - Tbb4) - G - B * (T - Td)

    lo = np.minimum(par.T_bb, T) * np.ones_like(G)
    hi = np.full_like(lo, 1.0e4)
    bad = g(hi) < 0.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        pos = g(mid) >= 0.0
        hi = np.where(pos, mid, hi)
        lo = np.where(pos, lo, mid)
    Td = np.where(bad, 1.0e4, 0.5 * (lo + hi))
    return Td, bad


# --------------------------------------------------------------------------
# fine-structure level populations (Sec. 4.6.2)
# --------------------------------------------------------------------------
def _two_level(g0, g1, E10, A10, C10, T):
    C01 = C10 * (g1 / g0) * np.exp(-E10 / T)
    return C01 / (C01 + C10 + A10)


def _three_level(g, E, A10, A20, A21, C10, C20, C21, T):
    """Steady populations (p0, p1, p2) of a 3-level atom.

    Statistical equilibrium of levels 1 and 2 with p0 set to 1,
      p1 (R10 + R12) - p2 R21 = R01,   -p1 R12 + p2 (R20 + R21) = R02,
    solved by Cramer's rule (determinant R10 R20 + R10 R21 + R12 R20, all terms
    positive), then normalised to p0 + p1 + p2 = 1.  Upward collision rates
    follow detailed balance, C_lu = C_ul (g_u / g_l) exp(-(E_u - E_l) / T).
    """
    g0, g1, g2 = g
    E1, E2 = E
    R01 = C10 * (g1 / g0) * np.exp(-E1 / T)
    R02 = C20 * (g2 / g0) * np.exp(-E2 / T)
    R12 = C21 * (g2 / g1) * np.exp(-(E2 - E1) / T)
    R10, R20, R21 = C10 + A10, C20 + A20, C21 + A21
    det = R10 * R20 + R10 * R21 + R12 * R20
    p1 = (R01 * (R20 + R21) + R21 * R02) / det
    p2 = (R02 * (R10 + R12) + R12 * R01) / det
    s = 1.0 + p1 + p2
    return 1.0 / s, p1 / s, p2 / s


def fine_structure(T, n, xH, xH2, xe, xCp, xC, xO):
    """Lambda_C+, Lambda_C, Lambda_O [erg cm^3 s^-1] (Sec. 4.6.2).

    Rate shapes: H-impact de-excitation of C II 158um, C I 610um and O I 63um
    follow the printed critical densities (C II: n_H,crit formula and
    n_e,crit = 53 T4^1/2; C I / O I: power laws through the printed values at
    10 K and 5000 K) with the recalled A coefficients; the other transitions
    and partners are stand-ins.
    """
    sd = _sd()
    T2, T4 = T / 100.0, T / 1.0e4
    # C+ (2 levels)
    g0, g1, E10, A10 = sd["cp_levels"]
    nc0, s0, s1 = C.CP_NCRIT_H
    k10H = (A10 / nc0) * T2 ** (s0 + s1 * np.log(T2))
    k10e = A10 / (C.CP_NCRIT_E * np.sqrt(T4))
    C10 = n * (xH * k10H + xH2 * sd["cp_h2_over_h"] * k10H + xe * k10e)
    f1 = _two_level(g0, g1, E10, A10, C10, T)
    lam_cp = xCp * f1 * A10 * C.K_B * E10 / n

    def three(levels, coll, ncrit):
        ga, gb, gc, E1, E2, a10, a20, a21 = levels
        r20, r21, rh2, ke0, kex = coll
        s = np.log(ncrit[0] / ncrit[1]) / np.log(500.0)
        kH = (a10 / ncrit[0]) * (T / 10.0) ** s
        ke = ke0 * T4 ** kex
        part = xH * kH + xH2 * rh2 * kH + xe * ke
        c10 = n * part
        c20 = n * r20 * part
        c21 = n * r21 * part
        p0, p1, p2 = _three_level((ga, gb, gc), (E1, E2), a10, a20, a21, c10, c20, c21, T)
        return (p1 * a10 * E1 + p2 * (a20 * E2 + a21 * (E2 - E1))) * C.K_B / n

    lam_c = xC * three(sd["c_levels"], sd["c_coll"], C.C_NCRIT_H)
    lam_o = xO * three(sd["o_levels"], sd["o_coll"], C.O_NCRIT_H)
    return lam_cp, lam_c, lam_o


def lambda_co(T, n, xCO, dvdr):
    """CO rotational cooling with the LVG column Ntilde = n_CO / |dv/dr| (Sec. 4.6.2) -- stand-in table."""
    Nt = n * xCO * C.PC / dvdr
    lT = np.log10(T)
    lN = np.log10(np.maximum(Nt, 1.0e-300))
    L0 = np.exp(LN10 * table2d("co", lT, lN, 0))
    nh = np.exp(LN10 * table2d("co", lT, lN, 1))
    return xCO * L0 / (1.0 + n / nh)


def lambda_rovib(T, n, xH, xH2):
    """H2 ro-vibrational cooling (Sec. 4.6.1) -- stand-in (LTE / low-density interpolation)."""
    sd = _sd()
    r0, r1, r2, r3, r4, r5, r6, v0, v1, v2, v3 = sd["rovib_lte"]
    T3 = T / 1.0e3
    Lrot = r0 * T3 ** r1 / (1.0 + r2 * T3 ** r3) * np.exp(-(r4 / T3) ** 3) + r5 * np.exp(-r6 / T3)
    Lvib = v0 * np.exp(-v1 / T3) + v2 * np.exp(-v3 / T3)
    Llte = Lrot + Lvib
    c0, c1, c2, c3, c4, lo, hi = sd["rovib_low"]
    lg = np.clip(np.log10(T), lo, hi)
    L0 = np.exp(LN10 * (c0 + lg * (c1 + lg * (c2 + lg * (c3 + lg * c4)))))
    npart = n * (xH + xH2)
    L = Llte * npart * L0 / (npart * L0 + Llte)
    return xH2 * L / n


# --------------------------------------------------------------------------
# full evaluation: rates, heating, cooling, net rates (Secs. 3, 4, 6.1)
# --------------------------------------------------------------------------
def q_cr_H2(n):
    """CR heating per ionisation in H2 vs density -- stand-in (piecewise linear in log10 n)."""
    q0, q1, q2, q3, l0, l1, l2, l3 = _sd()["q_cr_H2"]
    ln = np.log10(n)
    return np.interp(ln, [l0, l1, l2, l3], [q0, q1, q2, q3]) * C.EV


def evaluate(T, n, xH2, xHp, eq, rad, par, with_dust=True, chem_only=False):
    """Everything the source step needs at temperature T and abundances (x_H2, x_H+, eq).

    rad: dict with chi_PE, chi_LW, chi_H2, chi_C, phi (LyC photons cm^-2 s^-1),
    xi (primary CR rate), Neff.  Returns a dict with rate coefficients, the
    chemistry matrix pieces (F, D, I, Rr), heating Gamma [erg s^-1 per H],
    cooling Lambda [erg cm^3 s^-1], T_d, H = n Gamma - n^2 Lambda
    (Eq. e:ODE1), C_H2 and C_H+ (Eqs. e:HH, e:HII).
    """
    sd = _sd()
    Zd, Zg = par.Zd, par.Zg
    xe = eq["xe"]
    xH = np.maximum(1.0 - 2.0 * xH2 - xHp, 0.0)
    chi_PE, chi_LW, chi_H2 = rad["chi_PE"], rad["chi_LW"], rad["chi_H2"]
    phi, xi = rad["phi"], rad["xi"]
    psi = psi_charge(T, n, xe, chi_PE, chi_LW)
    # --- chemistry (Eqs. e:HH, e:HII) ---
    kgr = k_gr(T, Zd, par.kgr_const)
    zcrH2 = 2.0 * xi * (2.3 * xH2 + 1.5 * xH)
    zcrH = 0.5 * zcrH2
    zpd = C.ZETA_PD_ISRF * chi_H2
    zpiH2 = C.SIGMA_PI_H2 * phi
    zpiH = C.SIGMA_PI_H * phi
    kcdH, kcdH2 = k_cd_H(T), k_cd_H2(T)
    zcd = n * (xH * kcdH + xH2 * kcdH2)
    kci = k_ci_H(T)
    zci = kci * n * xe
    aB = alpha_B(T)
    agrH = alpha_gr(T, psi, sd["alpha_gr_Hp"], Zd)
    F = kgr * n
    D = 1.65 * zcrH2 + zpd + zpiH2 + zcd
    I = zpiH + zcrH + zci
    Rr = aB * n * xe + agrH * n
    out = dict(kgr=kgr, zcrH2=zcrH2, zcrH=zcrH, zpd=zpd, zpiH2=zpiH2, zpiH=zpiH, zcd=zcd, zci=zci,
               aB=aB, agrH=agrH, F=F, D=D, I=I, Rr=Rr, psi=psi,
               C_H2=F * xH - D * xH2, C_Hp=I * xH - Rr * xHp)
    if chem_only:
        return out
    # --- heating (Secs. 4.1-4.5) ---
    cPE, c1, c2, c3, c4, c5, c6 = C.PE_C
    G0 = C.G0_PER_CHI * chi_fuv(chi_PE, chi_LW)
    eps = (cPE + c1 * T ** c4) / (1.0 + c2 * psi ** c5 * (1.0 + c3 * psi ** c6))
    g_pe = 1.0e-26 * G0 * eps * Zd
    qa, qb, qc = sd["q_cr_H"]
    qH = (qa + qb * np.sqrt(xe / (xe + qc))) * C.EV
    g_cr = xi * (xH * qH + 2.0 * xH2 * q_cr_H2(n))
    g_pi = xH * C.Q_PI_H * zpiH + xH2 * C.Q_PI_H2 * zpiH2
    dcol = xH * k_H2_H(T) + xH2 * k_H2_H2(T)
    eff = n * dcol / (n * dcol + C.A_EFF + zpd)
    g_h2 = (kgr * n * xH * (0.2 * C.EV + 4.2 * C.EV * eff) + zpd * xH2 * C.F_PUMP * 2.0 * C.EV * eff
            + zpd * xH2 * 0.4 * C.EV)
    Gam = g_pe + g_cr + g_pi + g_h2
    out.update(G_pe=g_pe, G_cr=g_cr, G_pi=g_pi, G_h2=g_h2, Gamma=Gam)
    # --- cooling (Sec. 4.6) ---
    T4 = T / 1.0e4
    k12 = 5.31e-8 * T4 ** 0.15 / (1.0 + (T4 / 5.0) ** 0.65) * np.exp(-11.84 / T4)
    l_lya = xH * xe * C.K_B * C.E21_K * k12
    l_ci = C.E_CI * xH * xe * kci
    l_cd = C.E_CD * xH2 * (xH * kcdH + xH2 * kcdH2)
    l_rv = lambda_rovib(T, n, xH, xH2) if par.h2_rovib else np.zeros_like(T * n)
    ff0, gff = sd["ff"]
    l_ff = ff0 * gff * np.sqrt(T) * xe * xHp
    r0, r1 = sd["rr_energy"]
    l_rr = aB * C.K_B * T * (r0 + r1 * np.log(T4)) * xe * xHp
    l_hyd = l_lya + l_ci + l_rv + l_cd + l_ff + l_rr
    l_cp, l_c, l_o = fine_structure(T, n, xH, xH2, xe, eq["xCp"], eq["xC"], eq["xO"])
    l_co = lambda_co(T, n, eq["xCO"], par.dvdr_kms_pc)
    gr0, gr1, gr2, gr3 = sd["grrec"]
    l_gr = gr0 * T ** gr1 * psi ** (gr2 * T ** (-gr3)) * xe * Zd
    lnT4 = np.log(T4)
    fneb = 0.0
    for a in C.NEB_A[::-1]:
        fneb = fneb * lnT4 + a
    fneb = np.exp(LN10 * fneb)
    ne2 = n * xe / 100.0
    l_neb = Zg * xe * xHp * 3.68e-23 * np.exp(-3.86 / T4) * fneb / (
        np.sqrt(T4) * (1.0 + 0.12 * ne2 ** (0.38 - 0.12 * lnT4)))
    if with_dust:
        G = dust_heating_per_Zd(chi_PE, chi_LW, phi, rad["Neff"], par)
        Td, bad = dust_T(T, n, G, par)
    else:
        Td, bad = np.full_like(T * n, np.nan), np.zeros(np.shape(T * n), bool)
    l_gd = C.ALPHA_GD * np.sqrt(T) * (T - Td) * Zd
    S = 1.0 / (1.0 + np.exp(-C.SIG_A * (T - 0.5 * (C.SIG_T1 + C.SIG_T2)) / (C.SIG_T2 - C.SIG_T1)))
    lgT = np.log10(T)
    l_cie = np.exp(LN10 * table1d("cie", lgT, 0)) + Zg * np.exp(LN10 * table1d("cie", lgT, 1))
    Lam = l_hyd + (1.0 - S) * (l_cp + l_c + l_o + l_co + l_gr + l_neb + l_gd) + S * l_cie
    out.update(L_lya=l_lya, L_ci=l_ci, L_rovib=l_rv, L_cd=l_cd, L_ff=l_ff, L_rr=l_rr, L_cp=l_cp, L_c=l_c,
               L_o=l_o, L_co=l_co, L_grrec=l_gr, L_neb=l_neb, L_gd=l_gd, L_cie=l_cie, S=S, Lambda=Lam,
               Td=Td, Td_bad=bad)
    out["H"] = n * Gam - n * n * Lam
    return out
