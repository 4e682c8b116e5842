"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws inputs (densities, temperatures, abundances, source
maps); it holds none of the source step's arithmetic.  It is the one module
that both the HIP-path tests/benchmarks and the CPU oracle checks draw their
inputs from.

Recipes (all seeds derive from SeedSequence(20221014)):

* ``tiny(N)``  i.i.d. cells: log10 n ~ U[-2, 3], log10 T ~ U[1, 6],
  (2 x_H2, x_H+, x_H) ~ Dirichlet(1, 1, 1).  Used on 16^3 = 4096 cells with
  2 pc cells for the small configuration.
* ``grf_cube(N, dx_pc)`` lognormal density from a Gaussian random field: white
  noise smoothed by a Gaussian of sigma = 2 pc in Fourier space, re-standardised,
  n = exp(1.5 g - 1.5^2 / 2) (mean 1 cm^-3); T = 3e3 / ((1.1 + x_H+ - x_H2) n)
  clipped to [10, 1e7] K; abundances Dirichlet as above.
* ``point_sources(nsrc, box_cm)`` seeded uniform positions in the box, each source with
  Q = 1.24e50 s^-1 and L_FUV = 1.36e6 L_sun (a young cluster's LyC and FUV output).
* ``pts256``: the GRF recipe at 256^3 with 2 pc cells (the same 512 pc box), 16 point sources,
  xi_cr per cell log-uniform in [1e-17, 1e-15] s^-1, ten successive steps of 1e4 yr.
* ``pts512``: the ``pts256`` recipe at 512^3 with 2 pc cells (a 1024 pc box), 16 point sources, one
  step of 1e4 yr.
* ``thin(N)`` i.i.d. cells in an unattenuated field (chi = 1 in every band,
  xi_cr = 2e-16 s^-1, N_eff = 0): log10 n ~ U[0, 4], log10 T ~ U[1, 4],
  abundances Dirichlet as above.  Optically thin gas whose three relaxation times
  are short against long steps: the regime where the source step ends at the
  equilibrium of the coupled system.

The paper's TIGRESS snapshots are not available; these grids stand in for them.
"""
import numpy as np

PC = 3.0856775814913673e18
YR = 3.15576e7
SEED = 20221014


def _rngs(k, salt=0):
    ss = np.random.SeedSequence([SEED, salt])
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(k)]


def dirichlet_abundances(rng, N):
    d = rng.dirichlet([1.0, 1.0, 1.0], N)
    return 0.5 * d[:, 0], d[:, 1]


def tiny(N=4096, salt=0):
    """I.i.d. cells (log-uniform n and T, abundances uniform on the simplex)."""
    r = _rngs(3, salt)
    n = 10.0 ** r[0].uniform(-2.0, 3.0, N)
    T = 10.0 ** r[1].uniform(1.0, 6.0, N)
    xH2, xHp = dirichlet_abundances(r[2], N)
    return dict(n=n, T=T, xH2=xH2, xHp=xHp)


def grf_density(shape, dx_pc, sigma_ln=1.5, smooth_pc=2.0, salt=1):
    """Lognormal density with a Gaussian-smoothed Gaussian random field, mean 1 cm^-3."""
    nz, ny, nx = shape
    r = _rngs(1, salt)[0]
    g = r.standard_normal(shape)
    G = np.fft.rfftn(g)
    kz = np.fft.fftfreq(nz)[:, None, None]
    ky = np.fft.fftfreq(ny)[None, :, None]
    kx = np.fft.rfftfreq(nx)[None, None, :]
    s = smooth_pc / dx_pc  # sigma in cells
    G *= np.exp(-2.0 * (np.pi * s) ** 2 * (kx * kx + ky * ky + kz * kz))
    g = np.fft.irfftn(G, s=shape, axes=(0, 1, 2))
    g = (g - g.mean()) / g.std()
    return np.exp(sigma_ln * g - 0.5 * sigma_ln ** 2)


def grf_cube(N, dx_pc, salt=1):
    shape = (N, N, N)
    n = grf_density(shape, dx_pc, salt=salt)
    r = _rngs(1, salt + 100)[0]
    xH2, xHp = dirichlet_abundances(r, n.size)
    xH2 = xH2.reshape(shape)
    xHp = xHp.reshape(shape)
    T = np.clip(3.0e3 / ((1.1 + xHp - xH2) * n), 10.0, 1.0e7)
    return dict(n=n, T=T, xH2=xH2, xHp=xHp)


def thin(N=4096, salt=2):
    """I.i.d. optically thin cells; returns (state, radiation) with radiation arrays per cell."""
    r = _rngs(3, salt)
    n = 10.0 ** r[0].uniform(0.0, 4.0, N)
    T = 10.0 ** r[1].uniform(1.0, 4.0, N)
    xH2, xHp = dirichlet_abundances(r[2], N)
    one = np.ones(N)
    rad = dict(chi_PE=one, chi_LW=one.copy(), chi_H2=one.copy(), chi_C=one.copy(), phi=np.zeros(N),
               xi=np.full(N, 2.0e-16), Neff=np.zeros(N))
    return dict(n=n, T=T, xH2=xH2, xHp=xHp), rad


L_SUN = 3.828e33


def point_sources(nsrc, box_cm, salt=3):
    """Rows of (x_cm, y_cm, z_cm, Q, L_FUV) at seeded uniform positions inside the box."""
    r = _rngs(1, salt)[0]
    pos = r.uniform(0.0, 1.0, (nsrc, 3)) * np.asarray(box_cm, dtype=np.float64)[None, :]
    return np.concatenate([pos, np.full((nsrc, 1), 1.24e50), np.full((nsrc, 1), 1.36e6 * L_SUN)], axis=1)


def cr_map(shape, salt=4):
    r = _rngs(1, salt)[0]
    return 10.0 ** r.uniform(-17.0, -15.0, shape)


CONFIGS = {
    "tiny16": dict(grid=16, dx_pc=2.0, Zg=1.0, dt_yr=1.0e4, cr_mode=0),
    "grf128": dict(grid=128, dx_pc=4.0, Zg=1.0, dt_yr=1.0e4, cr_mode=1),
    "pts256": dict(grid=256, dx_pc=2.0, Zg=1.0, dt_yr=1.0e4, cr_mode=2, nsrc=16, steps=10),
    "pts512": dict(grid=512, dx_pc=2.0, Zg=1.0, dt_yr=1.0e4, cr_mode=2, nsrc=16, steps=1),
}


def make(name, grid=None):
    """Return (state dict with [nz, ny, nx] arrays, config dict)."""
    cfg = dict(CONFIGS[name])
    if grid is not None:
        cfg["grid"] = grid
    N = cfg["grid"]
    if name.startswith("tiny"):
        s = tiny(N ** 3)
        s = {k: v.reshape(N, N, N) for k, v in s.items()}
    else:
        s = grf_cube(N, cfg["dx_pc"])
    if name in ("pts256", "pts512"):
        box = N * cfg["dx_pc"] * PC
        s["xi"] = cr_map(s["n"].shape)
        cfg["sources"] = point_sources(cfg["nsrc"], (box, box, box))
    return s, cfg
