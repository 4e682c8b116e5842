// Six-ray diffuse-UV columns, shielding, N_eff and CR attenuation (Secs. 5.1-5.3).
//
// For every cell and each of +-x, +-y, +-z the exclusive upstream columns (N_H, N_H2, N_C)
// from the face the ray enters are accumulated in double, and each ray adds its attenuated,
// shielded weight (PE, LW, H2-weighted LW, C-weighted LW).  The grid is processed in 8^3 tiles
// (tile sums, exclusive scans of the tile sums along each line of tiles, then one pass per tile
// that forms all six rays of every cell and writes the results once); see the tiled pass below.
// Templated on R, the type of the transcendental cores (double: F64 outputs, float: MIXED
// outputs); exponents, columns and attenuation products stay double either way.
#pragma once
#include "physics.h"

namespace ism {

struct ColArgs {
  int32_t nx, ny, nz;
  double dx;
  const double *n, *xH2, *xC;
  void *chiPE, *chiLW, *chiH2, *chiC, *Neff, *xi;
  int32_t cr_mode;
  double chi0, Zd, xi0, sPE, sLW;
  const double *tab;  // full double table (C shielding at TAB_CS)
};

// (1 - exp(-y)) / y, the cell average of exp(-tau) over a cell of optical depth y.
__device__ __forceinline__ double g_slab(double y, double) {
  return y < 1e-4 ? 1.0 - y / 2.0 + y * y / 6.0 : -::expm1(-y) / y;
}
__device__ __forceinline__ double g_slab(double y, float) {
  return y < 1e-4 ? 1.0 - y / 2.0 + y * y / 6.0 : (double)(-::expm1f((float)-y)) / y;
}

// Eq. e:fshld_H2_DB with b5 from the coefficient file.  Both denominators are at least 1, so
// the reciprocal-based division serves; the constants' reciprocals come from the host.
template <class R>
__device__ __forceinline__ double f_shld_H2(double N) {
  const CoefT<double> &c = g_coef64;
  const double x = N * c.inv_fshld_N;
  const R s = Mx<R>::sq(R(1.0 + x));
  const double u = 1.0 + x * c.inv_b5;
  return fdivp(c.fshld[0], u * u) + fdivp(c.fshld[1], (double)s) * (double)Mx<R>::ex(-c.fshld[2] * (double)s);
}

// C self- and H2 cross-shielding: bilinear in log10 f over (log10 N_C, log10 N_H2).
// cs: the C-shielding table itself ([CS_NX][CS_NY], log10 f), e.g. its LDS copy.
template <class R>
__device__ __forceinline__ double f_shld_C(double NC, double NH2, const double *cs) {
  const CoefT<double> &c = g_coef64;
  const double lc = NC > 1e-300 ? Mx<R>::ln(NC) * INV_LN10D : -300.0;
  const double lh = NH2 > 1e-300 ? Mx<R>::ln(NH2) * INV_LN10D : -300.0;
  int i, j;
  double f, g;
  axis_pos(lc, c.cs_x0, c.cs_dx, c.cs_idx, CS_NX, i, f);
  axis_pos(lh, c.cs_y0, c.cs_dy, c.cs_idy, CS_NY, j, g);
  const double v00 = cs[i * CS_NY + j], v01 = cs[i * CS_NY + j + 1];
  const double v10 = cs[(i + 1) * CS_NY + j], v11 = cs[(i + 1) * CS_NY + j + 1];
  return (double)Mx<R>::ex(LN10D * ((v00 * (1.0 - g) + v01 * g) * (1.0 - f) + (v10 * (1.0 - g) + v11 * g) * f));
}

// Contribution of one ray direction to a cell with upstream columns (NH, NH2, NC) and
// own columns (qH, qH2, qC): dust attenuation to the entry face times the cell average
// (Eq. e:Erad with Delta s = dx), shielding at mid-cell.
template <class R>
__device__ __forceinline__ double4 ray_term(const ColArgs &a, double NH, double NH2, double NC, double qH,
                                            double qH2, double qC, const double *cs) {
  const double gPE = g_slab(a.sPE * qH, R(0)), gLW = g_slab(a.sLW * qH, R(0));
  const double wPE = (double)Mx<R>::ex(-a.sPE * NH) * gPE;
  const double wLW = (double)Mx<R>::ex(-a.sLW * NH) * gLW;
  const double mH2 = NH2 + 0.5 * qH2;
  const double mC = NC + 0.5 * qC;
  double4 r;
  r.x = wPE;
  r.y = wLW;
  r.z = wLW * f_shld_H2<R>(mH2);
  r.w = wLW * f_shld_C<R>(mC, mH2, cs);
  return r;
}

template <class O>
__device__ __forceinline__ void store_out(void *p, int64_t i, double v) {
  static_cast<O *>(p)[i] = (O)v;
}

__device__ __forceinline__ void load_cs(const double *g, double *s) {
  for (int k = threadIdx.x; k < CS_NX * CS_NY; k += blockDim.x) s[k] = g[TAB_CS + k];
  __syncthreads();
}

// Inclusive Hillis-Steele scan across the wave; returns the exclusive value and the total.
__device__ __forceinline__ double wave_excl(double v, int lane, double &total) {
  double x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  total = __shfl(x, 63, 64);
  const double e = __shfl_up(x, 1, 64);
  return lane == 0 ? 0.0 : e;
}

__device__ __forceinline__ void cell_q(const ColArgs &a, int64_t idx, double &qH, double &qH2, double &qC) {
  const double nn = a.n[idx];
  qH = nn * a.dx;
  qH2 = nn * a.xH2[idx] * a.dx;
  qC = a.xC ? nn * a.xC[idx] * a.dx : 0.0;
}

// ---------------------------------------------------------------- tiled six-ray pass
// The grid is cut into 8 x 8 x 8 tiles.  Three kernels:
//  1. columns_tilesum_kernel: per tile, the sums of (qH, qH2, qC) = (n, n x_H2, n x_C) dx along
//     every pencil of the tile on each axis (64 pencils per axis).
//  2. columns_offsets_kernel: per line of tiles (the tiles a full-length pencil crosses), the
//     exclusive sums of the tiles before (forward) and after (backward) each tile, each summed
//     in the direction a ray takes, so that a small column keeps its relative precision.
//  3. columns_tile_kernel: four waves per tile stage it in LDS (each wave two z-planes, each
//     lane one (x, y) position); per cell a lane forms the upstream columns of all six rays from
//     the tile offsets plus the in-tile cells before (or after) it, adds the six terms and
//     writes chi_PE, chi_LW, chi_H2, chi_C, N_eff and xi once.
// The dust attenuation exp(-sigma N_in) of a ray is the offset's exp(-sigma F) times the
// per-cell factors exp(-sigma qH) of the in-tile cells it crosses, so each cell costs two
// exponentials (its own factors) instead of two per ray; the cell average g(sigma qH) is the
// same for all six rays and multiplies their sum.  Columns and these products stay double.
constexpr int CT = 8;                       // tile edge
constexpr int CT_LANES = 64;                // tile sums: one wave per tile
constexpr int CT_THREADS = 256;             // tile pass: four waves per tile, two z-planes each
constexpr int CT_NS = CT * (CT + 1) * CT;   // LDS slots per field: x + 9 y + 72 z (bank spread)
__device__ __forceinline__ int ct_slot(int x, int y, int z) { return x + (CT + 1) * y + CT * (CT + 1) * z; }

struct TileGeo {
  int ntx, nty, ntz;
  int64_t lx, ly, lz;     // lines per axis: ny nz, nz nx, ny nx
  int64_t ox, oy, oz;     // offset of each axis's block in an (S, F or B) array: ntx lx, nty ly, ntz lz
  int64_t per_q;          // doubles per quantity in one array: ox + oy + oz
};

struct TileArgs {
  ColArgs c;
  TileGeo g;
  double *S, *F, *B;      // [3 quantities][per_q]: sums, forward and backward exclusive offsets
};

__host__ __device__ inline TileGeo tile_geo(int nx, int ny, int nz) {
  TileGeo g;
  g.ntx = (nx + CT - 1) / CT;
  g.nty = (ny + CT - 1) / CT;
  g.ntz = (nz + CT - 1) / CT;
  g.lx = (int64_t)ny * nz;
  g.ly = (int64_t)nz * nx;
  g.lz = (int64_t)ny * nx;
  g.ox = (int64_t)g.ntx * g.lx;
  g.oy = (int64_t)g.nty * g.ly;
  g.oz = (int64_t)g.ntz * g.lz;
  g.per_q = g.ox + g.oy + g.oz;
  return g;
}

// Index of the pencil sum of tile t along an axis, line l, in one quantity's block.
__device__ __forceinline__ int64_t tile_ix(const TileGeo &g, int ax, int t, int64_t l) {
  return ax == 0 ? (int64_t)t * g.lx + l : (ax == 1 ? g.ox + (int64_t)t * g.ly + l : g.ox + g.oy + (int64_t)t * g.lz + l);
}

// Work item w of a block is the pair of x-neighbouring tiles (2 px, py, pz) and (2 px + 1, py,
// pz), taken one after the other by the same wave: a tile row is 64 bytes, so the pair shares
// each 128-byte line and the second tile finds its lines in the CU's caches.
__device__ __forceinline__ int64_t tile_pairs(const TileGeo &g) {
  return (int64_t)((g.ntx + 1) / 2) * g.nty * g.ntz;
}
__device__ __forceinline__ bool tile_of(const TileGeo &g, int64_t w, int half, int &tx, int &ty, int &tz) {
  const int ntx2 = (g.ntx + 1) / 2;
  tx = 2 * (int)(w % ntx2) + half;
  const int64_t r = w / ntx2;
  ty = (int)(r % g.nty);
  tz = (int)(r / g.nty);
  return tx < g.ntx;
}

// Sum over the 8 lanes of a group: lanes l ^ m for m < 8 (x within a row) or m in {8, 16, 32}
// (y at fixed x).
template <int M0>
__device__ __forceinline__ double group_sum(double v) {
  v += __shfl_xor(v, M0, 64);
  v += __shfl_xor(v, 2 * M0, 64);
  v += __shfl_xor(v, 4 * M0, 64);
  return v;
}

__global__ __launch_bounds__(CT_LANES) void columns_tilesum_kernel(TileArgs t) {
  const ColArgs &a = t.c;
  const TileGeo &g = t.g;
  const int lane = threadIdx.x;
  const int lx = lane & 7, ly = lane >> 3;
  const int64_t nw = tile_pairs(g);
  for (int64_t w2 = 2 * (int64_t)blockIdx.x; w2 < 2 * nw; w2 += ((w2 & 1) ? 2 * (int64_t)gridDim.x - 1 : 1)) {
    int tx, ty, tz;
    if (!tile_of(g, w2 >> 1, (int)(w2 & 1), tx, ty, tz)) continue;
    const int gx = tx * CT + lx, gy = ty * CT + ly;
    const bool in_xy = gx < a.nx && gy < a.ny;
    double zs[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
    for (int z = 0; z < CT; ++z) {
      const int gz = tz * CT + z;
      double q[3] = {0.0, 0.0, 0.0};
      if (in_xy && gz < a.nz) cell_q(a, ((int64_t)gz * a.ny + gy) * a.nx + gx, q[0], q[1], q[2]);
      for (int k = 0; k < 3; ++k) {
        zs[k] += q[k];
        const double sx = group_sum<1>(q[k]);   // along x: the 8 lanes of row ly
        const double sy = group_sum<8>(q[k]);   // along y: the 8 lanes at column lx
        if (gz < a.nz) {
          if (lx == 0 && gy < a.ny) t.S[k * g.per_q + tile_ix(g, 0, tx, (int64_t)gz * a.ny + gy)] = sx;
          if (ly == 0 && gx < a.nx) t.S[k * g.per_q + tile_ix(g, 1, ty, (int64_t)gz * a.nx + gx)] = sy;
        }
      }
    }
    if (in_xy)
      for (int k = 0; k < 3; ++k) t.S[k * g.per_q + tile_ix(g, 2, tz, (int64_t)gy * a.nx + gx)] = zs[k];
  }
}

// One thread per (axis, line, direction): forward threads write F, backward threads write B.
__global__ __launch_bounds__(256) void columns_offsets_kernel(TileArgs t) {
  const TileGeo &g = t.g;
  const int64_t nl = g.lx + g.ly + g.lz;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= 2 * nl) return;
  const bool fwd = id < nl;
  int64_t l = fwd ? id : id - nl;
  int ax, nt;
  if (l < g.lx) { ax = 0; nt = g.ntx; }
  else if (l < g.lx + g.ly) { ax = 1; l -= g.lx; nt = g.nty; }
  else { ax = 2; l -= g.lx + g.ly; nt = g.ntz; }
  double *out = fwd ? t.F : t.B;
  double run[3] = {0.0, 0.0, 0.0};
  for (int s = 0; s < nt; ++s) {
    const int tt = fwd ? s : nt - 1 - s;
    const int64_t ix = tile_ix(g, ax, tt, l);
    for (int k = 0; k < 3; ++k) {
      out[k * g.per_q + ix] = run[k];
      run[k] += t.S[k * g.per_q + ix];
    }
  }
}

// Ray state entering a cell: dust attenuation in the two bands and the H2 and C columns.
struct RayIn {
  double P, L, H2, C;
};

template <class R>
__device__ __forceinline__ void add_ray(const RayIn &r, double hH2, double hC, const double *cs, double acc[4]) {
  const double mH2 = r.H2 + hH2, mC = r.C + hC;
  acc[0] += r.P;
  acc[1] += r.L;
  acc[2] += r.L * f_shld_H2<R>(mH2);
  acc[3] += r.L * f_shld_C<R>(mC, mH2, cs);
}

// e^-y for the running products and g(y) = (1 - e^-y) / y, the cell average, from one
// transcendental: below y = 0.35 e^-y - 1 (accurate however small y) gives both, above it e^-y
// does (1 - e^-y >= 0.29 there, so the subtraction keeps its digits, and e^-y keeps its own
// relative precision however thick the cell).
template <class R>
__device__ __forceinline__ void cell_atten(double y, double &e, double &gy) {
  double m;
  if (y <= 0.35) {
    m = std::is_same<R, double>::value ? fexpm1(-y) : (double)::expm1f((float)-y);
    e = 1.0 + m;
  } else {
    e = (double)Mx<R>::ex(-y);
    m = e - 1.0;
  }
  gy = y < 1e-4 ? 1.0 - y / 2.0 + y * y / 6.0 : -m / y;
}

template <class R>
__global__ __launch_bounds__(CT_THREADS) void columns_tile_kernel(TileArgs t) {
  __shared__ double s_cs[CS_NX * CS_NY];
  // per cell of the tile: (e^-y PE, e^-y LW) and (N_H2, N_C) of the cell, read as 16-byte pairs
  __shared__ double2 s_e[CT_NS], s_q[CT_NS];
  // per axis and pencil of the tile: Pf Lf H2f Cf (forward ray at the tile's entry face) and
  // Pb Lb H2b Cb (backward ray); pencils x: (y, z), y: (x, z), z: (x, y), index a + 8 b
  __shared__ double s_off[3][64][8];
  const ColArgs &a = t.c;
  const TileGeo &g = t.g;
  for (int k = threadIdx.x; k < CS_NX * CS_NY; k += blockDim.x) s_cs[k] = a.tab[TAB_CS + k];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int lx = lane & 7, ly = lane >> 3;
  const double fo = a.chi0 / 6.0;
  const int64_t nw = tile_pairs(g);
  for (int64_t w2 = 2 * (int64_t)blockIdx.x; w2 < 2 * nw; w2 += ((w2 & 1) ? 2 * (int64_t)gridDim.x - 1 : 1)) {
    int tx, ty, tz;
    if (!tile_of(g, w2 >> 1, (int)(w2 & 1), tx, ty, tz)) continue;
    const int gx = tx * CT + lx, gy = ty * CT + ly;
    const bool in_xy = gx < a.nx && gy < a.ny;
    __syncthreads();  // the previous tile's LDS reads are done
    // stage the tile: wave wv takes the z-planes 2 wv and 2 wv + 1
#pragma unroll
    for (int zz = 0; zz < CT / 4; ++zz) {
      const int z = (CT / 4) * wv + zz, gz = tz * CT + z;
      double qH = 0.0, qH2 = 0.0, qC = 0.0;
      if (in_xy && gz < a.nz) cell_q(a, ((int64_t)gz * a.ny + gy) * a.nx + gx, qH, qH2, qC);
      double eP, eL, gP, gL;
      cell_atten<R>(a.sPE * qH, eP, gP);
      cell_atten<R>(a.sLW * qH, eL, gL);
      const int sl = ct_slot(lx, ly, z);
      s_e[sl] = make_double2(eP, eL);
      s_q[sl] = make_double2(qH2, qC);
    }
    // the offsets of the tile's 3 x 64 pencils, dust columns turned into attenuation factors
    if (tid < 3 * 64) {
      const int ax = tid >> 6, p0 = lane & 7, p1 = lane >> 3;
      bool ok;
      int64_t l;
      int tt;
      if (ax == 0) {
        const int gyy = ty * CT + p0, gzz = tz * CT + p1;
        ok = gyy < a.ny && gzz < a.nz;
        l = (int64_t)gzz * a.ny + gyy;
        tt = tx;
      } else if (ax == 1) {
        const int gxx = tx * CT + p0, gzz = tz * CT + p1;
        ok = gxx < a.nx && gzz < a.nz;
        l = (int64_t)gzz * a.nx + gxx;
        tt = ty;
      } else {
        const int gxx = tx * CT + p0, gyy = ty * CT + p1;
        ok = gxx < a.nx && gyy < a.ny;
        l = (int64_t)gyy * a.nx + gxx;
        tt = tz;
      }
      double f[3] = {0.0, 0.0, 0.0}, b[3] = {0.0, 0.0, 0.0};
      if (ok) {
        const int64_t ix = tile_ix(g, ax, tt, l);
        for (int k = 0; k < 3; ++k) {
          f[k] = t.F[k * g.per_q + ix];
          b[k] = t.B[k * g.per_q + ix];
        }
      }
      double *o = s_off[ax][lane];
      o[0] = (double)Mx<R>::ex(-a.sPE * f[0]);
      o[1] = (double)Mx<R>::ex(-a.sLW * f[0]);
      o[2] = f[1];
      o[3] = f[2];
      o[4] = (double)Mx<R>::ex(-a.sPE * b[0]);
      o[5] = (double)Mx<R>::ex(-a.sLW * b[0]);
      o[6] = b[1];
      o[7] = b[2];
    }
    __syncthreads();
#pragma unroll 1
    for (int zz = 0; zz < CT / 4; ++zz) {
      const int z = (CT / 4) * wv + zz, gz = tz * CT + z;
      const int sl = ct_slot(lx, ly, z);
      const double2 qq = s_q[sl];
      const double hH2 = 0.5 * qq.x, hC = 0.5 * qq.y;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      // the six rays in the order +x, -x, +y, -y, +z, -z: the offset at the tile face times the
      // factors of the tile's cells the ray crosses before this one
#pragma unroll 1
      for (int ax = 0; ax < 3; ++ax) {
        const int mine = ax == 0 ? lx : (ax == 1 ? ly : z);
        const int pen = ax == 0 ? ly + 8 * z : (ax == 1 ? lx + 8 * z : lane);
        const int stride = ax == 0 ? 1 : (ax == 1 ? CT + 1 : CT * (CT + 1));
        const int base = ax == 0 ? ct_slot(0, ly, z) : (ax == 1 ? ct_slot(lx, 0, z) : ct_slot(lx, ly, 0));
        const double *o = s_off[ax][pen];
        RayIn f{o[0], o[1], o[2], o[3]}, b{o[4], o[5], o[6], o[7]};
        // the forward and the backward ray of the axis in one pass over the pencil: each cell's
        // factors are read once and multiply into whichever ray has crossed the cell
#pragma unroll
        for (int k = 0; k < CT; ++k) {
          const int s2 = base + k * stride;
          const double2 ee = s_e[s2], qv = s_q[s2];
          const double eP = ee.x, eL = ee.y, h = qv.x, c = qv.y;
          if (k < mine) {
            f.P *= eP;
            f.L *= eL;
            f.H2 += h;
            f.C += c;
          }
          if (k > mine) {
            b.P *= eP;
            b.L *= eL;
            b.H2 += h;
            b.C += c;
          }
        }
        add_ray<R>(f, hH2, hC, s_cs, acc);
        add_ray<R>(b, hH2, hC, s_cs, acc);
      }
      if (in_xy && gz < a.nz) {
        const int64_t idx = ((int64_t)gz * a.ny + gy) * a.nx + gx;
        const double qH = a.n[idx] * a.dx;  // staged above, so an L2 hit
        double e, gP, gL;
        cell_atten<R>(a.sPE * qH, e, gP);
        cell_atten<R>(a.sLW * qH, e, gL);
        const double cPE = fo * gP * acc[0];
        // (chi_PE can underflow to 0 in a thick enough cloud: the log with its special cases)
        const double Neff = a.chi0 > 0.0 ? -flog(cPE / a.chi0) / (g_coef64.sig_d_Neff * a.Zd) : 0.0;
        double xi = a.xi0;
        if (a.cr_mode == 1) {
          const double N0 = g_coef64.N0_cr;
          xi = Neff <= N0 ? a.xi0 : a.xi0 * N0 / (Neff > N0 ? Neff : N0);
        }
        store_out<R>(a.chiPE, idx, cPE);
        store_out<R>(a.chiLW, idx, fo * gL * acc[1]);
        store_out<R>(a.chiH2, idx, fo * gL * acc[2]);
        store_out<R>(a.chiC, idx, fo * gL * acc[3]);
        store_out<R>(a.Neff, idx, Neff);
        if (a.cr_mode != 2) store_out<R>(a.xi, idx, xi);
      }
    }
  }
}

// A beam of surface intensity chi0 entering through the x = 0 face along +x (plane-parallel
// slab): the +x ray of the six-ray pass with weight chi0, finalised in the same kernel.
template <class R>
__global__ __launch_bounds__(256) void columns_beam_kernel(ColArgs a) {
  __shared__ double s_cs[CS_NX * CS_NY];
  load_cs(a.tab, s_cs);
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= (int64_t)a.ny * a.nz) return;
  const int64_t base = row * a.nx;
  const int nch = (a.nx + 63) >> 6;
  double cH = 0.0, cH2 = 0.0, cC = 0.0;
  for (int ch = 0; ch < nch; ++ch) {
    const int i = (ch << 6) + lane;
    const bool ok = i < a.nx;
    double qH = 0.0, qH2 = 0.0, qC = 0.0;
    if (ok) cell_q(a, base + i, qH, qH2, qC);
    double tH, tH2, tC;
    const double eH = wave_excl(qH, lane, tH) + cH;
    const double eH2 = wave_excl(qH2, lane, tH2) + cH2;
    const double eC = wave_excl(qC, lane, tC) + cC;
    cH += tH;
    cH2 += tH2;
    cC += tC;
    if (ok) {
      const double4 t = ray_term<R>(a, eH, eH2, eC, qH, qH2, qC, s_cs);
      const int64_t idx = base + i;
      const double cPE = a.chi0 * t.x;
      const double Neff = a.chi0 > 0.0 ? -::log(cPE / a.chi0) / (g_coef64.sig_d_Neff * a.Zd) : 0.0;
      double xi = a.xi0;
      if (a.cr_mode == 1) {
        const double N0 = g_coef64.N0_cr;
        xi = Neff <= N0 ? a.xi0 : a.xi0 * N0 / (Neff > N0 ? Neff : N0);
      }
      store_out<R>(a.chiPE, idx, cPE);
      store_out<R>(a.chiLW, idx, a.chi0 * t.y);
      store_out<R>(a.chiH2, idx, a.chi0 * t.z);
      store_out<R>(a.chiC, idx, a.chi0 * t.w);
      store_out<R>(a.Neff, idx, Neff);
      if (a.cr_mode != 2) store_out<R>(a.xi, idx, xi);
    }
  }
}

// Local shielding-length radiation (Sec. 7.1.2): each cell sees the background field through
// N_shld = n L, with H2 and C self-shielding through half of its own H2 and C columns.
template <class R>
__global__ __launch_bounds__(256) void local_shield_kernel(int64_t ncell, const double *n, const double *xH2,
                                                            const double *xC, const double *L, R *chiPE, R *chiLW,
                                                            R *chiH2, R *chiC, R *Neff, R *xi, double chi0,
                                                            double sPE, double sLW, double xi0, int cr_mode,
                                                            const double *tab) {
  __shared__ double s_cs[CS_NX * CS_NY];
  load_cs(tab, s_cs);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncell) return;
  const double nL = n[i] * L[i];
  const double wPE = chi0 * (double)Mx<R>::ex(-sPE * nL);
  const double wLW = chi0 * (double)Mx<R>::ex(-sLW * nL);
  const double NH2 = 0.5 * xH2[i] * nL;
  const double NC = xC ? 0.5 * xC[i] * nL : 0.0;
  chiPE[i] = (R)wPE;
  chiLW[i] = (R)wLW;
  chiH2[i] = (R)(wLW * f_shld_H2<R>(NH2));
  chiC[i] = (R)(wLW * f_shld_C<R>(NC, NH2, s_cs));
  Neff[i] = (R)nL;
  if (cr_mode == 0) xi[i] = (R)xi0;
  else if (cr_mode == 1) xi[i] = (R)(nL <= g_coef64.N0_cr ? xi0 : xi0 * g_coef64.N0_cr / nL);
}

}  // namespace ism
