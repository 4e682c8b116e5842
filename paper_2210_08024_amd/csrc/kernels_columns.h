// Six-ray diffuse-UV columns, shielding, N_eff and CR attenuation (Secs. 5.1-5.3).
//
// For every cell and each of +-x, +-y, +-z the exclusive upstream columns (N_H, N_H2,
// N_C) from the face the ray enters are accumulated in double; each direction adds its
// attenuated, shielded weight to a per-cell double4 accumulator (PE, LW, H2-weighted LW,
// C-weighted LW) in the order +x, -x, +y, -y, +z, -z; the z pass scales by chi0/6 and
// writes chi_PE, chi_LW, chi_H2, chi_C, N_eff and xi_cr.
//  * x pass: one wave per x row, 64-cell chunks with wave-wide exclusive scans.
//  * y, z passes: pencils split into segments; a first kernel sums each segment, then
//    one lane per (pencil, segment) -- consecutive x, so loads coalesce -- starts from the
//    exclusive sum of the segments before (or after) it and marches through its segment
//    forward and backward with running sums in registers.
// Templated on R, the type of the transcendental cores (double: F64 outputs, float:
// MIXED outputs); exponents and sums stay double either way.
#pragma once
#include "physics.h"

namespace ism {

struct ColArgs {
  int32_t nx, ny, nz;
  double dx;
  const double *n, *xH2, *xC;
  double4 *acc;
  double *seg;  // segment sums: 3 arrays of nx * other * nseg
  void *chiPE, *chiLW, *chiH2, *chiC, *Neff, *xi;
  int32_t cr_mode;
  int32_t nseg, seglen;  // segments per pencil and their length along the axis
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

// Eq. e:fshld_H2_DB with b5 from the coefficient file.
template <class R>
__device__ __forceinline__ double f_shld_H2(double N) {
  const CoefT<double> &c = g_coef64;
  const double x = N / c.fshld[3];
  const R s = Mx<R>::sq(R(1.0 + x));
  const double u = 1.0 + x / c.b5;
  return c.fshld[0] / (u * u) + c.fshld[1] / (double)s * (double)Mx<R>::ex(-c.fshld[2] * (double)s);
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

template <class R>
__global__ __launch_bounds__(256) void columns_x_kernel(ColArgs a) {
  __shared__ double s_cs[CS_NX * CS_NY];
  load_cs(a.tab, s_cs);
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= (int64_t)a.ny * a.nz) return;
  const int64_t base = row * a.nx;
  const int nch = (a.nx + 63) >> 6;
  for (int dir = 0; dir < 2; ++dir) {
    double cH = 0.0, cH2 = 0.0, cC = 0.0;
    for (int cc = 0; cc < nch; ++cc) {
      const int ch = dir == 0 ? cc : nch - 1 - cc;
      const int i = dir == 0 ? (ch << 6) + lane : (ch << 6) + 63 - lane;
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
        if (dir == 0) {
          a.acc[base + i] = t;
        } else {
          double4 s = a.acc[base + i];
          s.x += t.x; s.y += t.y; s.z += t.z; s.w += t.w;
          a.acc[base + i] = s;
        }
      }
    }
  }
}

// Geometry of the y (AX = 1) and z (AX = 2) passes: lane id -> (i, segment, other index).
struct PencilPos {
  int i, seg, o, L;
  int64_t stride, base;
  bool ok;
};

template <int AX>
__device__ __forceinline__ PencilPos pencil_pos(const ColArgs &a) {
  PencilPos p;
  const int64_t lid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t other = AX == 1 ? a.nz : a.ny;
  p.i = (int)(lid % a.nx);
  const int64_t r = lid / a.nx;
  p.seg = (int)(r % a.nseg);
  p.o = (int)(r / a.nseg);
  p.ok = p.o < other;
  p.L = AX == 1 ? a.ny : a.nz;
  p.stride = AX == 1 ? (int64_t)a.nx : (int64_t)a.nx * a.ny;
  p.base = AX == 1 ? (int64_t)p.o * a.nx * a.ny + p.i : (int64_t)p.o * a.nx + p.i;
  return p;
}

// Sums of (qH, qH2, qC) over each segment of each pencil.
template <int AX>
__global__ __launch_bounds__(256) void columns_segsum_kernel(ColArgs a) {
  const PencilPos p = pencil_pos<AX>(a);
  if (!p.ok) return;
  const int m0 = p.seg * a.seglen;
  const int m1 = m0 + a.seglen < p.L ? m0 + a.seglen : p.L;
  double sH = 0.0, sH2 = 0.0, sC = 0.0;
  for (int m = m0; m < m1; ++m) {
    double qH, qH2, qC;
    cell_q(a, p.base + (int64_t)m * p.stride, qH, qH2, qC);
    sH += qH;
    sH2 += qH2;
    sC += qC;
  }
  const int64_t nseg_all = (int64_t)a.nx * (AX == 1 ? a.nz : a.ny) * a.nseg;
  const int64_t k = ((int64_t)p.o * a.nseg + p.seg) * a.nx + p.i;
  a.seg[k] = sH;
  a.seg[nseg_all + k] = sH2;
  a.seg[2 * nseg_all + k] = sC;
}

template <class O>
__device__ __forceinline__ void store_out(void *p, int64_t i, double v) {
  static_cast<O *>(p)[i] = (O)v;
}

// Forward then backward march through one segment; the z pass (AX = 2) finalises.
template <class R, int AX>
__global__ __launch_bounds__(256) void columns_march_kernel(ColArgs a) {
  __shared__ double s_cs[CS_NX * CS_NY];
  load_cs(a.tab, s_cs);
  const PencilPos p = pencil_pos<AX>(a);
  if (!p.ok) return;
  const int m0 = p.seg * a.seglen;
  const int m1 = m0 + a.seglen < p.L ? m0 + a.seglen : p.L;
  const int64_t nseg_all = (int64_t)a.nx * (AX == 1 ? a.nz : a.ny) * a.nseg;
  const double *sH = a.seg, *sH2 = a.seg + nseg_all, *sC = a.seg + 2 * nseg_all;
  const int64_t k0 = (int64_t)p.o * a.nseg * a.nx + p.i;  // segment s of this pencil at k0 + s nx
  for (int dir = 0; dir < 2; ++dir) {
    double cH = 0.0, cH2 = 0.0, cC = 0.0;
    if (dir == 0) {
      for (int s = 0; s < p.seg; ++s) {
        cH += sH[k0 + (int64_t)s * a.nx];
        cH2 += sH2[k0 + (int64_t)s * a.nx];
        cC += sC[k0 + (int64_t)s * a.nx];
      }
    } else {
      for (int s = a.nseg - 1; s > p.seg; --s) {
        cH += sH[k0 + (int64_t)s * a.nx];
        cH2 += sH2[k0 + (int64_t)s * a.nx];
        cC += sC[k0 + (int64_t)s * a.nx];
      }
    }
    for (int t = m0; t < m1; ++t) {
      const int m = dir == 0 ? t : m1 - 1 - (t - m0);
      const int64_t idx = p.base + (int64_t)m * p.stride;
      double qH, qH2, qC;
      cell_q(a, idx, qH, qH2, qC);
      const double4 w = ray_term<R>(a, cH, cH2, cC, qH, qH2, qC, s_cs);
      cH += qH;
      cH2 += qH2;
      cC += qC;
      double4 acc = a.acc[idx];
      acc.x += w.x; acc.y += w.y; acc.z += w.z; acc.w += w.w;
      if (AX == 2 && dir == 1) {
        const double f = a.chi0 / 6.0;
        const double cPE = f * acc.x;
        const double Neff = a.chi0 > 0.0 ? -::log(cPE / a.chi0) / (g_coef64.sig_d_Neff * a.Zd) : 0.0;
        double xi = a.xi0;
        if (a.cr_mode == 1) {
          const double N0 = g_coef64.N0_cr;
          xi = Neff <= N0 ? a.xi0 : a.xi0 * N0 / (Neff > N0 ? Neff : N0);
        }
        store_out<R>(a.chiPE, idx, cPE);
        store_out<R>(a.chiLW, idx, f * acc.y);
        store_out<R>(a.chiH2, idx, f * acc.z);
        store_out<R>(a.chiC, idx, f * acc.w);
        store_out<R>(a.Neff, idx, Neff);
        if (a.cr_mode != 2) store_out<R>(a.xi, idx, xi);
      } else {
        a.acc[idx] = acc;
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
