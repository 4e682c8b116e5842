// Six-ray diffuse-UV columns, shielding, N_eff and CR attenuation (Secs. 5.1-5.3).
//
// Three passes, one per axis, each a forward and a backward sweep that carries the
// exclusive upstream columns (N_H, N_H2, N_C, in double) from the face the ray
// enters.  Each sweep adds its direction's contribution to a per-cell double4
// accumulator (PE, LW, H2-weighted LW, C-weighted LW); the z pass scales by chi0/6
// and writes the outputs.  Direction order +x, -x, +y, -y, +z, -z.
//  * x pass: one wave per x-row, 64-cell chunks with wave-wide exclusive scans.
//  * y, z passes: one lane per pencil (consecutive x -> coalesced), marching along
//    the axis with running sums in registers.
#pragma once
#include "physics.h"

namespace ism {

struct ColArgs {
  int32_t nx, ny, nz;
  double dx;
  const double *n, *xH2, *xC;
  double4 *acc;
  void *chiPE, *chiLW, *chiH2, *chiC, *Neff, *xi;
  int32_t out_f32;
  int32_t cr_mode;
  double chi0, Zd, xi0, sPE, sLW;
  const double *tab;  // full double table (C shielding at TAB_CS)
};

__device__ __forceinline__ double g_slab(double y) {
  return y < 1e-4 ? 1.0 - y / 2.0 + y * y / 6.0 : -::expm1(-y) / y;
}

__device__ __forceinline__ double f_shld_H2(double N) {
  const CoefT<double> &c = g_coef64;
  const double x = N / c.fshld[3];
  const double s = ::sqrt(1.0 + x);
  const double u = 1.0 + x / c.b5;
  return c.fshld[0] / (u * u) + c.fshld[1] / s * ::exp(-c.fshld[2] * s);
}

// cs: the C-shielding table itself ([CS_NX][CS_NY], log10 f), e.g. its LDS copy.
__device__ __forceinline__ double f_shld_C(double NC, double NH2, const double *cs) {
  const CoefT<double> &c = g_coef64;
  const double lc = ::log10(NC > 1e-300 ? NC : 1e-300);
  const double lh = ::log10(NH2 > 1e-300 ? NH2 : 1e-300);
  int i, j;
  double f, g;
  axis_pos(lc, c.cs_x0, c.cs_dx, CS_NX, i, f);
  axis_pos(lh, c.cs_y0, c.cs_dy, CS_NY, j, g);
  const double *v = cs;
  const double v00 = v[i * CS_NY + j], v01 = v[i * CS_NY + j + 1];
  const double v10 = v[(i + 1) * CS_NY + j], v11 = v[(i + 1) * CS_NY + j + 1];
  return ::exp(LN10 * ((v00 * (1.0 - g) + v01 * g) * (1.0 - f) + (v10 * (1.0 - g) + v11 * g) * f));
}

// Contribution of one ray direction to a cell with upstream columns (NH, NH2, NC) and
// own columns (qH, qH2, qC).
__device__ __forceinline__ double4 ray_term(const ColArgs &a, double NH, double NH2, double NC, double qH,
                                            double qH2, double qC, const double *cs_tab) {
  const double gPE = g_slab(a.sPE * qH), gLW = g_slab(a.sLW * qH);
  const double wPE = ::exp(-a.sPE * NH) * gPE;
  const double wLW = ::exp(-a.sLW * NH) * gLW;
  const double mH2 = NH2 + 0.5 * qH2;
  const double mC = NC + 0.5 * qC;
  double4 r;
  r.x = wPE;
  r.y = wLW;
  r.z = wLW * f_shld_H2(mH2);
  r.w = wLW * f_shld_C(mC, mH2, cs_tab);
  return r;
}

__device__ __forceinline__ void load_cs(const double *g, double *s) {
  for (int k = threadIdx.x; k < CS_NX * CS_NY; k += blockDim.x) s[k] = g[TAB_CS + k];
  __syncthreads();
}

// Inclusive Hillis-Steele scan; exclusive value obtained by shifting one lane up.
__device__ __forceinline__ double wave_excl(double v, int lane, double &total) {
  double x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    double y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  total = __shfl(x, 63, 64);
  double e = __shfl_up(x, 1, 64);
  return lane == 0 ? 0.0 : e;
}

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
      if (ok) {
        const double nn = a.n[base + i];
        qH = nn * a.dx;
        qH2 = nn * a.xH2[base + i] * a.dx;
        qC = a.xC ? nn * a.xC[base + i] * a.dx : 0.0;
      }
      double tH, tH2, tC;
      const double eH = wave_excl(qH, lane, tH) + cH;
      const double eH2 = wave_excl(qH2, lane, tH2) + cH2;
      const double eC = wave_excl(qC, lane, tC) + cC;
      cH += tH;
      cH2 += tH2;
      cC += tC;
      if (ok) {
        const double4 t = ray_term(a, eH, eH2, eC, qH, qH2, qC, s_cs);
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

template <class O>
__device__ __forceinline__ void store_out(void *p, int64_t i, double v) {
  static_cast<O *>(p)[i] = (O)v;
}

// Sweep along y (AX = 1) or z (AX = 2); lanes are consecutive x.  The z pass finalises.
template <int AX>
__global__ __launch_bounds__(64) void columns_yz_kernel(ColArgs a) {
  __shared__ double s_cs[CS_NX * CS_NY];
  load_cs(a.tab, s_cs);
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= a.nx) return;
  const int o = blockIdx.y;  // the other transverse index: k for AX = 1, j for AX = 2
  const int L = AX == 1 ? a.ny : a.nz;
  const int64_t stride = AX == 1 ? (int64_t)a.nx : (int64_t)a.nx * a.ny;
  const int64_t base = AX == 1 ? (int64_t)o * a.nx * a.ny + i : (int64_t)o * a.nx + i;
  for (int dir = 0; dir < 2; ++dir) {
    double cH = 0.0, cH2 = 0.0, cC = 0.0;
    for (int s = 0; s < L; ++s) {
      const int m = dir == 0 ? s : L - 1 - s;
      const int64_t idx = base + (int64_t)m * stride;
      const double nn = a.n[idx];
      const double qH = nn * a.dx;
      const double qH2 = nn * a.xH2[idx] * a.dx;
      const double qC = a.xC ? nn * a.xC[idx] * a.dx : 0.0;
      const double4 t = ray_term(a, cH, cH2, cC, qH, qH2, qC, s_cs);
      cH += qH;
      cH2 += qH2;
      cC += qC;
      double4 acc = a.acc[idx];
      acc.x += t.x; acc.y += t.y; acc.z += t.z; acc.w += t.w;
      if (AX == 2 && dir == 1) {
        const double f = a.chi0 / 6.0;
        const double cPE = f * acc.x;
        const double Neff = a.chi0 > 0.0 ? -::log(cPE / a.chi0) / (g_coef64.sig_d_Neff * a.Zd) : 0.0;
        double xi = a.xi0;
        if (a.cr_mode == 1) {
          const double N0 = g_coef64.N0_cr;
          xi = Neff <= N0 ? a.xi0 : a.xi0 * N0 / (Neff > N0 ? Neff : N0);
        }
        if (a.out_f32) {
          store_out<float>(a.chiPE, idx, cPE);
          store_out<float>(a.chiLW, idx, f * acc.y);
          store_out<float>(a.chiH2, idx, f * acc.z);
          store_out<float>(a.chiC, idx, f * acc.w);
          store_out<float>(a.Neff, idx, Neff);
          if (a.cr_mode != 2) store_out<float>(a.xi, idx, xi);
        } else {
          store_out<double>(a.chiPE, idx, cPE);
          store_out<double>(a.chiLW, idx, f * acc.y);
          store_out<double>(a.chiH2, idx, f * acc.z);
          store_out<double>(a.chiC, idx, f * acc.w);
          store_out<double>(a.Neff, idx, Neff);
          if (a.cr_mode != 2) store_out<double>(a.xi, idx, xi);
        }
      } else {
        a.acc[idx] = acc;
      }
    }
  }
}

}  // namespace ism
