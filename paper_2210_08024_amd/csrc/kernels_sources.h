// Point-source radiation by long characteristics: the many-ray limit of the ray tracing of
// Sec. 5.1 (Eq. e:Erad) evaluated at cell centres.
//
// One lane per cell; the lane walks the straight segment from the source to its cell centre
// through the grid (voxel traversal: at each step the nearest of the three next plane
// crossings), integrating n, n x_H2 and n x_C times the length inside each cell, in double.
// One launch per source: all rays of a launch converge on the same source, so neighbouring
// lanes and concurrent waves walk through the same cells near it and the loads hit the
// caches.  Each source adds
//   chi_PE += chi_s exp(-sigma_PE Z'_d N_H),  chi_LW += chi_s exp(-sigma_LW Z'_d N_H),
//   chi_H2 += (LW term) f_shld,H2(N_H2),      chi_C += (LW term) f_shld,C(N_C, N_H2),
//   phi    += Q exp(-sigma_LyC Z'_d N_H) / (4 pi r^2)  inside the Stromgren radius,
// with chi_s = L_FUV / (16 pi^2 r^2 J^D_FUV) (Eq. e:chi_FUV; equal normalised intensities in
// the two bands) and r at least half a cell.
#pragma once
#include "kernels_columns.h"

namespace ism {

constexpr int MAX_SOURCES = 256;

struct SrcDev {
  double x, y, z;  // position in cell units from the grid corner
  double Q, L;     // ionising photons s^-1, FUV luminosity erg s^-1
  double Rst;      // Stromgren radius, cm
};

__constant__ SrcDev g_src[MAX_SOURCES];

struct PsArgs {
  int32_t nx, ny, nz, nsrc;
  int32_t s0, s1;         // sources handled by this launch
  double dx;
  const double *n, *xH2, *xC;
  void *chiPE, *chiLW, *chiH2, *chiC, *phi;
  double sPE, sLW, sLyC;  // dust cross sections times Z'_d
  double chi_norm;        // 1 / (16 pi^2 J^D_FUV)
  const double *tab;
};

template <class R>
__global__ __launch_bounds__(256) void point_sources_kernel(PsArgs a) {
  __shared__ double s_cs[CS_NX * CS_NY];
  load_cs(a.tab, s_cs);
  const int64_t ncell = (int64_t)a.nx * a.ny * a.nz;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ncell) return;
  const int ci = (int)(idx % a.nx), cj = (int)((idx / a.nx) % a.ny), ck = (int)(idx / ((int64_t)a.nx * a.ny));
  const double c[3] = {ci + 0.5, cj + 0.5, ck + 0.5};
  const int dims[3] = {a.nx, a.ny, a.nz};
  const int max_steps = a.nx + a.ny + a.nz + 4;
  double aPE = 0.0, aLW = 0.0, aH2 = 0.0, aC = 0.0, aphi = 0.0;
  for (int s = a.s0; s < a.s1; ++s) {
    const SrcDev src = g_src[s];
    const double p0[3] = {src.x, src.y, src.z};
    double d[3], tmax[3], tdel[3];
    int v[3], step[3];
    double len2 = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      d[q] = c[q] - p0[q];
      len2 += d[q] * d[q];
      int vq = (int)floor(p0[q]);
      v[q] = vq < 0 ? 0 : (vq > dims[q] - 1 ? dims[q] - 1 : vq);
      if (d[q] > 0.0) {
        step[q] = 1;
        tmax[q] = ((double)(v[q] + 1) - p0[q]) / d[q];
        tdel[q] = 1.0 / d[q];
      } else if (d[q] < 0.0) {
        step[q] = -1;
        tmax[q] = ((double)v[q] - p0[q]) / d[q];
        tdel[q] = -1.0 / d[q];
      } else {
        step[q] = 0;
        tmax[q] = 2.0;
        tdel[q] = 2.0;
      }
    }
    const double Lcm = sqrt(len2) * a.dx;
    double t = 0.0, NH = 0.0, NH2 = 0.0, NC = 0.0;
    for (int it = 0; it < max_steps; ++it) {
      const int q = tmax[0] <= tmax[1] ? (tmax[0] <= tmax[2] ? 0 : 2) : (tmax[1] <= tmax[2] ? 1 : 2);
      const double tn = tmax[q] < 1.0 ? tmax[q] : 1.0;
      const double seg = (tn - t) * Lcm;
      const int64_t vi = (int64_t)v[0] + (int64_t)a.nx * ((int64_t)v[1] + (int64_t)a.ny * v[2]);
      const double nn = a.n[vi] * seg;
      NH += nn;
      NH2 += nn * a.xH2[vi];
      if (a.xC) NC += nn * a.xC[vi];
      if (tmax[q] >= 1.0) break;
      t = tn;
      const int vn = v[q] + step[q];
      v[q] = vn < 0 ? 0 : (vn > dims[q] - 1 ? dims[q] - 1 : vn);
      tmax[q] += tdel[q];
    }
    const double rcm = fmax(Lcm, 0.5 * a.dx);
    const double chi = src.L * a.chi_norm / (rcm * rcm);
    const double wPE = chi * (double)Mx<R>::ex(-a.sPE * NH);
    const double wLW = chi * (double)Mx<R>::ex(-a.sLW * NH);
    aPE += wPE;
    aLW += wLW;
    aH2 += wLW * f_shld_H2<R>(NH2);
    aC += wLW * f_shld_C<R>(NC, NH2, s_cs);
    if (Lcm < src.Rst) aphi += src.Q * (double)Mx<R>::ex(-a.sLyC * NH) / (12.566370614359172954 * rcm * rcm);
  }
  R *pPE = (R *)a.chiPE, *pLW = (R *)a.chiLW, *pH2 = (R *)a.chiH2, *pC = (R *)a.chiC, *pphi = (R *)a.phi;
  pPE[idx] = (R)((double)pPE[idx] + aPE);
  pLW[idx] = (R)((double)pLW[idx] + aLW);
  pH2[idx] = (R)((double)pH2[idx] + aH2);
  pC[idx] = (R)((double)pC[idx] + aC);
  pphi[idx] = (R)((double)pphi[idx] + aphi);
}

}  // namespace ism
