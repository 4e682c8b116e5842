// Adaptive ray tracing of point sources (Sec. 5.1, Eqs. e:Erad, e:Erad_H2, e:chi_H2).
//
// Packets start at each source along the HEALPix directions of level l0 (12 4^l0 of them) and
// walk the grid cell by cell.  In a cell crossed over ds, band j (PE, LW: dust; LyC: H, H2 and
// dust) deposits L_in,j (1 - exp(-alpha_j ds)) / alpha_j, with L_in,j = L_j exp(-tau_j) /
// N_ray(l) and tau_j from the source to the entry face; the LW deposit is also weighted by
// f_shld,H2 and f_shld,C of the columns to the middle of the segment.  Before entering a cell
// at distance r a packet is dropped when every tau_j exceeds tau_max, and split into its four
// nested children (same r, own directions, the parent's columns) when fewer than Phi_c rays
// of its level cross a cell there: N_ray(l) dx^2 / (4 pi r^2) < Phi_c.
//
// The tracing is level-synchronous: one launch per HEALPix level, one lane per packet.  The
// first launch makes its packets from the lane index; every launch appends the children of
// its split packets to the next level's list (one atomic per wave; the four children of a
// parent are adjacent, so neighbouring lanes of the next launch walk neighbouring rays).
// Deposits are atomic adds into the output fields, so the summation order, and the last bits
// of the result, vary between runs.  Distances inside the kernel are in cell units.
//
// With a flux output the packets also deposit their chi_PE, chi_LW and phi additions times
// their direction (Eq. e:Frad): nine more sums per cell, band-major (PE, LW, LyC) then x, y, z.
// PE and LW become band energy fluxes (the packet's FUV luminosity shared as J^D_PE : J^D_LW,
// the Draine field's shares), LyC a photon flux.  radiation_force_kernel turns them into the
// force per volume on the gas-dust mixture (Sec. 6.2) with the grain-destruction switch.
#pragma once
#include "kernels_sources.h"

namespace ism {

constexpr int ART_MAX_LEVEL = 13;  // 12 4^13 pixels still fit a 32-bit index
constexpr double EXIT_TOL = 1e-10;  // cells

struct ArtRay {  // 48 bytes
  uint32_t pix;
  uint16_t src;
  uint16_t pad;
  double r;                    // start distance from the source, cell units
  double NH, NH2, NC, tauLyC;  // columns (cm^-2) and LyC optical depth from the source
};

struct ArtArgs {
  int32_t nx, ny, nz, nsrc;
  int32_t level, max_level;
  int64_t nin;                  // packets in this launch
  const ArtRay *in;             // null: the launch makes nsrc x 12 4^level packets at r = 0
  ArtRay *out;                  // children (capacity 4 nin when level < max_level)
  unsigned long long *nout;
  double dx;                    // cm
  double R2split;               // split when r^2 > R2split (cell units)
  double tau_max;
  const double *n, *xH2, *xHp, *xC;
  void *chiPE, *chiLW, *chiH2, *chiC, *phi;
  double sPE, sLW, sdLyC, spiH, spiH2;  // dust cross sections x Z'_d; photoionisation
  double fuv_norm;              // 1 / (4 pi dV J^D_FUV)
  double phi_norm;              // 1 / dV
  double *budget;               // [nsrc][6]: escaped PE, LW, LyC, dropped PE, LW, LyC; or null
  const double *tab;
  void *flux;                   // null, or 9 arrays of ncell (band-major, then x, y, z)
  int64_t ncell;
  double kPE, kLW;              // 4 pi J^D_PE, 4 pi J^D_LW: chi additions to energy fluxes
};

// Gather every other bit (bits 0, 2, 4, ...) of a 32-bit word into the low half.
__device__ __forceinline__ uint32_t even_bits(uint32_t x) {
  x &= 0x55555555u;
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0F0F0F0Fu;
  x = (x | (x >> 4)) & 0x00FF00FFu;
  x = (x | (x >> 8)) & 0x0000FFFFu;
  return x;
}

// Centre of HEALPix pixel p (nested numbering) at a level (Gorski et al. 2005): the base pixel
// and the in-face coordinates give the ring index (counted from the north pole) and the
// position in the ring; polar rings hold 4 nr pixels at z = +-(1 - nr^2 / (3 nside^2)), the
// equatorial belt's rings 4 nside pixels at z = 2 (2 nside - ring) / (3 nside), every other
// belt ring shifted by half a pixel.
__device__ __forceinline__ void healpix_dir(int level, uint32_t p, double u[3]) {
  const int64_t ns = 1ll << level;
  const uint32_t f = p >> (2 * level);
  const uint32_t ipf = p & (uint32_t)(ns * ns - 1);
  const int64_t ix = even_bits(ipf), iy = even_bits(ipf >> 1);
  const int64_t ring_base = (int64_t)(f >> 2) + 2;                     // 2, 3, 4 by row of faces
  const int64_t col_base = f < 4 ? 2 * f + 1 : (f < 8 ? 2 * (f - 4) : 2 * (f - 8) + 1);
  const int64_t jr = ring_base * ns - ix - iy - 1;
  int64_t nr, shift;
  double z, sth;
  const double inv3n2 = 1.0 / (3.0 * (double)(ns * ns));
  if (jr < ns) {
    nr = jr;
    shift = 0;
    const double t = (double)(nr * nr) * inv3n2;  // 1 - z
    z = 1.0 - t;
    sth = sqrt(t * (2.0 - t));
  } else if (jr > 3 * ns) {
    nr = 4 * ns - jr;
    shift = 0;
    const double t = (double)(nr * nr) * inv3n2;
    z = t - 1.0;
    sth = sqrt(t * (2.0 - t));
  } else {
    nr = ns;
    shift = (jr - ns) & 1;
    z = (double)(2 * ns - jr) * 2.0 / (3.0 * (double)ns);
    sth = sqrt((1.0 - z) * (1.0 + z));
  }
  int64_t jp = (col_base * nr + ix - iy + 1 + shift) / 2;
  if (jp > 4 * ns) jp -= 4 * ns;
  if (jp < 1) jp += 4 * ns;
  // phi / pi, so that directions in a coordinate plane (phi a multiple of pi/2) get exactly
  // zero components
  const double phi_pi = ((double)jp - 0.5 * (double)(shift + 1)) / (double)(2 * nr);
  double sp, cp;
  sincospi(phi_pi, &sp, &cp);
  u[0] = sth * cp;
  u[1] = sth * sp;
  u[2] = z;
}

__device__ __forceinline__ double expm1_neg(double y, double) { return ::expm1(-y); }
__device__ __forceinline__ double expm1_neg(double y, float) { return (double)::expm1f((float)-y); }

// (1 - exp(-y)) / y for y >= 0 and exp(-y): from one expm1 while exp(-y) is near 1 (where
// 1 - exp(-y) would cancel), from one exp beyond (where 1 + expm1(-y) would).
template <class R>
__device__ __forceinline__ void absorb(double y, double &g, double &e) {
  if (y < 1e-8) {
    g = 1.0 - 0.5 * y;
    e = 1.0 - y;
  } else if (y < 0.5) {
    const double m = expm1_neg(y, R(0));
    g = -m / y;
    e = 1.0 + m;
  } else {
    e = (double)Mx<R>::ex(-y);
    g = (1.0 - e) / y;
  }
}

// Per-lane LDS stride of the combine, in elements of R: a multiple of 16 bytes such that the
// eight lanes served by one pass of a 128-bit LDS access fall in distinct banks.
template <class R, int NV> struct SlotStride;
template <> struct SlotStride<float, 5> { static constexpr int v = 12; };
template <> struct SlotStride<float, 14> { static constexpr int v = 20; };
template <> struct SlotStride<double, 5> { static constexpr int v = 6; };
template <> struct SlotStride<double, 14> { static constexpr int v = 14; };
template <class R> struct Vec16;
template <> struct Vec16<float> { using T = float4; static constexpr int n = 4; };
template <> struct Vec16<double> { using T = double2; static constexpr int n = 2; };

// Lanes of one wave exchange values through LDS below.  The LDS executes a wave's
// instructions in order, so only the compiler has to be kept from moving or forwarding memory
// accesses across an exchange point: an empty asm statement that clobbers memory.
__device__ __forceinline__ void lane_exchange() {
  __builtin_amdgcn_wave_barrier();
  __asm__ __volatile__("" ::: "memory");
}

// Entries per wave of the leader table (a power of two); hash of a cell index into it.
constexpr int ART_HTAB = 256;
__device__ __forceinline__ uint32_t cell_hash(int32_t vi) { return ((uint32_t)vi * 2654435761u) >> 24; }

// Deposits of one step of a wave's packets.  Neighbouring lanes walk neighbouring directions,
// so several of them often add into the same cell in the same step; global atomics to one
// address serialise, so the lanes of a cell first agree on one leader: each depositing lane
// writes its lane number at its cell's hash in the wave's table, and the number left there
// leads every lane of that cell; cells that lost their entry to another cell pick leaders in
// a loop over their distinct cells.  Where no two lanes share a cell each lane deposits its
// own values; otherwise each leader stores its NV values in its LDS slot, the other lanes of
// its cell add theirs there, and the leaders alone update the fields f[0 .. NV-1] at the cell.
// Cell indices are below 2^31 (checked on the host), so a key is one 32-bit word.
template <class R, int NV>
__device__ __forceinline__ void wave_deposit(R *const f[NV], R *slot, int *htab, bool dep, int32_t vi,
                                             const double v[NV]) {
  const int lane = threadIdx.x & 63;
  if (!__ballot(dep)) return;
  const uint32_t h = cell_hash(vi);
  if (dep) htab[h] = lane;
  lane_exchange();
  int leader = dep ? htab[h] : lane;
  lane_exchange();
  const int32_t wkey = __shfl(vi, leader);
  uint64_t pend = __ballot(dep && wkey != vi);
  while (pend) {
    const int first = __builtin_ctzll(pend);
    const int32_t key = __builtin_amdgcn_readlane(vi, first);
    const bool same = dep && vi == key;
    if (same) leader = first;
    pend &= ~__ballot(same);
  }
  R t[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) t[k] = (R)v[k];
  const bool lead = dep && leader == lane;
  const bool follow = dep && leader != lane;
  if (__ballot(follow)) {
    using V = typename Vec16<R>::T;
    constexpr int W = Vec16<R>::n, NW = (NV + W - 1) / W, S = SlotStride<R, NV>::v;
    static_assert(S >= NW * W && (S * sizeof(R)) % 16 == 0, "slot stride");
    V *mine = reinterpret_cast<V *>(slot + S * lane);
    if (lead) {
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        R q[W];
#pragma unroll
        for (int e = 0; e < W; ++e) q[e] = W * w + e < NV ? t[W * w + e] : R(0);
        V x;
        __builtin_memcpy(&x, q, sizeof(V));
        mine[w] = x;
      }
    }
    lane_exchange();
    if (follow) {
      R *dst = slot + S * leader;
#pragma unroll
      for (int k = 0; k < NV; ++k) atomicAdd(dst + k, t[k]);
    }
    lane_exchange();
    if (lead) {
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const V x = mine[w];
        R q[W];
        __builtin_memcpy(q, &x, sizeof(V));
#pragma unroll
        for (int e = 0; e < W; ++e)
          if (W * w + e < NV) t[W * w + e] = q[e];
      }
    }
    lane_exchange();
  }
  if (lead) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
      if (t[k] != R(0)) atomicAdd(f[k] + vi, t[k]);
  }
}

template <class R, bool FLUX>
__global__ __launch_bounds__(256) void art_level_kernel(ArtArgs a) {
  constexpr int NV = FLUX ? 14 : 5;
  constexpr int SS = SlotStride<R, NV>::v;
  __shared__ double s_cs[CS_NX * CS_NY];
  __shared__ __align__(16) R s_slot[256 * SS];  // per lane: its cell's NV sums while it leads
  __shared__ int s_htab[4 * ART_HTAB];          // per wave: the leader table
  extern __shared__ double s_budget[];  // [nsrc][6] when a.budget is set
  load_cs(a.tab, s_cs);
  if (a.budget) {
    for (int k = threadIdx.x; k < 6 * a.nsrc; k += blockDim.x) s_budget[k] = 0.0;
    __syncthreads();
  }
  R *slot = s_slot + SS * 64 * (threadIdx.x >> 6);
  int *htab = s_htab + ART_HTAB * (threadIdx.x >> 6);
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = id < a.nin;
  const int level = a.level;
  const double nray = 12.0 * (double)(1ll << (2 * level));
  const int dims[3] = {a.nx, a.ny, a.nz};
  ArtRay ray{};
  if (live) {
    if (a.in) {
      ray = a.in[id];
    } else {
      const int64_t np0 = 12ll << (2 * level);
      ray.src = (uint16_t)(id / np0);
      ray.pix = (uint32_t)(id % np0);
    }
  }
  const SrcDev S = g_src[live ? ray.src : 0];
  const double s[3] = {S.x, S.y, S.z};
  double u[3];
  healpix_dir(level, live ? ray.pix : 0u, u);
  int c[3], step[3];
  double tmax[3], inv[3];
  bool inside = live;
  double r = ray.r;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double pq = s[q] + r * u[q];
    c[q] = (int)floor(pq);
    inside = inside && pq >= 0.0 && c[q] < dims[q];
    if (u[q] > 0.0) {
      step[q] = 1;
      inv[q] = 1.0 / u[q];
      tmax[q] = ((double)(c[q] + 1) - s[q]) * inv[q];
    } else if (u[q] < 0.0) {
      step[q] = -1;
      inv[q] = 1.0 / u[q];
      tmax[q] = ((double)c[q] - s[q]) * inv[q];
    } else {
      step[q] = 0;
      inv[q] = 0.0;
      tmax[q] = 1e300;
    }
  }
  // distance to the domain exit; a packet whose next piece would start within EXIT_TOL cells
  // of it has left (a plane crossing that coincides with the exit, up to rounding, must not
  // count as a cell entry)
  double r_exit = 1e300;
#pragma unroll
  for (int q = 0; q < 3; ++q)
    if (step[q] != 0) r_exit = fmin(r_exit, ((step[q] > 0 ? (double)dims[q] : 0.0) - s[q]) * inv[q]);
  const double Lfuv = S.L / nray, Lq = S.Q / nray;
  double NH = ray.NH, NH2 = ray.NH2, NC = ray.NC, tL = ray.tauLyC;
  double ePE = (double)Mx<R>::ex(-a.sPE * NH), eLW = (double)Mx<R>::ex(-a.sLW * NH);
  double eL = (double)Mx<R>::ex(-tL);
  bool split = false, dropped = false, active = inside;
  const int max_steps = a.nx + a.ny + a.nz + 3;
  int it = 0;
  // one cell per trip, uniform over the wave so that its deposits can be combined
  while (__ballot(active)) {
    // arguments re-read per trip (see kernel_args): none of them is held across the walk
    const ArtArgs &A = kernel_args<ArtArgs>();
    bool dep = false;
    int32_t vi = 0;
    double v[NV];
    if (active) {
      if (++it > max_steps) {
        active = false;
      } else {
        const int q = tmax[0] <= tmax[1] ? (tmax[0] <= tmax[2] ? 0 : 2) : (tmax[1] <= tmax[2] ? 1 : 2);
        const double rn = tmax[q];
        if (rn > r) {
          // a piece of positive length starts here: the checks at its entry face
          if (r >= r_exit - EXIT_TOL) {
            active = false;
          } else if (fmin(fmin(A.sPE * NH, A.sLW * NH), tL) > A.tau_max) {
            active = false;
            dropped = true;
          } else if (level < A.max_level && r * r > A.R2split) {
            active = false;
            split = true;
          } else {
            const double ds = (rn - r) * A.dx;
            vi = c[0] + A.nx * (c[1] + A.ny * c[2]);
            const double nn = A.n[vi], x2 = A.xH2[vi], xp = A.xHp[vi];
            const double xc = A.xC ? A.xC[vi] : 0.0;
            const double xHI = fmax(1.0 - 2.0 * x2 - xp, 0.0);
            const double aL = nn * (xHI * A.spiH + x2 * A.spiH2 + A.sdLyC);
            double gPE, gLW, gL, fPE, fLW, fL;
            absorb<R>(A.sPE * nn * ds, gPE, fPE);
            absorb<R>(A.sLW * nn * ds, gLW, fLW);
            absorb<R>(aL * ds, gL, fL);
            const double mH2 = NH2 + 0.5 * nn * x2 * ds, mC = NC + 0.5 * nn * xc * ds;
            const double wLW = Lfuv * eLW * ds * gLW * A.fuv_norm;
            v[0] = Lfuv * ePE * ds * gPE * A.fuv_norm;
            v[1] = wLW;
            v[2] = wLW * f_shld_H2<R>(mH2);
            v[3] = wLW * f_shld_C<R>(mC, mH2, s_cs);
            v[4] = Lq * eL * ds * gL * A.phi_norm;
            if constexpr (FLUX) {
#pragma unroll
              for (int q2 = 0; q2 < 3; ++q2) {
                v[5 + q2] = A.kPE * v[0] * u[q2];
                v[8 + q2] = A.kLW * v[1] * u[q2];
                v[11 + q2] = v[4] * u[q2];
              }
            }
            dep = true;
            NH += nn * ds;
            NH2 += nn * x2 * ds;
            NC += nn * xc * ds;
            tL += aL * ds;
            ePE *= fPE;
            eLW *= fLW;
            eL *= fL;
            r = rn;
          }
        }
        if (active) {
          c[q] += step[q];
          if (c[q] < 0 || c[q] >= dims[q])
            active = false;
          else
            tmax[q] = ((double)(step[q] > 0 ? c[q] + 1 : c[q]) - s[q]) * inv[q];
        }
      }
    }
    R *fields[NV];
    fields[0] = (R *)A.chiPE;
    fields[1] = (R *)A.chiLW;
    fields[2] = (R *)A.chiH2;
    fields[3] = (R *)A.chiC;
    fields[4] = (R *)A.phi;
    if constexpr (FLUX) {
#pragma unroll
      for (int k = 0; k < 9; ++k) fields[5 + k] = (R *)A.flux + (int64_t)k * A.ncell;
    }
    wave_deposit<R, NV>(fields, slot, htab, dep, vi, v);
  }
  if (live && a.budget && !split) {
    // the packet ends here: lost through the boundary or dropped at tau > tau_max
    const int o = 6 * ray.src + (dropped ? 3 : 0);
    atomicAdd(&s_budget[o + 0], S.L * exp(-a.sPE * NH) / nray);
    atomicAdd(&s_budget[o + 1], S.L * exp(-a.sLW * NH) / nray);
    atomicAdd(&s_budget[o + 2], S.Q * exp(-tL) / nray);
  }
  ray.r = r;
  ray.NH = NH;
  ray.NH2 = NH2;
  ray.NC = NC;
  ray.tauLyC = tL;
  // children of the split packets: one reservation per wave
  const uint64_t mask = __ballot(split);
  if (mask) {
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(a.nout, 4ull * (unsigned long long)__popcll(mask));
    base = __shfl(base, leader);
    if (split) {
      const unsigned long long k = base + 4ull * __popcll(mask & ((1ull << lane) - 1ull));
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) {
        ArtRay cr = ray;
        cr.pix = 4u * ray.pix + (uint32_t)ch;
        a.out[k + ch] = cr;
      }
    }
  }
  if (a.budget) {
    __syncthreads();
    for (int k = threadIdx.x; k < 6 * a.nsrc; k += blockDim.x)
      if (s_budget[k] != 0.0) atomicAdd(&a.budget[k], s_budget[k]);
  }
}

// Radiation force per volume on the gas-dust mixture (Sec. 6.2): sum over bands of
// alpha_j F_j / c with the trace's opacities (PE, LW: dust; LyC: dust, H and H2) and h nu_LyC
// per LyC photon.  Grains count as destroyed (appendix on grain destruction) where T exceeds
// T_destroy or P_rad = |F| / c exceeds prad_ratio_max times P = 2 n k_B T, F the total flux of
// the three bands; there the dust part is dropped and only LyC photoionisation pushes.  With
// mom the momentum density takes f dt, and with etot the total energy the change of
// rho v^2 / 2 at rho = mu_H m_H n.  All arithmetic in double; one thread per cell.
struct ForceArgs {
  int64_t ncell;
  const double *n, *T, *xH2, *xHp;
  const void *flux;   // 9 x ncell, the path's precision
  void *f;            // 3 x ncell, the path's precision
  uint8_t *dust_off;  // or null
  double *mom, *etot; // or null
  double dt;
  double T_destroy, prad_ratio_max;
  double sPE, sLW, sdLyC, spiH, spiH2;  // dust cross sections x Z'_d; photoionisation
  double hnu, inv_c, two_kB, rho_per_n;
};

template <class R>
__global__ __launch_bounds__(256) void radiation_force_kernel(ForceArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.ncell) return;
  const R *F = (const R *)a.flux;
  const int64_t N = a.ncell;
  double Fb[3][3];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int q = 0; q < 3; ++q) Fb[b][q] = (double)F[(3 * b + q) * N + i];
#pragma unroll
  for (int q = 0; q < 3; ++q) Fb[2][q] *= a.hnu;
  const double nn = a.n[i], T = a.T[i], x2 = a.xH2[i], xp = a.xHp[i];
  double F2 = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double t = Fb[0][q] + Fb[1][q] + Fb[2][q];
    F2 += t * t;
  }
  const double prad = sqrt(F2) * a.inv_c;
  const bool off = T > a.T_destroy || prad > a.prad_ratio_max * (a.two_kB * nn * T);
  const double keep = off ? 0.0 : 1.0;
  const double xHI = fmax(1.0 - 2.0 * x2 - xp, 0.0);
  const double agas = nn * (xHI * a.spiH + x2 * a.spiH2);
  double f[3];
#pragma unroll
  for (int q = 0; q < 3; ++q)
    f[q] = (keep * nn * (a.sPE * Fb[0][q] + a.sLW * Fb[1][q] + a.sdLyC * Fb[2][q]) + agas * Fb[2][q]) * a.inv_c;
  R *fo = (R *)a.f;
#pragma unroll
  for (int q = 0; q < 3; ++q) fo[q * N + i] = (R)f[q];
  if (a.dust_off) a.dust_off[i] = off ? 1 : 0;
  if (a.mom) {
    double p0[3], p1[3], d2 = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      p0[q] = a.mom[q * N + i];
      p1[q] = p0[q] + f[q] * a.dt;
      a.mom[q * N + i] = p1[q];
    }
    if (a.etot) {
      const double rho = a.rho_per_n * nn;
      if (rho > 0.0) {
        d2 = (p1[0] * p1[0] + p1[1] * p1[1] + p1[2] * p1[2]) - (p0[0] * p0[0] + p0[1] * p0[1] + p0[2] * p0[2]);
        a.etot[i] += d2 / (2.0 * rho);
      }
    }
  }
}

__global__ void art_zero_kernel(double *p, int64_t n, unsigned long long *cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
  if (i == 0 && cnt) *cnt = 0ull;
}

}  // namespace ism
