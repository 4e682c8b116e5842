// Source-step kernels: the subcycled heating/cooling + chemistry update (Sec. 6.1)
// and the per-cell diagnostics of the microphysics.
#pragma once
#include "physics.h"

namespace ism {

__constant__ CoefT<double> g_coef64;
__constant__ CoefT<float> g_coef32;

// The double coefficients through a pointer laundered by an empty asm at each use site: the
// compiler may not hoist their scalar loads out of the substep loop, which otherwise keeps
// hundreds of constants live across it and spills them into vector registers.
__device__ __forceinline__ const CoefT<double> &coef64() {
  const __attribute__((address_space(4))) CoefT<double> *p =
      (const __attribute__((address_space(4))) CoefT<double> *)&g_coef64;
  asm volatile("" : "+s"(p));
  return *(const CoefT<double> *)p;
}

template <class R> __device__ __forceinline__ const CoefT<R> &coef();
template <> __device__ __forceinline__ const CoefT<double> &coef<double>() { return coef64(); }
template <> __device__ __forceinline__ const CoefT<float> &coef<float>() {
  const __attribute__((address_space(4))) CoefT<float> *p =
      (const __attribute__((address_space(4))) CoefT<float> *)&g_coef32;
  asm volatile("" : "+s"(p));
  return *(const CoefT<float> *)p;
}

template <class R> struct CloseTol;
template <> struct CloseTol<double> { static constexpr double v = 1e-12; };
template <> struct CloseTol<float> { static constexpr float v = 2.5e-7f; };

template <class R>
struct StepArgs {
  int64_t ncell;
  double dt;
  const double *n;
  double *T, *xH2, *xHp;
  const R *chiPE, *chiLW, *chiH2, *chiC, *phi, *xi, *Neff;
  R *xCp, *xCO, *xe;
  int32_t *nsub;
  uint8_t *status;
  const R *tab;
  ParT<R> pr;
  ParT<double> pd;
  int64_t *queue;  // persistent variant: next unclaimed cell (device counter), else unused
  // persistent variant only: when idx is set, work item k is cell idx[k] and the item count
  // is *count (read on the device); st_or is or-ed into every status written
  const int32_t *idx;
  const unsigned long long *count;
  uint32_t st_or;
};

// Per-lane state of one cell while it is being subcycled.
template <class R>
struct CellState {
  double nd, K, Tmu, xH2, xHp, t;
  Rad<R> *r;  // the cell's radiation and fixed terms: the lane's slot in LDS (it frees 24
              // registers a lane in FP64, read once or twice per evaluation)
  EqS<R> e;
  double tdi, tds;  // the last dust temperature as a line in T: T_d ~ tdi + tds T
  int32_t ns;
  uint32_t st;
};

template <class R>
__device__ __forceinline__ void cell_begin(const StepArgs<R> &a, int64_t i, CellState<R> &s, const R *tab) {
  const CoefT<R> &c = coef<R>();
  s.nd = a.n[i];
  Rad<R> rr;
  rr.chiPE = a.chiPE[i];
  rr.chiLW = a.chiLW[i];
  rr.chiH2 = a.chiH2[i];
  rr.chiC = a.chiC[i];
  rr.phi = a.phi ? a.phi[i] : R(0);
  rr.xi = a.xi[i];
  rr.Neff = a.Neff[i];
  fixed_terms(rr, s.nd, c, a.pr);
  *s.r = rr;
  const double T0 = a.T[i];
  s.xH2 = a.xH2[i];
  s.xHp = a.xHp[i];
  const double muH = a.pd.muH;
  s.K = s.nd * muH * K_B / (g_coef64.gamma - 1.0);
  s.e = eq_species<R>(T0, R(s.nd), s.xH2, s.xHp, *s.r, c, a.pr, tab, CloseTol<R>::v, 50);
  s.Tmu = T0 * (1.1 + (double)s.e.xe - s.xH2) / muH;
  s.t = 0.0;
  s.ns = 0;
  s.st = 0;
  s.tdi = 0.0;  // no dust temperature yet: the first solve starts cold
  s.tds = 0.0;
}

// One substep of Sec. 6.1 for the lane's cell; returns true when the cell is finished.
template <class R>
__device__ __forceinline__ bool cell_substep(const StepArgs<R> &a, CellState<R> &s, const R *tab) {
  const CoefT<R> &c = coef<R>();
  const ParT<R> &p = a.pr;
  const double muH = a.pd.muH, eps = a.pd.eps_sub, delta = a.pd.fd_rel, dt = a.dt;
  const double mu_den = 1.1 + (double)s.e.xe - s.xH2;
  // quotients whose denominators are positive and of normal size (mu, T_mu, K, the update's
  // determinant >= 1): the reciprocal-based division
  const double Ta = fdivp(muH * s.Tmu, mu_den);
  // H at T and at T (1 + fd_rel): one instance of the evaluation, run twice.  Each dust
  // temperature solve starts from the last one carried along its slope.
  Tq qk = make_tq<R>(Ta);
  const PreLogs pre = pre_logs<R>(R(s.nd), s.e, p);
  Eval<R> v;
  double H2 = 0.0;
  bool td_bad = false;
#pragma unroll 1
  for (int k = 0; k < 2; ++k) {
    const Eval<R> w = evaluate<R, false, false>(qk, s.nd, s.xH2, s.xHp, s.e, *s.r, c, p, tab,
                                                s.tdi + s.tds * qk.T, nullptr, k == 0, &pre);
    td_bad = td_bad || w.td_bad;
    if (k == 0) {
      v = w;
      s.tds = w.Tds;
      s.tdi = w.Td - w.Tds * Ta;
      qk = shift_tq<R>(qk, a.pd);
    } else {
      H2 = w.H;
    }
  }
  const double H = v.H;
  const double en = s.K * s.Tmu;
  const double rem = dt - s.t;
  double dts = rem;
  const double aH = fabs(H), a1 = fabs((double)v.CH2), a2 = fabs((double)v.CHp);
  if (aH > 0.0) dts = fmin(dts, eps * en / aH);
  if (a1 > 0.0) dts = fmin(dts, eps / a1);
  if (a2 > 0.0) dts = fmin(dts, eps / a2);
  const double dH = fdivp(H2 - H, delta * s.Tmu);
  double den = s.K - dts * dH;
  if (den <= 0.1 * s.K) { den = s.K; s.st |= ISM_ST_DENOM_GUARD; }
  if (td_bad) s.st |= ISM_ST_TD_UNBRACKETED;
  double Tmu_new = s.Tmu + fdivp(dts * H, den);
  const double Tmu_min = fdivp(a.pd.T_floor * mu_den, muH);
  if (Tmu_new < Tmu_min) { Tmu_new = Tmu_min; s.st |= ISM_ST_T_FLOOR; }
  // abundances: rate coefficients at T^{n+1} = mu^n T_mu^{n+1}, abundance factors frozen at step n
  const double Tp = fdivp(muH * Tmu_new, mu_den);
  const Tq qp = make_tq<R>(Tp);  // shared by the rates and the closure at T^{n+1}
  Eval<R> vc = evaluate<R, true, false>(qp, s.nd, s.xH2, s.xHp, s.e, *s.r, c, p, tab, 0.0, nullptr);
  const double F = vc.F, D = vc.D, I = vc.I, Rr = vc.Rr;
  const double det = 1.0 + dts * (2.0 * F + D + I + Rr) + dts * dts * (2.0 * F * Rr + D * I + D * Rr);
  const double idet = fdivp(1.0, det);
  const double xa = (s.xH2 * (1.0 + dts * (I + Rr)) + F * dts * (1.0 - s.xHp) + F * dts * dts * Rr) * idet;
  const double xb = (s.xHp * (1.0 + dts * (2.0 * F + D)) + I * dts * (1.0 - 2.0 * s.xH2) + I * dts * dts * D) * idet;
  s.e = eq_species<R>(qp, R(s.nd), xa, xb, *s.r, c, p, tab, CloseTol<R>::v, 50);
  const bool fin = isfinite(Tmu_new) && isfinite(xa) && isfinite(xb);
  if (!fin) s.st |= ISM_ST_NONFINITE;
  const bool last = (dts == rem);
  s.t = last ? dt : s.t + dts;
  s.ns += 1;
  const bool cap = (s.ns >= a.pd.max_sub) && !last;
  if (cap) s.st |= ISM_ST_SUBSTEP_CAP;
  s.Tmu = Tmu_new;
  s.xH2 = xa;
  s.xHp = xb;
  return last || cap || !fin;
}

template <class R>
__device__ __forceinline__ void cell_end(const StepArgs<R> &a, int64_t i, const CellState<R> &s) {
  a.T[i] = a.pd.muH * s.Tmu / (1.1 + (double)s.e.xe - s.xH2);
  a.xH2[i] = s.xH2;
  a.xHp[i] = s.xHp;
  if (a.xCp) a.xCp[i] = s.e.xCp;
  if (a.xCO) a.xCO[i] = s.e.xCO;
  if (a.xe) a.xe[i] = s.e.xe;
  if (a.nsub) a.nsub[i] = s.ns;
  if (a.status) a.status[i] = (uint8_t)(s.st | a.st_or);
}

template <class R>
__device__ __forceinline__ void stage_tables(const R *g, R *s_tab) {
  for (int k = threadIdx.x; k < TAB_STEP; k += blockDim.x) s_tab[k] = g[k];
  __syncthreads();
}

// One lane per cell, a plain 1-D grid.
template <class R>
__global__ __launch_bounds__(256) void step_simple_kernel(StepArgs<R> a) {
  __shared__ R s_tab[TAB_STEP];
  stage_tables(a.tab, s_tab);
  __shared__ Rad<R> s_rad[256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.ncell) return;
  CellState<R> s;
  s.r = &s_rad[threadIdx.x];
  cell_begin(a, i, s, s_tab);
  while (!cell_substep(a, s, s_tab)) {
  }
  cell_end(a, i, s);
}

// Persistent variant: a grid sized to the chip; every lane keeps one cell in flight and,
// when its cell finishes, claims the next unclaimed cell from a device counter (one
// atomic per wave per refill, ranks by popcount), so lanes stay busy however uneven the
// substep counts are.  A finished lane waits until REFILL_BATCH lanes of its wave are done
// (or no lane is still working): the whole wave runs the refill (loads, fixed terms, entry
// closure) whenever any lane takes it, so taking it for a dozen lanes at once beats taking it
// for one or two lanes in nearly every pass.  Every lane leaves once the counter passes ncell
// and its cell is done; *a.queue must hold the number of lanes in the grid at launch.
// Waves per SIMD: three for the FP64 kernel (168 registers a lane), four for the mixed one (128):
// more waves hide more of the long dependent transcendental sequences than fewer waves with more
// registers do.  The kernels fit there because the lane's radiation terms live in LDS and the
// cooling terms are summed as they are formed.
constexpr int REFILL_BATCH = 12;
template <class R> struct StepWaves { static constexpr int v = 3; };
template <> struct StepWaves<float> { static constexpr int v = 4; };

template <class R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(StepWaves<R>::v))) void step_queue_kernel(
    StepArgs<R>) {
  using A = StepArgs<R>;
  __shared__ R s_tab[TAB_STEP];
  stage_tables(kernel_args<A>().tab, s_tab);
  const int lane = threadIdx.x & 63;
  const int64_t nitem = kernel_args<A>().count ? (int64_t)*kernel_args<A>().count : kernel_args<A>().ncell;
  int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool active = cell < nitem;
  __shared__ Rad<R> s_rad[256];
  CellState<R> s;
  s.r = &s_rad[threadIdx.x];
  if (active) {
    const A &a = kernel_args<A>();
    cell_begin(a, a.idx ? (int64_t)a.idx[cell] : cell, s, s_tab);
  }
  bool idle = false;  // cell finished, waiting for the wave's next refill
  while (__ballot(active || idle) != 0) {
    if (active && cell_substep(kernel_args<A>(), s, s_tab)) {
      const A &a = kernel_args<A>();
      cell_end(a, a.idx ? (int64_t)a.idx[cell] : cell, s);
      active = false;
      idle = true;
    }
    const uint64_t m = __ballot(idle);
    if (m != 0 && (__popcll(m) >= REFILL_BATCH || __ballot(active) == 0)) {
      const A &a = kernel_args<A>();
      const int leader = __ffsll((unsigned long long)m) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd((unsigned long long *)a.queue, (unsigned long long)__popcll(m));
      base = __shfl(base, leader, 64);
      if (idle) {
        idle = false;
        cell = (int64_t)base + __popcll(m & ((1ull << lane) - 1ull));
        active = cell < nitem;
        if (active) cell_begin(a, a.idx ? (int64_t)a.idx[cell] : cell, s, s_tab);
      }
    }
  }
}

__global__ void queue_init_kernel(int64_t *q, int64_t v) { *q = v; }

// Per-cell diagnostics (ism_rates).
template <class R>
struct RatesArgs {
  int64_t ncell;
  const double *n, *T, *xH2, *xHp;
  const R *chiPE, *chiLW, *chiH2, *chiC, *phi, *xi, *Neff;
  R *out;
  const R *tab;
  ParT<R> pr;
};

template <class R>
__global__ __launch_bounds__(128) void rates_kernel(RatesArgs<R> a) {
  __shared__ R s_tab[TAB_STEP];
  stage_tables(a.tab, s_tab);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.ncell) return;
  const CoefT<R> &c = coef<R>();
  Rad<R> r;
  r.chiPE = a.chiPE[i];
  r.chiLW = a.chiLW[i];
  r.chiH2 = a.chiH2[i];
  r.chiC = a.chiC[i];
  r.phi = a.phi ? a.phi[i] : R(0);
  r.xi = a.xi[i];
  r.Neff = a.Neff[i];
  const double nd = a.n[i];
  fixed_terms(r, nd, c, a.pr);
  const double T = a.T[i];
  const double xH2 = a.xH2[i], xHp = a.xHp[i];
  EqS<R> e = eq_species<R>(T, R(nd), xH2, xHp, r, c, a.pr, s_tab, CloseTol<R>::v, 50);
  R d[NDIAG];
  evaluate<R, false, true>(T, nd, xH2, xHp, e, r, c, a.pr, s_tab, R(0), d);
#pragma unroll
  for (int k = 0; k < NDIAG; ++k) a.out[(int64_t)k * a.ncell + i] = d[k];
}

}  // namespace ism
