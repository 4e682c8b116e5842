// Acceptance of learned predictions for the source step.
//
// The plain subcycled step is path dependent wherever a cell's relaxation times are comparable
// to dt, so a predicted post-step state can stand in for it only where the plain result no
// longer depends on the path: all three variables (T, x_H2, x_H+) relax much faster than dt
// and the cell ends at the equilibrium of the coupled system.  A prediction is accepted when
//   1. Newton from the prediction converges to a root of
//        g = (dT/dt, C_H2, C_H+) = (H mu_H / ((1.1 + x_e - x_H2) K), C_H2, C_H+)
//      (Jacobian by forward differences, equilibrium C/O/e re-solved at every probe),
//   2. every eigenvalue of the Jacobian at the root has real part below -fast/dt (Routh-Hurwitz
//      on J + (fast/dt) I), so the linearised dynamics contract by e^-fast over the step,
//   3. the root lies within a factor e^0.1 in T of the prediction (basin of the prediction),
//   4. T moves from T_0 toward the root: dT/dt at the input state and at three temperatures
//      log-spaced between T_0 and the root (abundances at the root) all have the sign of
//      T_root - T_0, so no other thermal equilibrium lies between them,
//   5. the plain step's own end state is at the root to the output tolerance.  Near the root
//      the plain step's last substep is one long implicit jump whose coefficients are frozen
//      at the state it starts from, so its end state lags the root by L' (Y_prev - Y_root),
//      L' the sensitivity of that jump to its starting state.  L' is taken by forward
//      differences of one substep of length dt started at the root and at the root perturbed
//      in each variable; the starting state of the last jump lies between the input state and
//      the root, so |Y_prev - Y_root| <= |Y_0 - Y_root| componentwise, and the cell is
//      accepted when sum_v |L'_wv| |Y_0,v - Y_root,v| <= out_tol / 2 of each output's scale
//      (and the unperturbed jump reproduces the root).
// Before any prediction, a pre-test on the input state (surr_pretest_kernel) requires both
// chemical relaxation rates and the thermal one to be fast there as well: the plain step's path
// starts at the input state, and a cell that relaxes slowly there does so along a path its end
// state depends on.
// Only the cells that pass are predicted and certified; the same test at the seed opens the
// certification.  Accepted cells take the root (equilibrium C/O/e at the root); the others are
// appended to a list for the plain step.
#pragma once
#include "kernels_step.h"

namespace ism {

struct AcceptArgs {
  const int32_t *cand;              // candidate cells (listed by surr_pretest_kernel)
  const unsigned long long *ncand;  // their number (device counter)
  double dt;
  const double *n;
  double *T, *xH2, *xHp;
  const float *chiPE, *chiLW, *chiH2, *chiC, *phi, *xi, *Neff;
  float *xCp, *xCO, *xe;
  int32_t *nsub;
  uint8_t *status;
  const float *pred;  // [candidate][3] predicted x_H2, x_H+, log10 T; null = the input state itself
  const float *tab;
  ParT<float> pr;
  ParT<double> pd;
  int32_t *rej;                 // rejected cells, appended (order unspecified)
  unsigned long long *nrej;     // number of rejected cells (device counter)
  double fast;                  // required dt * rate margin
  double tol;                   // relative Newton convergence tolerance
  int maxit;
  double out_tol;               // relative tolerance the accepted outputs must meet
};

__device__ __forceinline__ bool hurwitz_shifted(const double (&J)[3][3], double s) {
  double M[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) M[a][b] = J[a][b] + (a == b ? s : 0.0);
  const double tr = M[0][0] + M[1][1] + M[2][2];
  const double m2 = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) + (M[0][0] * M[2][2] - M[0][2] * M[2][0]) +
                    (M[1][1] * M[2][2] - M[1][2] * M[2][1]);
  const double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                     M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                     M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
  const double c2 = -tr, c1 = m2, c0 = -det;
  return c2 > 0.0 && c0 > 0.0 && c2 * c1 > c0;
}

// Solve J d = -g by Cramer's rule; false if singular.
__device__ __forceinline__ bool solve3(const double (&J)[3][3], const double (&g)[3], double (&d)[3]) {
  const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  if (!(fabs(det) > 0.0) || !isfinite(det)) return false;
  const double inv = 1.0 / det;
  // adjugate rows
  const double a10 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  const double a11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  const double a12 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  const double a20 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  const double a21 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  const double a22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  d[0] = -(c00 * g[0] + a10 * g[1] + a20 * g[2]) * inv;
  d[1] = -(c01 * g[0] + a11 * g[1] + a21 * g[2]) * inv;
  d[2] = -(c02 * g[0] + a12 * g[1] + a22 * g[2]) * inv;
  return isfinite(d[0]) && isfinite(d[1]) && isfinite(d[2]);
}

// Both chemical relaxation rates must be fast on their own: dt (2 F + D) and dt (I + R) at
// least fast / 2 (a NaN passes here and fails the Newton solve).
__device__ __forceinline__ bool chem_fast(const Eval<float> &v, double dt, double fast) {
  return !(dt * (2.0 * (double)v.F + (double)v.D) < 0.5 * fast || dt * ((double)v.I + (double)v.Rr) < 0.5 * fast);
}

__device__ __forceinline__ void load_rad(Rad<float> &r, const float *chiPE, const float *chiLW, const float *chiH2,
                                         const float *chiC, const float *phi, const float *xi, const float *Neff,
                                         int64_t i) {
  r.chiPE = chiPE[i];
  r.chiLW = chiLW[i];
  r.chiH2 = chiH2[i];
  r.chiC = chiC[i];
  r.phi = phi ? phi[i] : 0.f;
  r.xi = xi[i];
  r.Neff = Neff[i];
}

// Append v to list for the lanes that take it: one atomic per wave, ranks by popcount.  Called
// by every lane of the wave.
__device__ __forceinline__ void wave_append(bool take, int32_t v, int32_t *list, unsigned long long *cnt) {
  const uint64_t m = __ballot(take);
  if (m == 0) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((unsigned long long)m) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(cnt, (unsigned long long)__popcll(m));
  base = __shfl(base, leader, 64);
  if (take) list[base + __popcll(m & ((1ull << lane) - 1ull))] = v;
}

// Append v to list a (take) or to list b (otherwise) for every live thread of the block: one
// global atomic per block and list, ranks from the waves' ballots.  Called by every thread of the
// block (it synchronises the block).  A single
// counter taking one atomic from every wave of a large grid serialises them, so the lists the
// pre-test builds from every cell are appended per block; the certification, whose lanes diverge
// and whose list is short, appends per wave.
template <int NT>
__device__ __forceinline__ void block_append2(bool live, bool take, int32_t v, int32_t *la, unsigned long long *ca,
                                              int32_t *lb, unsigned long long *cb) {
  constexpr int NW = NT / 64;
  __shared__ uint32_t s_cnt[2][NW];
  __shared__ unsigned long long s_base[2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t ma = __ballot(live && take), mb = __ballot(live && !take);
  if (lane == 0) {
    s_cnt[0][w] = (uint32_t)__popcll(ma);
    s_cnt[1][w] = (uint32_t)__popcll(mb);
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    uint32_t tot = 0;
    for (int k = 0; k < NW; ++k) tot += s_cnt[threadIdx.x][k];
    s_base[threadIdx.x] = tot ? atomicAdd(threadIdx.x == 0 ? ca : cb, (unsigned long long)tot) : 0ull;
  }
  __syncthreads();
  const int which = take ? 0 : 1;
  unsigned long long off = s_base[which];
  for (int k = 0; k < w; ++k) off += s_cnt[which][k];
  const uint64_t m = take ? ma : mb;
  if (live) (take ? la : lb)[off + __popcll(m & ((1ull << lane) - 1ull))] = v;
  __syncthreads();  // the counts are read before a later call rewrites them
}

struct PreArgs {
  int64_t ncell;
  double dt;
  const double *n, *T, *xH2, *xHp;
  const float *chiPE, *chiLW, *chiH2, *chiC, *phi, *xi, *Neff;
  const float *tab;
  ParT<float> pr;
  ParT<double> pd;
  double fast;
  const int32_t *in;                 // thermal test: the cells to test
  const unsigned long long *nin;     //   and their number (device counter)
  int32_t *pass, *rej;               // cells that pass, cells that fall back (appended, order unspecified)
  unsigned long long *npass, *nrej;  // their counts (device counters)
};

// Closure iterations of the pre-test: the test compares rates with a threshold, so the closure
// need not converge (x_e after four fixed-point iterations from x_e0 + x_C,tot).
constexpr int PRETEST_CLOSE_IT = 4;

__device__ __forceinline__ void pre_cell(const PreArgs &a, int64_t i, Rad<float> &r, EqS<float> &e, double &nd,
                                         double &T0, double &x20, double &xp0, const float *s_tab) {
  const CoefT<float> &c = coef<float>();
  nd = a.n[i];
  load_rad(r, a.chiPE, a.chiLW, a.chiH2, a.chiC, a.phi, a.xi, a.Neff, i);
  fixed_terms(r, nd, c, a.pr);
  T0 = a.T[i];
  x20 = a.xH2[i];
  xp0 = a.xHp[i];
  e = eq_species<float>(T0, (float)nd, x20, xp0, r, c, a.pr, s_tab, CloseTol<float>::v, PRETEST_CLOSE_IT);
}

// The pre-test on the input state, first part, one lane per cell: both chemical relaxation rates
// fast (a chemistry-only probe: closure and rate coefficients).  Cells that pass go to the
// thermal test, the others to the fallback list.
constexpr int PRETEST_THREADS = 1024;
__global__ __launch_bounds__(PRETEST_THREADS) void surr_pretest_kernel(PreArgs a) {
  __shared__ float s_tab[TAB_STEP];
  stage_tables(a.tab, s_tab);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < a.ncell;
  bool pass = false;
  if (live) {
    Rad<float> r;
    EqS<float> e;
    double nd, T0, x20, xp0;
    pre_cell(a, i, r, e, nd, T0, x20, xp0, s_tab);
    const Eval<float> v =
        evaluate<float, true, false>(T0, nd, x20, xp0, e, r, coef<float>(), a.pr, s_tab, 0.f, nullptr);
    pass = chem_fast(v, a.dt, a.fast);
  }
  block_append2<PRETEST_THREADS>(live, pass, (int32_t)i, a.pass, a.npass, a.rej, a.nrej);
}

// Second part, over the cells that passed the first (grid-stride over blocks): the thermal
// relaxation rate -(dH/dT_mu) / K from the step's own forward difference (two evaluations of H,
// Sec. 6.1) must be fast as well.  Passing cells are the candidates for the network and the
// certification.
__global__ __launch_bounds__(256) void surr_pretest_thermal_kernel(PreArgs a) {
  __shared__ float s_tab[TAB_STEP];
  stage_tables(a.tab, s_tab);
  const int64_t nitem = (int64_t)*a.nin;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k0 = (int64_t)blockIdx.x * blockDim.x; k0 < nitem; k0 += stride) {
    const int64_t k = k0 + threadIdx.x;
    const bool live = k < nitem;
    const int64_t i = live ? (int64_t)a.in[k] : 0;
    bool pass = false;
    if (live) {
      Rad<float> r;
      EqS<float> e;
      double nd, T0, x20, xp0;
      pre_cell(a, i, r, e, nd, T0, x20, xp0, s_tab);
      const double muH = a.pd.muH;
      const double K = nd * muH * K_B / (g_coef64.gamma - 1.0);
      const double Tmu = T0 * (1.1 + (double)e.xe - x20) / muH;
      const Tq q = make_tq<float>(T0);
      const PreLogs pre = pre_logs<float>((float)nd, e, a.pr);
      const Eval<float> w0 =
          evaluate<float, false, false>(q, nd, x20, xp0, e, r, coef<float>(), a.pr, s_tab, 0.0, nullptr, false, &pre);
      const Eval<float> w1 = evaluate<float, false, false>(shift_tq<float>(q, a.pd), nd, x20, xp0, e, r, coef<float>(),
                                                           a.pr, s_tab, w0.Td, nullptr, false, &pre);
      const double dH = (w1.H - w0.H) / (a.pd.fd_rel * Tmu);
      pass = -dH * a.dt >= 0.5 * a.fast * K;  // false for a NaN as well
    }
    block_append2<256>(live, pass, (int32_t)i, a.pass, a.npass, a.rej, a.nrej);
  }
}

// Certification of candidate k (cell i): true when the prediction's root is accepted (and
// written to the cell's outputs).
__device__ __forceinline__ bool accept_cell(const AcceptArgs &a, int64_t k, int64_t i, const float *s_tab) {
  bool ok = false;
  {
    const CoefT<float> &c = coef<float>();
    const ParT<float> &p = a.pr;
    const double muH = a.pd.muH, dt = a.dt, delta = a.pd.fd_rel;
    const double nd = a.n[i];
    Rad<float> r;
    load_rad(r, a.chiPE, a.chiLW, a.chiH2, a.chiC, a.phi, a.xi, a.Neff, i);
    fixed_terms(r, nd, c, p);
    const double T0 = a.T[i], x20 = a.xH2[i], xp0 = a.xHp[i];
    const double K = nd * muH * K_B / (g_coef64.gamma - 1.0);
    // seed, clamped to the physical range
    double u[3];
    if (a.pred) {
      u[0] = exp10((double)a.pred[3 * k + 2]);
      u[1] = (double)a.pred[3 * k + 0];
      u[2] = (double)a.pred[3 * k + 1];
    } else {
      u[0] = T0;
      u[1] = x20;
      u[2] = xp0;
    }
    u[0] = fmin(fmax(u[0], a.pd.T_floor), 1e9);
    u[1] = fmin(fmax(u[1], 0.0), 0.5);
    u[2] = fmin(fmax(u[2], 0.0), 1.0);
    if (2.0 * u[1] + u[2] > 1.0) {
      const double f = 1.0 / (2.0 * u[1] + u[2]);
      u[1] *= f;
      u[2] *= f;
    }
    const double Tseed = u[0];
    const double srate = a.fast / fmax(dt, 1e-300);
    // pre-test on a chemistry-only probe (no heating, cooling or dust temperature): both
    // chemical relaxation rates must be fast on their own
    {
      const EqS<float> e = eq_species<float>(u[0], (float)nd, u[1], u[2], r, c, p, s_tab, CloseTol<float>::v, 50);
      const Eval<float> v = evaluate<float, true, false>(u[0], nd, u[1], u[2], e, r, c, p, s_tab, 0.f, nullptr);
      if (!chem_fast(v, dt, a.fast)) u[0] = -1.0;
    }
    double J[3][3], gb[3], h[3] = {0.0, 0.0, 0.0};
    int phase = 0, k = 0, it = 0;
    double dir = 0.0;
    double tdg = 0.0;
#pragma unroll 1
    for (; u[0] > 0.0;) {
      // arguments and coefficients laundered per iteration (kept out of scalar registers across the loop)
      const AcceptArgs &A = kernel_args<AcceptArgs>();
      const CoefT<float> &C = coef<float>();
      const ParT<float> &P = A.pr;
      // probe point
      double Tq = u[0], aq = u[1], bq = u[2];
      if (phase == 0) {
        if (k == 1) Tq = u[0] * (1.0 + delta);
        else if (k == 2) aq = u[1] + h[1];
        else if (k == 3) bq = u[2] + h[2];
      } else if (k == 0) {
        Tq = T0; aq = x20; bq = xp0;
      } else {
        Tq = T0 * exp((double)k * 0.25 * log(u[0] / T0));
      }
      const EqS<float> e = eq_species<float>(Tq, (float)nd, aq, bq, r, C, P, s_tab, CloseTol<float>::v, 50);
      const Eval<float> v = evaluate<float, false, false>(Tq, nd, aq, bq, e, r, C, P, s_tab, tdg, nullptr);
      tdg = v.Td;
      const double gT = v.H * muH / ((1.1 + (double)e.xe - aq) * K);
      const double g1 = v.CH2, g2 = v.CHp;
      if (phase == 0) {
        if (k == 0) {
          gb[0] = gT; gb[1] = g1; gb[2] = g2;
          // pre-test: both chemical relaxation rates must be fast on their own
          if (!chem_fast(v, dt, A.fast)) break;
          h[1] = 1e-3 * fmax(u[1], 1e-6);
          if (2.0 * (u[1] + h[1]) + u[2] > 1.0) h[1] = -h[1];
          h[2] = 1e-3 * fmax(u[2], 1e-6);
          if (2.0 * u[1] + u[2] + h[2] > 1.0) h[2] = -h[2];
          k = 1;
          continue;
        }
        const double step = k == 1 ? u[0] * delta : h[k - 1];
        J[0][k - 1] = (gT - gb[0]) / step;
        J[1][k - 1] = (g1 - gb[1]) / step;
        J[2][k - 1] = (g2 - gb[2]) / step;
        if (k < 3) { ++k; continue; }
        // full Jacobian at u
        if (it == 0 && !hurwitz_shifted(J, 0.5 * srate)) break;
        double d[3];
        if (!solve3(J, gb, d)) break;
        const double un0 = u[0] + d[0], un1 = u[1] + d[1], un2 = u[2] + d[2];
        const bool inside = un0 >= A.pd.T_floor && un0 <= 1e9 && un1 >= 0.0 && un2 >= 0.0 &&
                            2.0 * un1 + un2 <= 1.0;
        const bool conv = inside && fabs(d[0]) <= A.tol * un0 && fabs(d[1]) <= A.tol * fmax(un1, 1e-10) &&
                          fabs(d[2]) <= A.tol * fmax(un2, 1e-10);
        u[0] = fmin(fmax(un0, A.pd.T_floor), 1e9);
        u[1] = fmin(fmax(un1, 0.0), 0.5);
        u[2] = fmin(fmax(un2, 0.0), 1.0 - 2.0 * u[1]);
        ++it;
        k = 0;
        if (conv) {
          if (!hurwitz_shifted(J, srate)) break;
          if (fabs(log(u[0] / Tseed)) > 0.1) break;
          if (fabs(u[0] - T0) <= 1e-3 * T0) { ok = true; break; }
          dir = u[0] > T0 ? 1.0 : -1.0;
          phase = 1;
          continue;
        }
        if (it >= A.maxit) break;
        continue;
      }
      // phase 1: no thermal equilibrium between T_0 and the root
      if (!(gT * dir > 0.0)) break;
      if (k == 3) { ok = true; break; }
      ++k;
    }
    if (ok) {
      // 5. lag of the plain step's final jump: one substep of length dt from the root and
      // from the root perturbed in T, x_H2, x_H+
      StepArgs<float> sa{};
      sa.dt = dt;
      sa.pr = a.pr;
      sa.pd = a.pd;
      const double scale[3] = {u[0], fmax(u[1], 1e-7), fmax(u[2], 1e-7)};
      const double hv[3] = {1e-3 * u[0], 1e-3 * fmax(u[1], 1e-8), 1e-3 * fmax(u[2], 1e-8)};
      const double dev[3] = {fabs(T0 - u[0]), fabs(x20 - u[1]), fabs(xp0 - u[2])};
      double base[3] = {0.0, 0.0, 0.0}, err[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
      for (int v = -1; v < 3 && ok; ++v) {
        double y0 = u[0], y1 = u[1], y2 = u[2];
        if (v == 0) y0 += hv[0];
        if (v == 1) y1 = 2.0 * (y1 + hv[1]) + y2 <= 1.0 ? y1 + hv[1] : y1 - hv[1];
        if (v == 2) y2 = 2.0 * y1 + y2 + hv[2] <= 1.0 ? y2 + hv[2] : y2 - hv[2];
        CellState<float> cs;
        cs.nd = nd;
        cs.K = K;
        cs.r = &r;
        cs.e = eq_species<float>(y0, (float)nd, y1, y2, r, c, p, s_tab, CloseTol<float>::v, 50);
        cs.Tmu = y0 * (1.1 + (double)cs.e.xe - y1) / muH;
        cs.xH2 = y1;
        cs.xHp = y2;
        cs.t = 0.0;
        cs.ns = 0;
        cs.st = 0;
        cs.tdi = tdg;  // a flat line through the dust temperature found at the root
        cs.tds = 0.0;
        cell_substep(sa, cs, s_tab);
        const double o[3] = {muH * cs.Tmu / (1.1 + (double)cs.e.xe - cs.xH2), cs.xH2, cs.xHp};
        if (v < 0) {
          // the root must be a fixed point of a single full-length substep
          ok = cs.t >= dt && cs.st == 0;
#pragma unroll
          for (int w = 0; w < 3; ++w) {
            base[w] = o[w];
            ok = ok && fabs(o[w] - u[w]) <= 0.1 * a.out_tol * scale[w];
          }
        } else {
          const double step = v == 0 ? hv[0] : (v == 1 ? y1 - u[1] : y2 - u[2]);
#pragma unroll
          for (int w = 0; w < 3; ++w) err[w] += fabs((o[w] - base[w]) / step) * dev[v];
        }
      }
#pragma unroll
      for (int w = 0; w < 3; ++w) ok = ok && err[w] <= 0.5 * a.out_tol * scale[w];
    }
    if (ok) {
      const EqS<float> e = eq_species<float>(u[0], (float)nd, u[1], u[2], r, c, p, s_tab, CloseTol<float>::v, 50);
      a.T[i] = u[0];
      a.xH2[i] = u[1];
      a.xHp[i] = u[2];
      if (a.xCp) a.xCp[i] = e.xCp;
      if (a.xCO) a.xCO[i] = e.xCO;
      if (a.xe) a.xe[i] = e.xe;
      if (a.nsub) a.nsub[i] = 0;
      if (a.status) a.status[i] = 0;
    }
  }
  return ok;
}

// The candidates in a grid-stride loop over waves (the count is known on the device only);
// rejected candidates are appended to the fallback list.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void accept_kernel(AcceptArgs a) {
  __shared__ float s_tab[TAB_STEP];
  stage_tables(a.tab, s_tab);
  const int lane = threadIdx.x & 63;
  const int64_t nitem = (int64_t)*a.ncand;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); k0 < nitem; k0 += stride) {
    const int64_t k = k0 + lane;
    const bool live = k < nitem;
    const int64_t i = live ? (int64_t)a.cand[k] : 0;
    const bool ok = live && accept_cell(a, k, i, s_tab);
    wave_append(live && !ok, (int32_t)i, a.rej, a.nrej);
  }
}

__global__ void counter_reset_kernel(unsigned long long *c) { *c = 0ull; }

__global__ void counter_copy_kernel(const unsigned long long *c, int64_t *out) { *out = (int64_t)*c; }

}  // namespace ism
