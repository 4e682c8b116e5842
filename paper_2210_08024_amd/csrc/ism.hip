// libism: C ABI of the MI355X ISM photochemistry + heating/cooling source step.
// Host side: coefficient loading, argument validation, per-device state, launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <algorithm>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ism.h"
#include "coef.h"
#include "coef_load.h"
#include "kernels_step.h"
#include "kernels_columns.h"
#include "kernels_mlp.h"
#include "kernels_surr.h"
#include "kernels_order.h"
#include "kernels_sources.h"
#include "kernels_art.h"

using namespace ism;
using ism::host::coef_to_f32;
using ism::host::load_coefficients;

// Scratch of ism_chem_cool_step_noalloc: one copy per device, held for the life of the process.
// Layout: [0, 256) work-queue counter; [256, ...) the cell ordering (order_bytes(ncell)).  Host
// code never names it after init: it uses the per-device address taken there.
static __device__ __align__(256) uint8_t scratch[ISM_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

ism_status fail(ism_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

struct DevState {
  bool ready = false;
  double *tab64 = nullptr;
  float *tab32 = nullptr;
  int num_cu = 0;
  int occ64 = 0, occ32 = 0;  // resident 256-thread blocks per CU of the persistent step kernels
  int occ_col64 = 0, occ_col32 = 0;  // resident blocks per CU of the column tile kernels
  bool simple_step = false;   // ISM_STEP_KERNEL=simple selects the one-lane-per-cell grid
  uint8_t *noalloc = nullptr;  // this device's copy of `scratch` (hipGetSymbolAddress at init)
};

// Library scratch of one (device, stream): every call takes the scratch of the stream it is
// enqueued on, so calls on different streams never share memory.  Buffers grow with
// stream-ordered allocation (hipFreeAsync / hipMallocAsync on that stream): no device-wide
// synchronisation, and a buffer is released only after the work queued before it on the stream.
struct StreamScratch {
  void *col = nullptr;  // six-ray columns: tile sums and offsets
  size_t col_b = 0;
  void *ord = nullptr;  // cell ordering: keys, histogram, cursor, ordered list
  size_t ord_b = 0;
  void *surr = nullptr;  // surrogate step: predictions and the rejected list
  size_t surr_b = 0;
  void *ctl = nullptr;  // [0] work-queue counter (int64), [1] rejected-cell count (uint64)
  size_t ctl_b = 0;
  void *art[2] = {nullptr, nullptr};  // ray tracing: packet lists of two levels
  size_t art_b[2] = {0, 0};
  unsigned long long *art_count_host = nullptr;  // pinned: children appended by a level
};

std::mutex g_mu;
std::map<int, DevState> g_dev;
std::map<std::pair<int, hipStream_t>, StreamScratch> g_ss;

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(ISM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

ism_status current_state(DevState **out, int *dev_out = nullptr) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_dev.find(dev);
  if (it == g_dev.end() || !it->second.ready)
    return fail(ISM_E_STATE, "ism_init has not been called for device " + std::to_string(dev));
  *out = &it->second;
  if (dev_out) *dev_out = dev;
  return ISM_OK;
}

ism_status check_params(const ism_params *p) {
  if (!p) return fail(ISM_E_ARG, "params is NULL");
  if (p->order_cells < 0 || p->order_cells > 2) return fail(ISM_E_ARG, "order_cells must be 0, 1 or 2");
  if (!(p->Zg > 0.0) || !std::isfinite(p->Zg)) return fail(ISM_E_ARG, "Zg must be finite and > 0");
  if (!(p->Zd > 0.0) || !std::isfinite(p->Zd)) return fail(ISM_E_ARG, "Zd must be finite and > 0");
  if (!(p->chi0 >= 0.0) || !std::isfinite(p->chi0)) return fail(ISM_E_ARG, "chi0 must be finite and >= 0");
  if (!(p->xi_cr0 >= 0.0) || !std::isfinite(p->xi_cr0)) return fail(ISM_E_ARG, "xi_cr0 must be finite and >= 0");
  if (!(p->dvdr_kms_pc > 0.0)) return fail(ISM_E_ARG, "dvdr_kms_pc must be > 0");
  if (!(p->eps_sub > 0.0 && p->eps_sub <= 1.0)) return fail(ISM_E_ARG, "eps_sub must be in (0, 1]");
  if (!(p->fd_rel > 0.0 && p->fd_rel < 0.5)) return fail(ISM_E_ARG, "fd_rel must be in (0, 0.5)");
  if (!(p->T_floor > 0.0)) return fail(ISM_E_ARG, "T_floor must be > 0");
  if (!(p->T_bb > 0.0 && p->T_bb < 1e4)) return fail(ISM_E_ARG, "T_bb must be in (0, 1e4)");
  if (!(p->tau_opt_ratio > 0.0)) return fail(ISM_E_ARG, "tau_opt_ratio must be > 0");
  if (p->cr_mode < 0 || p->cr_mode > 2) return fail(ISM_E_ARG, "cr_mode must be 0, 1 or 2");
  if (p->max_substeps < 1) return fail(ISM_E_ARG, "max_substeps must be >= 1");
  return ISM_OK;
}

template <class R>
ParT<R> make_par(const ism_params *p, const CoefT<double> &c) {
  ParT<R> q;
  q.Zg = (R)p->Zg; q.Zd = (R)p->Zd; q.chi0 = (R)p->chi0; q.dvdr = (R)p->dvdr_kms_pc;
  q.eps_sub = (R)p->eps_sub; q.fd_rel = (R)p->fd_rel; q.T_floor = (R)p->T_floor; q.T_bb = (R)p->T_bb;
  q.tau_ratio = (R)p->tau_opt_ratio;
  q.xCt = (R)(c.xCt_per_Zg * p->Zg);
  q.xOt = (R)(c.xOt_per_Zg * p->Zg);
  q.muH = (R)(c.muH0 - c.muH_slope * (p->Zg - 1.0));
  q.lnZd = (R)std::log(p->Zd);
  q.idvdr = (R)(1.0 / p->dvdr_kms_pc);
  const double fd1 = 1.0 + p->fd_rel;
  q.fd_ln = (R)std::log(fd1);
  q.fd_inv = (R)(1.0 / fd1);
  q.fd_sqrt = (R)std::sqrt(fd1);
  q.kgr_const = p->kgr_const; q.h2_rovib = p->h2_rovib; q.max_sub = p->max_substeps; q.cr_mode = p->cr_mode;
  return q;
}

CoefT<double> g_host_coef;  // last loaded coefficients (host copy for make_par)

// The scratch record of (current device, stream); std::map keeps the address stable.
StreamScratch *stream_scratch(int dev, hipStream_t stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  return &g_ss[std::make_pair(dev, stream)];
}

// Make *p hold at least `bytes` (stream-ordered; contents are not kept across growth).
ism_status grow(void **p, size_t *cap, size_t bytes, hipStream_t stream, const char *what) {
  if (*cap >= bytes && *p) return ISM_OK;
  if (*p) {
    hipError_t e = hipFreeAsync(*p, stream);
    if (e != hipSuccess) return fail(ISM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
  *p = nullptr;
  *cap = 0;
  const size_t want = std::max<size_t>(bytes, 256);
  hipError_t e = hipMallocAsync(p, want, stream);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(ISM_E_NOMEM, std::string(what) + " (" + std::to_string(want) + " bytes): " + hipGetErrorString(e));
  }
  *cap = want;
  return ISM_OK;
}

// Scratch bytes of the cell ordering for n items.
size_t order_bytes(int64_t n) {
  const size_t key_b = (size_t)((n * 2 + 255) / 256 * 256), bins_b = (size_t)ORDER_BINS * 4;
  const size_t out_b = (size_t)((n * 4 + 255) / 256 * 256);
  return key_b + 2 * bins_b + out_b;
}

// Order `n` items (cells, or the cells listed in `items`, `*count` of them when count is set)
// by temperature regime (or previous substep counts); *out receives the ordered cell list, laid
// out in `base` (order_bytes(n) bytes of scratch).
void order_cells(uint8_t *base, int64_t n, const unsigned long long *count, const int32_t *items, const double *T,
                 const int32_t *nsub, int32_t **out, hipStream_t stream) {
  const size_t key_b = (size_t)((n * 2 + 255) / 256 * 256), bins_b = (size_t)ORDER_BINS * 4;
  OrderArgs a{n, count, items, T, nsub, (uint16_t *)base, (uint32_t *)(base + key_b),
              (uint32_t *)(base + key_b + bins_b), (int32_t *)(base + key_b + 2 * bins_b), 0};
  // the slab of a cell: the top ORDER_BITS - ORDER_T_BITS bits of its index below n (the cells
  // of a list are grid indices below n as well)
  int bits = 0;
  while (bits < 62 && ((int64_t)1 << bits) < n) ++bits;
  a.cshift = bits > ORDER_BITS - ORDER_T_BITS ? bits - (ORDER_BITS - ORDER_T_BITS) : 0;
  const dim3 grid((unsigned)((n + ORDER_CHUNK - 1) / ORDER_CHUNK));
  hipLaunchKernelGGL(order_zero_kernel, dim3(1), dim3(ORDER_THREADS), 0, stream, a.hist);
  hipLaunchKernelGGL(order_key_kernel, grid, dim3(ORDER_THREADS), 0, stream, a);
  hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(ORDER_THREADS), 0, stream, a);
  hipLaunchKernelGGL(order_scatter_kernel, grid, dim3(ORDER_THREADS), 0, stream, a);
  *out = a.out;
}

// Scratch bytes of the tiled six-ray pass: sums, forward and backward offsets, 3 quantities each.
size_t columns_bytes(const ism_grid *g) {
  const TileGeo tg = tile_geo(g->nx, g->ny, g->nz);
  return 9 * (size_t)tg.per_q * sizeof(double);
}

// Launch the tiled six-ray pass (the three kernels of kernels_columns.h) with `buf` holding
// columns_bytes(grid) bytes.
ism_status launch_columns6(const DevState *st, const ism_grid *g, const ism_params *p, bool f32, const double *n,
                           const double *xH2, const double *xC, void *chi_PE, void *chi_LW, void *chi_H2,
                           void *chi_C, void *N_eff, void *xi_cr, void *buf, hipStream_t stream) {
  TileArgs t{};
  ColArgs &a = t.c;
  a.nx = g->nx; a.ny = g->ny; a.nz = g->nz; a.dx = g->dx_cm;
  a.n = n; a.xH2 = xH2; a.xC = xC;
  a.chiPE = chi_PE; a.chiLW = chi_LW; a.chiH2 = chi_H2; a.chiC = chi_C; a.Neff = N_eff; a.xi = xi_cr;
  a.cr_mode = p->cr_mode;
  a.chi0 = p->chi0; a.Zd = p->Zd; a.xi0 = p->xi_cr0;
  a.sPE = g_host_coef.sig_d_abs[2] * p->Zd;
  a.sLW = g_host_coef.sig_d_abs[1] * p->Zd;
  a.tab = st->tab64;
  t.g = tile_geo(g->nx, g->ny, g->nz);
  t.S = (double *)buf;
  t.F = t.S + 3 * t.g.per_q;
  t.B = t.F + 3 * t.g.per_q;
  const int64_t pairs = (int64_t)((t.g.ntx + 1) / 2) * t.g.nty * t.g.ntz;
  const int cu = std::max(st->num_cu, 1);
  // the sums kernel: one wave per block, no LDS; the tile kernel's grid is what stays resident
  // (its LDS and registers set the count), each block taking an equal share of the tile pairs
  const int occ = std::max(f32 ? st->occ_col32 : st->occ_col64, 1);
  const unsigned g1 = (unsigned)std::min<int64_t>(pairs, (int64_t)cu * 16);
  const unsigned g3 = (unsigned)std::min<int64_t>(pairs, (int64_t)cu * occ);
  hipLaunchKernelGGL(columns_tilesum_kernel, dim3(g1), dim3(CT_LANES), 0, stream, t);
  const int64_t lines = 2 * (t.g.lx + t.g.ly + t.g.lz);
  hipLaunchKernelGGL(columns_offsets_kernel, dim3((unsigned)((lines + 255) / 256)), dim3(256), 0, stream, t);
  if (f32) hipLaunchKernelGGL(columns_tile_kernel<float>, dim3(g3), dim3(CT_THREADS), 0, stream, t);
  else hipLaunchKernelGGL(columns_tile_kernel<double>, dim3(g3), dim3(CT_THREADS), 0, stream, t);
  HIP_TRY(hipGetLastError());
  return ISM_OK;
}

ism_status check_step(const ism_params *p, ism_precision prec, int64_t ncell, double dt_s, const double *n,
                      const double *T, const double *xH2, const double *xHp, const void *chi_PE, const void *chi_LW,
                      const void *chi_H2, const void *chi_C, const void *xi_cr, const void *N_eff) {
  if (ism_status s = check_params(p)) return s;
  if (prec != ISM_PREC_F64 && prec != ISM_PREC_MIXED) return fail(ISM_E_ARG, "invalid precision");
  if (ncell < 0) return fail(ISM_E_ARG, "ncell must be >= 0");
  if (!(dt_s >= 0.0) || !std::isfinite(dt_s)) return fail(ISM_E_ARG, "dt_s must be finite and >= 0");
  if (ncell == 0) return ISM_OK;
  if (!n || !T || !xH2 || !xHp || !chi_PE || !chi_LW || !chi_H2 || !chi_C || !xi_cr || !N_eff)
    return fail(ISM_E_ARG, "a required array is NULL");
  return ISM_OK;
}

// Whether the step orders its cells (order_cells 1 or 2, the persistent kernel, int32 indices).
bool step_orders(const DevState *st, const ism_params *p, int64_t ncell) {
  return p->order_cells && !st->simple_step && ncell <= (int64_t)INT32_MAX;
}

// Enqueue the source step on `stream`: the cell ordering into `ord` (order_bytes(ncell) bytes;
// null when step_orders is false), the work-queue counter `q` (set by a kernel, so the sequence
// holds no memset), then the persistent kernel.
void launch_step(const DevState *st, const ism_params *p, ism_precision prec, int64_t ncell, double dt_s,
                 const double *n, double *T, double *xH2, double *xHp, const void *chi_PE, const void *chi_LW,
                 const void *chi_H2, const void *chi_C, const void *phi_LyC, const void *xi_cr, const void *N_eff,
                 void *xCp, void *xCO, void *xe, int32_t *nsub, uint8_t *status, int64_t *q, uint8_t *ord,
                 hipStream_t stream) {
  const int64_t want = (ncell + 255) / 256;
  int32_t *order = nullptr;
  if (ord) order_cells(ord, ncell, nullptr, nullptr, T, p->order_cells == 2 ? nsub : nullptr, &order, stream);
  if (prec == ISM_PREC_F64) {
    StepArgs<double> a{ncell, dt_s, n, T, xH2, xHp, (const double *)chi_PE, (const double *)chi_LW,
                       (const double *)chi_H2, (const double *)chi_C, (const double *)phi_LyC,
                       (const double *)xi_cr, (const double *)N_eff, (double *)xCp, (double *)xCO, (double *)xe,
                       nsub, status, st->tab64, make_par<double>(p, g_host_coef), make_par<double>(p, g_host_coef), q,
                       order, nullptr, 0u};
    if (st->simple_step) {
      hipLaunchKernelGGL(step_simple_kernel<double>, dim3((unsigned)want), dim3(256), 0, stream, a);
    } else {
      const int64_t grid = std::min<int64_t>(want, (int64_t)st->num_cu * std::max(st->occ64, 1));
      hipLaunchKernelGGL(queue_init_kernel, dim3(1), dim3(1), 0, stream, q, grid * 256);
      hipLaunchKernelGGL(step_queue_kernel<double>, dim3((unsigned)grid), dim3(256), 0, stream, a);
    }
  } else {
    StepArgs<float> a{ncell, dt_s, n, T, xH2, xHp, (const float *)chi_PE, (const float *)chi_LW,
                      (const float *)chi_H2, (const float *)chi_C, (const float *)phi_LyC,
                      (const float *)xi_cr, (const float *)N_eff, (float *)xCp, (float *)xCO, (float *)xe,
                      nsub, status, st->tab32, make_par<float>(p, g_host_coef), make_par<double>(p, g_host_coef), q,
                      order, nullptr, 0u};
    if (st->simple_step) {
      hipLaunchKernelGGL(step_simple_kernel<float>, dim3((unsigned)want), dim3(256), 0, stream, a);
    } else {
      const int64_t grid = std::min<int64_t>(want, (int64_t)st->num_cu * std::max(st->occ32, 1));
      hipLaunchKernelGGL(queue_init_kernel, dim3(1), dim3(1), 0, stream, q, grid * 256);
      hipLaunchKernelGGL(step_queue_kernel<float>, dim3((unsigned)grid), dim3(256), 0, stream, a);
    }
  }
}

const char *kDiagNames[NDIAG] = {
    "xCp", "xCO", "xe", "Td", "kgr", "zcrH2", "zpd", "zpiH2", "zcd", "zpiH", "zcrH", "zci", "aB",
    "agrH", "psi", "G_pe", "G_cr", "G_pi", "G_h2", "Gamma", "L_lya", "L_ci", "L_rovib", "L_cd", "L_ff", "L_rr",
    "L_cp", "L_c", "L_o", "L_co", "L_grrec", "L_neb", "L_gd", "L_cie", "S", "Lambda", "H", "C_H2", "C_Hp"};

}  // namespace

// ====================================================================== C ABI
extern "C" {

void ism_params_default(ism_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->Zg = 1.0; p->Zd = 1.0; p->chi0 = 1.0; p->xi_cr0 = 2.0e-16; p->dvdr_kms_pc = 1.0; p->eps_sub = 0.1;
  p->fd_rel = 1.0e-3; p->T_floor = 1.0; p->T_bb = 6.0; p->tau_opt_ratio = 1.87;
  p->cr_mode = 0; p->kgr_const = 0; p->h2_rovib = 1; p->max_substeps = 100000; p->order_cells = 1;
}

const char *ism_last_error(void) { return g_err.c_str(); }

int32_t ism_ndiag(void) { return NDIAG; }

const char *ism_diag_name(int32_t k) { return (k >= 0 && k < NDIAG) ? kDiagNames[k] : nullptr; }

ism_status ism_init(int device, const char *path) {
  g_err.clear();
  CoefT<double> c64;
  std::vector<double> tab;
  std::string err;
  if (!path) return fail(ISM_E_ARG, "coefficient path is NULL");
  if (!load_coefficients(path, c64, tab, err)) return fail(ISM_E_TABLE, err);
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(ISM_E_ARG, "device index out of range");
  int prev = 0;
  HIP_TRY(hipGetDevice(&prev));
  HIP_TRY(hipSetDevice(device));
  CoefT<float> c32;
  coef_to_f32(c64, c32);
  std::vector<float> tab32(tab.begin(), tab.end());
  ism_status rc = ISM_OK;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    DevState &st = g_dev[device];
    hipError_t e = hipSuccess;
    if (!st.tab64) e = hipMalloc(&st.tab64, TAB_TOTAL * sizeof(double));
    if (e == hipSuccess && !st.tab32) e = hipMalloc(&st.tab32, TAB_TOTAL * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(st.tab64, tab.data(), TAB_TOTAL * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(st.tab32, tab32.data(), TAB_TOTAL * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(g_coef64), &c64, sizeof(c64));
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(g_coef32), &c32, sizeof(c32));
    if (e == hipSuccess) e = hipDeviceGetAttribute(&st.num_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&st.occ64, step_queue_kernel<double>, 256, 0);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&st.occ32, step_queue_kernel<float>, 256, 0);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&st.occ_col64, columns_tile_kernel<double>, CT_THREADS, 0);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&st.occ_col32, columns_tile_kernel<float>, CT_THREADS, 0);
    // the allocation-free step's scratch: its address on this device (the device is current)
    if (e == hipSuccess && !st.noalloc) e = hipGetSymbolAddress((void **)&st.noalloc, HIP_SYMBOL(scratch));
    if (e == hipSuccess) {
      const char *k = std::getenv("ISM_STEP_KERNEL");
      st.simple_step = k && std::string(k) == "simple";
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) rc = fail(ISM_E_DEVICE, std::string("ism_init: ") + hipGetErrorString(e));
    else { st.ready = true; g_host_coef = c64; }
  }
  (void)hipSetDevice(prev);
  return rc;
}

ism_status ism_shutdown(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int prev = 0;
  (void)hipGetDevice(&prev);
  for (auto &kv : g_dev) {
    if (hipSetDevice(kv.first) != hipSuccess) continue;
    (void)hipDeviceSynchronize();
    if (kv.second.tab64) (void)hipFree(kv.second.tab64);
    if (kv.second.tab32) (void)hipFree(kv.second.tab32);
    for (auto &ss : g_ss) {
      if (ss.first.first != kv.first) continue;
      StreamScratch &x = ss.second;
      for (void *q : {x.col, x.ord, x.surr, x.ctl, x.art[0], x.art[1]})
        if (q) (void)hipFree(q);
      if (x.art_count_host) (void)hipHostFree(x.art_count_host);
    }
  }
  g_ss.clear();
  g_dev.clear();
  (void)hipSetDevice(prev);
  return ISM_OK;
}

ism_status ism_stream_release(hipStream_t stream) {
  g_err.clear();
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  StreamScratch x;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ss.find(std::make_pair(dev, stream));
    if (it == g_ss.end()) return ISM_OK;
    x = it->second;
    g_ss.erase(it);
  }
  for (void *q : {x.col, x.ord, x.surr, x.ctl, x.art[0], x.art[1]})
    if (q) HIP_TRY(hipFreeAsync(q, stream));
  if (x.art_count_host) {
    // the pinned count is read back only inside ism_ray_trace, after a stream synchronisation
    HIP_TRY(hipHostFree(x.art_count_host));
  }
  return ISM_OK;
}

ism_status ism_columns6(const ism_grid *g, const ism_params *p, ism_precision prec, const double *n,
                        const double *xH2, const double *xC, void *chi_PE, void *chi_LW, void *chi_H2, void *chi_C,
                        void *N_eff, void *xi_cr, hipStream_t stream) {
  g_err.clear();
  if (!g) return fail(ISM_E_ARG, "grid is NULL");
  if (ism_status s = check_params(p)) return s;
  if (prec != ISM_PREC_F64 && prec != ISM_PREC_MIXED) return fail(ISM_E_ARG, "invalid precision");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(ISM_E_ARG, "grid dimensions must be >= 1");
  if (!(g->dx_cm > 0.0) || !std::isfinite(g->dx_cm)) return fail(ISM_E_ARG, "dx_cm must be finite and > 0");
  if (g->nx > (1 << 24) || g->ny > (1 << 24) || g->nz > (1 << 24) ||
      (int64_t)g->nx * g->ny * g->nz > ((int64_t)1 << 40))
    return fail(ISM_E_ARG, "grid too large (each dimension at most 2^24 cells, at most 2^40 cells)");
  if (!n || !xH2 || !chi_PE || !chi_LW || !chi_H2 || !chi_C || !N_eff)
    return fail(ISM_E_ARG, "n, xH2 and all chi/N_eff outputs must be non-NULL");
  if (p->cr_mode != 2 && !xi_cr) return fail(ISM_E_ARG, "xi_cr output is NULL (cr_mode 0/1 writes it)");
  DevState *st;
  int dev = 0;
  if (ism_status s = current_state(&st, &dev)) return s;
  StreamScratch *ss = stream_scratch(dev, stream);
  if (ism_status s = grow(&ss->col, &ss->col_b, columns_bytes(g), stream, "columns scratch")) return s;
  return launch_columns6(st, g, p, prec == ISM_PREC_MIXED, n, xH2, xC, chi_PE, chi_LW, chi_H2, chi_C, N_eff, xi_cr,
                         ss->col, stream);
}

ism_status ism_rates(const ism_params *p, ism_precision prec, int64_t ncell, const double *n, const double *T,
                     const double *xH2, const double *xHp, const void *chi_PE, const void *chi_LW,
                     const void *chi_H2, const void *chi_C, const void *phi_LyC, const void *xi_cr,
                     const void *N_eff, void *out, hipStream_t stream) {
  g_err.clear();
  if (ism_status s = check_params(p)) return s;
  if (prec != ISM_PREC_F64 && prec != ISM_PREC_MIXED) return fail(ISM_E_ARG, "invalid precision");
  if (ncell < 0) return fail(ISM_E_ARG, "ncell must be >= 0");
  if (ncell == 0) return ISM_OK;
  if (!n || !T || !xH2 || !xHp || !chi_PE || !chi_LW || !chi_H2 || !chi_C || !xi_cr || !N_eff || !out)
    return fail(ISM_E_ARG, "a required array is NULL");
  DevState *st;
  if (ism_status s = current_state(&st)) return s;
  const unsigned blocks = (unsigned)((ncell + 127) / 128);
  if (prec == ISM_PREC_F64) {
    RatesArgs<double> a{ncell, n, T, xH2, xHp, (const double *)chi_PE, (const double *)chi_LW,
                        (const double *)chi_H2, (const double *)chi_C, (const double *)phi_LyC,
                        (const double *)xi_cr, (const double *)N_eff, (double *)out, st->tab64,
                        make_par<double>(p, g_host_coef)};
    hipLaunchKernelGGL(rates_kernel<double>, dim3(blocks), dim3(128), 0, stream, a);
  } else {
    RatesArgs<float> a{ncell, n, T, xH2, xHp, (const float *)chi_PE, (const float *)chi_LW,
                       (const float *)chi_H2, (const float *)chi_C, (const float *)phi_LyC,
                       (const float *)xi_cr, (const float *)N_eff, (float *)out, st->tab32,
                       make_par<float>(p, g_host_coef)};
    hipLaunchKernelGGL(rates_kernel<float>, dim3(blocks), dim3(128), 0, stream, a);
  }
  HIP_TRY(hipGetLastError());
  return ISM_OK;
}

ism_status ism_chem_cool_step(const ism_params *p, ism_precision prec, int64_t ncell, double dt_s, const double *n,
                              double *T, double *xH2, double *xHp, const void *chi_PE, const void *chi_LW,
                              const void *chi_H2, const void *chi_C, const void *phi_LyC, const void *xi_cr,
                              const void *N_eff, void *xCp, void *xCO, void *xe, int32_t *nsub, uint8_t *status,
                              hipStream_t stream) {
  g_err.clear();
  if (ism_status s = check_step(p, prec, ncell, dt_s, n, T, xH2, xHp, chi_PE, chi_LW, chi_H2, chi_C, xi_cr, N_eff))
    return s;
  if (ncell == 0) return ISM_OK;
  DevState *st;
  int dev = 0;
  if (ism_status s = current_state(&st, &dev)) return s;
  StreamScratch *ss = stream_scratch(dev, stream);
  if (ism_status s = grow(&ss->ctl, &ss->ctl_b, 256, stream, "work-queue counter")) return s;
  uint8_t *ord = nullptr;
  if (step_orders(st, p, ncell)) {
    if (ism_status s = grow(&ss->ord, &ss->ord_b, order_bytes(ncell), stream, "order scratch")) return s;
    ord = (uint8_t *)ss->ord;
  }
  launch_step(st, p, prec, ncell, dt_s, n, T, xH2, xHp, chi_PE, chi_LW, chi_H2, chi_C, phi_LyC, xi_cr, N_eff, xCp,
              xCO, xe, nsub, status, (int64_t *)ss->ctl, ord, stream);
  HIP_TRY(hipGetLastError());
  return ISM_OK;
}

ism_status ism_chem_cool_step_noalloc(const ism_params *p, ism_precision prec, int64_t ncell, double dt_s,
                                      const double *n, double *T, double *xH2, double *xHp, const void *chi_PE,
                                      const void *chi_LW, const void *chi_H2, const void *chi_C,
                                      const void *phi_LyC, const void *xi_cr, const void *N_eff, void *xCp,
                                      void *xCO, void *xe, int32_t *nsub, uint8_t *status, hipStream_t stream) {
  g_err.clear();
  if (ism_status s = check_step(p, prec, ncell, dt_s, n, T, xH2, xHp, chi_PE, chi_LW, chi_H2, chi_C, xi_cr, N_eff))
    return s;
  if (ncell == 0) return ISM_OK;
  DevState *st;
  if (ism_status s = current_state(&st)) return s;
  if (!st->noalloc) return fail(ISM_E_STATE, "no allocation-free scratch on this device");
  const bool ordered = step_orders(st, p, ncell);
  if (ordered && (ncell > (int64_t)ISM_NOALLOC_MAX_ORDERED_CELLS ||
                  256 + order_bytes(ncell) > (size_t)ISM_NOALLOC_SCRATCH_BYTES))
    return fail(ISM_E_ARG, "ism_chem_cool_step_noalloc: with order_cells 1 or 2 ncell must be at most " +
                               std::to_string((long long)ISM_NOALLOC_MAX_ORDERED_CELLS));
  launch_step(st, p, prec, ncell, dt_s, n, T, xH2, xHp, chi_PE, chi_LW, chi_H2, chi_C, phi_LyC, xi_cr, N_eff, xCp,
              xCO, xe, nsub, status, (int64_t *)st->noalloc, ordered ? st->noalloc + 256 : nullptr, stream);
  HIP_TRY(hipGetLastError());
  return ISM_OK;
}

// ====================================================================== surrogate
}  // extern "C"

struct ism_surrogate {
  int device = 0;
  int num_cu = 1;
  float *params = nullptr;  // theta | adam m | adam v | grad scratch, NPARAM floats each
  uint8_t *img = nullptr;   // forward image | backward image
  float norm_host[26];      // mu_x sd_x mu_y sd_y (passed by value with every launch)
  int64_t step = 0;
  void *work = nullptr;     // training workspace, grown stream-ordered
  size_t work_bytes = 0;
  float *staging = nullptr;  // pinned: params on their way to or from the device
  hipEvent_t staged = nullptr;  // recorded after the last upload out of `staging`
  float *theta() const { return params; }
  float *adam_m() const { return params + mlp::NPARAM; }
  float *adam_v() const { return params + 2 * mlp::NPARAM; }
  uint8_t *fimg() const { return img; }
  uint8_t *bimg() const { return img + mlp::FI_BYTES; }
};

namespace {

uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

ism_status surr_check(const ism_surrogate *m) {
  if (!m) return fail(ISM_E_ARG, "surrogate is NULL");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != m->device) return fail(ISM_E_ARG, "surrogate belongs to another device");
  return ISM_OK;
}

// The standardisation as a launch argument.
mlp::Norm surr_norm(const ism_surrogate *m) {
  mlp::Norm d{};
  for (int k = 0; k < mlp::NIN; ++k) {
    d.v[mlp::NRM_MUX + k] = m->norm_host[k];
    d.v[mlp::NRM_ISDX + k] = (float)(1.0 / (double)m->norm_host[10 + k]);
  }
  for (int k = 0; k < mlp::NOUT; ++k) {
    d.v[mlp::NRM_MUY + k] = m->norm_host[20 + k];
    d.v[mlp::NRM_SDY + k] = m->norm_host[23 + k];
    d.v[mlp::NRM_ISDY + k] = (float)(1.0 / (double)m->norm_host[23 + k]);
  }
  return d;
}

// BF16 weight images from the FP32 parameters, enqueued on `stream` (the images' padding is
// zeroed once at creation and never written by the pack kernel).
ism_status surr_pack(ism_surrogate *m, hipStream_t stream) {
  hipLaunchKernelGGL(mlp::mlp_pack_kernel, dim3((mlp::NPARAM + 255) / 256), dim3(256), 0, stream, m->theta(),
                     m->fimg(), m->bimg());
  HIP_TRY(hipGetLastError());
  return ISM_OK;
}

// Per-batch buffers of a training or backward pass.
struct SurrWork {
  uint16_t *h0, *h1, *h2, *h3;
  float *z1, *z2, *z3, *d4, *part, *loss_part;
  int64_t chunk;
  int nchunk, grid_fwd;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int fwd_grid(const ism_surrogate *m, int64_t B) {
  // tiles go to the waves of all blocks in turn (wave-major), so a batch of at least one tile
  // per CU spreads over every CU
  return (int)std::max<int64_t>(1, std::min<int64_t>((B + mlp::WTILE - 1) / mlp::WTILE, m->num_cu));
}

ism_status surr_work(ism_surrogate *m, int64_t B, SurrWork &w, hipStream_t stream) {
  w.chunk = std::max<int64_t>(64, ((B + 127) / 128 + 63) / 64 * 64);
  w.nchunk = (int)((B + w.chunk - 1) / w.chunk);
  w.grid_fwd = fwd_grid(m, B);
  const size_t sz[10] = {align256((size_t)B * mlp::K1 * 2), align256((size_t)B * mlp::NH * 2),
                         align256((size_t)B * mlp::NH * 2), align256((size_t)B * mlp::NH * 2),
                         align256((size_t)B * mlp::NH * 4), align256((size_t)B * mlp::NH * 4),
                         align256((size_t)B * mlp::NH * 4), align256((size_t)B * mlp::NOUT * 4),
                         align256((size_t)w.nchunk * mlp::NPARAM * 4),
                         align256((size_t)w.grid_fwd * mlp::FWD_WAVES * 4)};
  size_t total = 0;
  for (size_t x : sz) total += x;
  if (ism_status s = grow(&m->work, &m->work_bytes, total, stream, "surrogate workspace")) return s;
  uint8_t *p = (uint8_t *)m->work;
  void *ptr[10];
  for (int i = 0; i < 10; ++i) {
    ptr[i] = p;
    p += sz[i];
  }
  w.h0 = (uint16_t *)ptr[0]; w.h1 = (uint16_t *)ptr[1]; w.h2 = (uint16_t *)ptr[2]; w.h3 = (uint16_t *)ptr[3];
  w.z1 = (float *)ptr[4]; w.z2 = (float *)ptr[5]; w.z3 = (float *)ptr[6]; w.d4 = (float *)ptr[7];
  w.part = (float *)ptr[8]; w.loss_part = (float *)ptr[9];
  return ISM_OK;
}

// Forward with stored activations, backward through the layers, per-chunk weight gradients.
void surr_fwd_bwd(ism_surrogate *m, const float *X, const float *Yt, const float *dY, int64_t B, SurrWork &w,
                  hipStream_t stream) {
  mlp::FwdArgs fa{};
  fa.X = X; fa.B = B; fa.fimg = m->fimg(); fa.norm = surr_norm(m);
  fa.h0 = w.h0; fa.h1 = w.h1; fa.h2 = w.h2; fa.h3 = w.h3; fa.z1 = w.z1; fa.z2 = w.z2; fa.z3 = w.z3;
  const float *d4 = dY;
  if (Yt) {
    fa.Yt = Yt; fa.dscale = (float)(2.0 / (3.0 * (double)B)); fa.d4 = w.d4; fa.loss_part = w.loss_part;
    d4 = w.d4;
    hipLaunchKernelGGL(mlp::mlp_fwd_kernel<2>, dim3(w.grid_fwd), dim3(mlp::FWD_THREADS), 0, stream, fa);
  } else {
    hipLaunchKernelGGL(mlp::mlp_fwd_kernel<1>, dim3(w.grid_fwd), dim3(mlp::FWD_THREADS), 0, stream, fa);
  }
  mlp::BwdArgs ba{B, m->bimg(), d4, w.z1, w.z2, w.z3};
  hipLaunchKernelGGL(mlp::mlp_bwd_kernel, dim3(w.grid_fwd), dim3(mlp::FWD_THREADS), 0, stream, ba);
  mlp::DwArgs da{B, w.chunk, w.h0, w.h1, w.h2, w.h3, w.z1, w.z2, w.z3, d4, w.part};
  hipLaunchKernelGGL(mlp::mlp_dw_kernel, dim3(w.nchunk, 4), dim3(mlp::DW_THREADS), 0, stream, da);
}

}  // namespace

extern "C" {

ism_status ism_surrogate_create(ism_surrogate **out, uint64_t seed) {
  g_err.clear();
  if (!out) return fail(ISM_E_ARG, "out is NULL");
  *out = nullptr;
  DevState *st;
  int dev = 0;
  if (ism_status s = current_state(&st, &dev)) return s;
  ism_surrogate *m = new ism_surrogate();
  m->device = dev;
  m->num_cu = std::max(st->num_cu, 1);
  for (int k = 0; k < 26; ++k) m->norm_host[k] = (k >= 10 && k < 20) || k >= 23 ? 1.f : 0.f;
  std::vector<float> theta(mlp::NPARAM, 0.f);
  const int fan_in[4] = {mlp::NIN, mlp::NH, mlp::NH, mlp::NH};
  const int woff[4] = {mlp::OFF_W1, mlp::OFF_W2, mlp::OFF_W3, mlp::OFF_W4};
  const int wlen[4] = {mlp::NH * mlp::NIN, mlp::NH * mlp::NH, mlp::NH * mlp::NH, mlp::NOUT * mlp::NH};
  for (int l = 0; l < 4; ++l) {
    const double lim = std::sqrt(6.0 / fan_in[l]);
    for (int i = 0; i < wlen[l]; ++i) {
      const uint64_t u = splitmix64(seed * 0x100000001B3ull + (uint64_t)(woff[l] + i));
      const double x = (double)(u >> 11) * (1.0 / 9007199254740992.0);
      theta[woff[l] + i] = (float)(lim * (2.0 * x - 1.0));
    }
  }
  hipError_t e = hipMalloc(&m->params, 4 * (size_t)mlp::NPARAM * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->img, mlp::FI_BYTES + mlp::BI_BYTES);
  if (e == hipSuccess) e = hipHostMalloc(&m->staging, 3 * (size_t)mlp::NPARAM * sizeof(float));
  if (e == hipSuccess) e = hipEventCreateWithFlags(&m->staged, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMemset(m->params, 0, 4 * (size_t)mlp::NPARAM * sizeof(float));
  if (e == hipSuccess) e = hipMemset(m->img, 0, mlp::FI_BYTES + mlp::BI_BYTES);
  if (e == hipSuccess) e = hipMemcpy(m->params, theta.data(), mlp::NPARAM * sizeof(float), hipMemcpyHostToDevice);
  ism_status rc = e == hipSuccess ? ISM_OK : fail(ISM_E_NOMEM, std::string("surrogate: ") + hipGetErrorString(e));
  if (rc == ISM_OK) rc = surr_pack(m, nullptr);
  if (rc == ISM_OK && hipDeviceSynchronize() != hipSuccess) rc = fail(ISM_E_DEVICE, "surrogate: pack failed");
  if (rc != ISM_OK) {
    ism_surrogate_destroy(m);
    return rc;
  }
  *out = m;
  return ISM_OK;
}

ism_status ism_surrogate_destroy(ism_surrogate *m) {
  if (!m) return ISM_OK;
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  if (m->params) (void)hipFree(m->params);
  if (m->img) (void)hipFree(m->img);
  if (m->work) (void)hipFree(m->work);
  if (m->staging) (void)hipHostFree(m->staging);
  if (m->staged) (void)hipEventDestroy(m->staged);
  (void)hipSetDevice(prev);
  delete m;
  return ISM_OK;
}

ism_status ism_surrogate_set_norm(ism_surrogate *m, const float *mu_x, const float *sd_x, const float *mu_y,
                                  const float *sd_y) {
  g_err.clear();
  if (ism_status s = surr_check(m)) return s;
  if (!mu_x || !sd_x || !mu_y || !sd_y) return fail(ISM_E_ARG, "a normalisation array is NULL");
  for (int k = 0; k < mlp::NIN; ++k)
    if (!std::isfinite(mu_x[k]) || !(sd_x[k] > 0.f) || !std::isfinite(sd_x[k]))
      return fail(ISM_E_ARG, "mu_x must be finite and sd_x finite and > 0");
  for (int k = 0; k < mlp::NOUT; ++k)
    if (!std::isfinite(mu_y[k]) || !(sd_y[k] > 0.f) || !std::isfinite(sd_y[k]))
      return fail(ISM_E_ARG, "mu_y must be finite and sd_y finite and > 0");
  std::memcpy(m->norm_host, mu_x, 10 * sizeof(float));
  std::memcpy(m->norm_host + 10, sd_x, 10 * sizeof(float));
  std::memcpy(m->norm_host + 20, mu_y, 3 * sizeof(float));
  std::memcpy(m->norm_host + 23, sd_y, 3 * sizeof(float));
  return ISM_OK;
}

ism_status ism_surrogate_forward(ism_surrogate *m, const float *X, float *Y, int64_t B, hipStream_t stream) {
  g_err.clear();
  if (ism_status s = surr_check(m)) return s;
  if (B < 0) return fail(ISM_E_ARG, "B must be >= 0");
  if (B == 0) return ISM_OK;
  if (!X || !Y) return fail(ISM_E_ARG, "X and Y must not be NULL");
  mlp::FwdArgs fa{};
  fa.X = X; fa.B = B; fa.fimg = m->fimg(); fa.norm = surr_norm(m); fa.Y = Y;
  hipLaunchKernelGGL(mlp::mlp_fwd_kernel<0>, dim3(fwd_grid(m, B)), dim3(mlp::FWD_THREADS), 0, stream, fa);
  HIP_TRY(hipGetLastError());
  return ISM_OK;
}

ism_status ism_surrogate_backward(ism_surrogate *m, const float *X, const float *dY, float *grad, int64_t B,
                                  hipStream_t stream) {
  g_err.clear();
  if (ism_status s = surr_check(m)) return s;
  if (B < 1) return fail(ISM_E_ARG, "B must be >= 1");
  if (!X || !dY || !grad) return fail(ISM_E_ARG, "X, dY and grad must not be NULL");
  SurrWork w;
  if (ism_status s = surr_work(m, B, w, stream)) return s;
  surr_fwd_bwd(m, X, nullptr, dY, B, w, stream);
  mlp::AdamArgs aa{};
  aa.part = w.part; aa.nchunk = w.nchunk; aa.grad = grad; aa.adam = 0;
  hipLaunchKernelGGL(mlp::mlp_reduce_adam_kernel, dim3((mlp::NPARAM + mlp::RA_PARAMS - 1) / mlp::RA_PARAMS), dim3(256), 0, stream, aa);
  HIP_TRY(hipGetLastError());
  return ISM_OK;
}

ism_status ism_surrogate_train_step(ism_surrogate *m, const float *X, const float *Y, int64_t B, float lr,
                                    float *loss_dev, hipStream_t stream) {
  g_err.clear();
  if (ism_status s = surr_check(m)) return s;
  if (B < 1) return fail(ISM_E_ARG, "B must be >= 1");
  if (!X || !Y) return fail(ISM_E_ARG, "X and Y must not be NULL");
  if (!std::isfinite(lr) || lr < 0.f) return fail(ISM_E_ARG, "lr must be finite and >= 0");
  SurrWork w;
  if (ism_status s = surr_work(m, B, w, stream)) return s;
  surr_fwd_bwd(m, X, Y, nullptr, B, w, stream);
  const int64_t t = m->step + 1;
  mlp::AdamArgs aa{};
  aa.part = w.part; aa.nchunk = w.nchunk; aa.theta = m->theta(); aa.m = m->adam_m(); aa.v = m->adam_v();
  aa.fimg = m->fimg(); aa.bimg = m->bimg(); aa.lr = lr; aa.b1 = 0.9f; aa.b2 = 0.999f; aa.eps = 1e-8f;
  aa.bc1 = (float)(1.0 - std::pow(0.9, (double)t));
  aa.bc2 = (float)(1.0 - std::pow(0.999, (double)t));
  aa.adam = 1;
  if (loss_dev)
    hipLaunchKernelGGL(mlp::mlp_loss_kernel, dim3(1), dim3(256), 0, stream, w.loss_part,
                       w.grid_fwd * mlp::FWD_WAVES, 1.0 / (3.0 * (double)B), loss_dev);
  hipLaunchKernelGGL(mlp::mlp_reduce_adam_kernel, dim3((mlp::NPARAM + mlp::RA_PARAMS - 1) / mlp::RA_PARAMS), dim3(256), 0, stream, aa);
  HIP_TRY(hipGetLastError());
  m->step = t;
  return ISM_OK;
}

ism_status ism_surrogate_get_params(const ism_surrogate *m, float *flat, hipStream_t stream) {
  g_err.clear();
  if (ism_status s = surr_check(m)) return s;
  if (!flat) return fail(ISM_E_ARG, "flat is NULL");
  HIP_TRY(hipEventSynchronize(m->staged));
  HIP_TRY(hipMemcpyAsync(m->staging, m->params, 3 * (size_t)mlp::NPARAM * sizeof(float), hipMemcpyDeviceToHost,
                         stream));
  HIP_TRY(hipStreamSynchronize(stream));
  std::memcpy(flat, m->staging, 3 * (size_t)mlp::NPARAM * sizeof(float));
  flat[3 * mlp::NPARAM] = (float)m->step;
  std::memcpy(flat + 3 * mlp::NPARAM + 1, m->norm_host, sizeof(m->norm_host));
  return ISM_OK;
}

ism_status ism_surrogate_set_params(ism_surrogate *m, const float *flat, hipStream_t stream) {
  g_err.clear();
  if (ism_status s = surr_check(m)) return s;
  if (!flat) return fail(ISM_E_ARG, "flat is NULL");
  for (size_t i = 0; i < (size_t)ISM_SURR_STATE_FLOATS; ++i)
    if (!std::isfinite(flat[i])) return fail(ISM_E_ARG, "state holds a non-finite value");
  const float step = flat[3 * mlp::NPARAM];
  if (step < 0.f || step != std::floor(step)) return fail(ISM_E_ARG, "step must be a whole number >= 0");
  const float *nh = flat + 3 * mlp::NPARAM + 1;
  for (int k = 10; k < 20; ++k)
    if (!(nh[k] > 0.f)) return fail(ISM_E_ARG, "sd_x must be > 0");
  for (int k = 23; k < 26; ++k)
    if (!(nh[k] > 0.f)) return fail(ISM_E_ARG, "sd_y must be > 0");
  // the staging buffer may still feed the previous upload: wait for that copy alone
  HIP_TRY(hipEventSynchronize(m->staged));
  std::memcpy(m->staging, flat, 3 * (size_t)mlp::NPARAM * sizeof(float));
  HIP_TRY(hipMemcpyAsync(m->params, m->staging, 3 * (size_t)mlp::NPARAM * sizeof(float), hipMemcpyHostToDevice,
                         stream));
  HIP_TRY(hipEventRecord(m->staged, stream));
  m->step = (int64_t)step;
  std::memcpy(m->norm_host, nh, sizeof(m->norm_host));
  return surr_pack(m, stream);
}

ism_status ism_columns_beam(const ism_grid *g, const ism_params *p, ism_precision prec, const double *n,
                            const double *xH2, const double *xC, void *chi_PE, void *chi_LW, void *chi_H2,
                            void *chi_C, void *N_eff, void *xi_cr, hipStream_t stream) {
  g_err.clear();
  if (!g) return fail(ISM_E_ARG, "grid is NULL");
  if (ism_status s = check_params(p)) return s;
  if (prec != ISM_PREC_F64 && prec != ISM_PREC_MIXED) return fail(ISM_E_ARG, "invalid precision");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(ISM_E_ARG, "grid dimensions must be >= 1");
  if (!(g->dx_cm > 0.0) || !std::isfinite(g->dx_cm)) return fail(ISM_E_ARG, "dx_cm must be finite and > 0");
  if (!n || !xH2 || !chi_PE || !chi_LW || !chi_H2 || !chi_C || !N_eff)
    return fail(ISM_E_ARG, "n, xH2 and all chi/N_eff outputs must be non-NULL");
  if (p->cr_mode != 2 && !xi_cr) return fail(ISM_E_ARG, "xi_cr output is NULL (cr_mode 0/1 writes it)");
  DevState *st;
  if (ism_status s = current_state(&st)) return s;
  ColArgs a{};
  a.nx = g->nx; a.ny = g->ny; a.nz = g->nz; a.dx = g->dx_cm;
  a.n = n; a.xH2 = xH2; a.xC = xC;
  a.chiPE = chi_PE; a.chiLW = chi_LW; a.chiH2 = chi_H2; a.chiC = chi_C; a.Neff = N_eff; a.xi = xi_cr;
  a.cr_mode = p->cr_mode;
  a.chi0 = p->chi0; a.Zd = p->Zd; a.xi0 = p->xi_cr0;
  a.sPE = g_host_coef.sig_d_abs[2] * p->Zd;
  a.sLW = g_host_coef.sig_d_abs[1] * p->Zd;
  a.tab = st->tab64;
  const int64_t rows = (int64_t)g->ny * g->nz;
  const dim3 grid((unsigned)((rows + 3) / 4));
  if (prec == ISM_PREC_MIXED) hipLaunchKernelGGL(columns_beam_kernel<float>, grid, dim3(256), 0, stream, a);
  else hipLaunchKernelGGL(columns_beam_kernel<double>, grid, dim3(256), 0, stream, a);
  HIP_TRY(hipGetLastError());
  return ISM_OK;
}

ism_status ism_local_shielding(const ism_params *p, ism_precision prec, int64_t ncell, const double *n,
                               const double *xH2, const double *xC, const double *L_cm, void *chi_PE, void *chi_LW,
                               void *chi_H2, void *chi_C, void *N_eff, void *xi_cr, hipStream_t stream) {
  g_err.clear();
  if (ism_status s = check_params(p)) return s;
  if (prec != ISM_PREC_F64 && prec != ISM_PREC_MIXED) return fail(ISM_E_ARG, "invalid precision");
  if (ncell < 0) return fail(ISM_E_ARG, "ncell must be >= 0");
  if (ncell == 0) return ISM_OK;
  if (!n || !xH2 || !L_cm || !chi_PE || !chi_LW || !chi_H2 || !chi_C || !N_eff || (!xi_cr && p->cr_mode != 2))
    return fail(ISM_E_ARG, "a required array is NULL");
  DevState *st;
  if (ism_status s = current_state(&st)) return s;
  const double sPE = g_host_coef.sig_d_abs[2] * p->Zd, sLW = g_host_coef.sig_d_abs[1] * p->Zd;
  const dim3 grid((unsigned)((ncell + 255) / 256));
  if (prec == ISM_PREC_F64)
    hipLaunchKernelGGL(local_shield_kernel<double>, grid, dim3(256), 0, stream, ncell, n, xH2, xC, L_cm,
                       (double *)chi_PE, (double *)chi_LW, (double *)chi_H2, (double *)chi_C, (double *)N_eff,
                       (double *)xi_cr, p->chi0, sPE, sLW, p->xi_cr0, p->cr_mode, st->tab64);
  else
    hipLaunchKernelGGL(local_shield_kernel<float>, grid, dim3(256), 0, stream, ncell, n, xH2, xC, L_cm,
                       (float *)chi_PE, (float *)chi_LW, (float *)chi_H2, (float *)chi_C, (float *)N_eff,
                       (float *)xi_cr, p->chi0, sPE, sLW, p->xi_cr0, p->cr_mode, st->tab64);
  HIP_TRY(hipGetLastError());
  return ISM_OK;
}

ism_status ism_point_sources(const ism_grid *g, const ism_params *p, ism_precision prec, int32_t nsrc,
                             const ism_source *src, const double *n, const double *xH2, const double *xC,
                             void *chi_PE, void *chi_LW, void *chi_H2, void *chi_C, void *phi_LyC,
                             hipStream_t stream) {
  g_err.clear();
  if (!g) return fail(ISM_E_ARG, "grid is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(ISM_E_ARG, "grid dimensions must be >= 1");
  if (!(g->dx_cm > 0.0) || !std::isfinite(g->dx_cm)) return fail(ISM_E_ARG, "dx_cm must be finite and > 0");
  if (ism_status s = check_params(p)) return s;
  if (prec != ISM_PREC_F64 && prec != ISM_PREC_MIXED) return fail(ISM_E_ARG, "invalid precision");
  if (nsrc < 0 || nsrc > MAX_SOURCES) return fail(ISM_E_ARG, "nsrc must be in [0, 256]");
  if (nsrc == 0) return ISM_OK;
  if (!src || !n || !xH2 || !chi_PE || !chi_LW || !chi_H2 || !chi_C || !phi_LyC)
    return fail(ISM_E_ARG, "a required array is NULL");
  DevState *st;
  if (ism_status s = current_state(&st)) return s;
  const double box[3] = {g->nx * g->dx_cm, g->ny * g->dx_cm, g->nz * g->dx_cm};
  const double Rst_pref = 3.0 / (4.0 * M_PI * g_host_coef.alpha_B[0]);  // alpha_B(1e4 K), mean density 1
  SrcDev h[MAX_SOURCES];
  for (int s = 0; s < nsrc; ++s) {
    const double pos[3] = {src[s].x_cm, src[s].y_cm, src[s].z_cm};
    for (int q = 0; q < 3; ++q)
      if (!(pos[q] >= 0.0 && pos[q] < box[q])) return fail(ISM_E_ARG, "a source lies outside the grid");
    if (!(src[s].Q >= 0.0) || !std::isfinite(src[s].Q) || !(src[s].L_FUV >= 0.0) || !std::isfinite(src[s].L_FUV))
      return fail(ISM_E_ARG, "source Q and L_FUV must be finite and >= 0");
    h[s] = SrcDev{pos[0] / g->dx_cm, pos[1] / g->dx_cm, pos[2] / g->dx_cm, src[s].Q, src[s].L_FUV,
                  std::cbrt(Rst_pref * src[s].Q)};
  }
  HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(g_src), h, sizeof(SrcDev) * nsrc));
  const double Zd = p->Zd;
  PsArgs a{g->nx, g->ny, g->nz, nsrc, 0, 0, g->dx_cm, n, xH2, xC, chi_PE, chi_LW, chi_H2, chi_C, phi_LyC,
           g_host_coef.sig_d_abs[2] * Zd, g_host_coef.sig_d_abs[1] * Zd, g_host_coef.sig_d_abs[0] * Zd,
           1.0 / (16.0 * M_PI * M_PI * g_host_coef.J_FUV), st->tab64};
  const int64_t ncell = (int64_t)g->nx * g->ny * g->nz;
  const dim3 grid((unsigned)((ncell + 255) / 256));
  for (int s = 0; s < nsrc; ++s) {
    a.s0 = s;
    a.s1 = s + 1;
    if (prec == ISM_PREC_F64)
      hipLaunchKernelGGL(point_sources_kernel<double>, grid, dim3(256), 0, stream, a);
    else
      hipLaunchKernelGGL(point_sources_kernel<float>, grid, dim3(256), 0, stream, a);
  }
  HIP_TRY(hipGetLastError());
  return ISM_OK;
}

// Packet list b with room for at least `rays` packets (grows, never shrinks).
// Packet list b of the stream's scratch with room for at least `rays` packets (grows, never
// shrinks), and the pinned host word the child count is read back into.
ism_status art_list(StreamScratch *ss, int b, int64_t rays, hipStream_t stream) {
  if (!ss->art_count_host) {
    hipError_t e = hipHostMalloc(&ss->art_count_host, sizeof(unsigned long long));
    if (e != hipSuccess) return fail(ISM_E_NOMEM, std::string("ray counter (host): ") + hipGetErrorString(e));
  }
  const int64_t want = std::max<int64_t>(rays, 1 << 16);
  if (ss->art_b[b] < sizeof(ArtRay) * (size_t)rays || !ss->art[b])
    if (ism_status s = grow(&ss->art[b], &ss->art_b[b], sizeof(ArtRay) * (size_t)want, stream, "ray list"))
      return s;
  return ISM_OK;
}

ism_status ism_ray_trace(const ism_grid *g, const ism_params *p, ism_precision prec, int32_t nsrc,
                         const ism_source *src, const ism_art_options *opt, const double *n, const double *xH2,
                         const double *xHp, const double *xC, void *chi_PE, void *chi_LW, void *chi_H2,
                         void *chi_C, void *phi_LyC, void *flux, double *budget, hipStream_t stream) {
  g_err.clear();
  if (!g) return fail(ISM_E_ARG, "grid is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(ISM_E_ARG, "grid dimensions must be >= 1");
  if ((int64_t)g->nx * g->ny * g->nz > (int64_t)INT32_MAX)
    return fail(ISM_E_ARG, "grid too large for the ray tracer (at most 2^31 - 1 cells)");
  if (!(g->dx_cm > 0.0) || !std::isfinite(g->dx_cm)) return fail(ISM_E_ARG, "dx_cm must be finite and > 0");
  if (ism_status s = check_params(p)) return s;
  if (prec != ISM_PREC_F64 && prec != ISM_PREC_MIXED) return fail(ISM_E_ARG, "invalid precision");
  if (nsrc < 0 || nsrc > MAX_SOURCES) return fail(ISM_E_ARG, "nsrc must be in [0, 256]");
  ism_art_options o{4, 13, 4.0, 30.0};
  if (opt) o = *opt;
  if (o.level0 < 0 || o.level0 > o.max_level || o.max_level > ART_MAX_LEVEL)
    return fail(ISM_E_ARG, "need 0 <= level0 <= max_level <= 13");
  if (!(o.rays_per_cell > 0.0) || !std::isfinite(o.rays_per_cell))
    return fail(ISM_E_ARG, "rays_per_cell must be finite and > 0");
  if (!(o.tau_max > 0.0)) return fail(ISM_E_ARG, "tau_max must be > 0");
  if (nsrc == 0) return ISM_OK;
  if (!src || !n || !xH2 || !xHp || !chi_PE || !chi_LW || !chi_H2 || !chi_C || !phi_LyC)
    return fail(ISM_E_ARG, "a required array is NULL");
  DevState *st;
  int dev = 0;
  if (ism_status s = current_state(&st, &dev)) return s;
  StreamScratch *ss = stream_scratch(dev, stream);
  if (ism_status s = grow(&ss->ctl, &ss->ctl_b, 256, stream, "ray counter")) return s;
  unsigned long long *art_count = (unsigned long long *)ss->ctl + 2;
  const double box[3] = {g->nx * g->dx_cm, g->ny * g->dx_cm, g->nz * g->dx_cm};
  SrcDev h[MAX_SOURCES];
  for (int s = 0; s < nsrc; ++s) {
    const double pos[3] = {src[s].x_cm, src[s].y_cm, src[s].z_cm};
    for (int q = 0; q < 3; ++q)
      if (!(pos[q] >= 0.0 && pos[q] < box[q])) return fail(ISM_E_ARG, "a source lies outside the grid");
    if (!(src[s].Q >= 0.0) || !std::isfinite(src[s].Q) || !(src[s].L_FUV >= 0.0) || !std::isfinite(src[s].L_FUV))
      return fail(ISM_E_ARG, "source Q and L_FUV must be finite and >= 0");
    h[s] = SrcDev{pos[0] / g->dx_cm, pos[1] / g->dx_cm, pos[2] / g->dx_cm, src[s].Q, src[s].L_FUV, 0.0};
  }
  HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(g_src), h, sizeof(SrcDev) * nsrc));
  const double Zd = p->Zd;
  const double dV = g->dx_cm * g->dx_cm * g->dx_cm;
  ArtArgs a{};
  a.nx = g->nx; a.ny = g->ny; a.nz = g->nz; a.nsrc = nsrc;
  a.max_level = o.max_level;
  a.dx = g->dx_cm;
  a.tau_max = o.tau_max;
  a.n = n; a.xH2 = xH2; a.xHp = xHp; a.xC = xC;
  a.chiPE = chi_PE; a.chiLW = chi_LW; a.chiH2 = chi_H2; a.chiC = chi_C; a.phi = phi_LyC;
  a.sPE = g_host_coef.sig_d_abs[2] * Zd;
  a.sLW = g_host_coef.sig_d_abs[1] * Zd;
  a.sdLyC = g_host_coef.sig_d_abs[0] * Zd;
  a.spiH = g_host_coef.sig_pi_H;
  a.spiH2 = g_host_coef.sig_pi_H2;
  a.fuv_norm = 1.0 / (4.0 * M_PI * dV * g_host_coef.J_FUV);
  a.phi_norm = 1.0 / dV;
  a.budget = budget;
  a.tab = st->tab64;
  a.flux = flux;
  a.ncell = (int64_t)g->nx * g->ny * g->nz;
  a.kPE = 4.0 * M_PI * g_host_coef.J_PE;
  a.kLW = 4.0 * M_PI * g_host_coef.J_LW;
  if (budget)
    hipLaunchKernelGGL(art_zero_kernel, dim3((unsigned)((6 * nsrc + 255) / 256)), dim3(256), 0, stream, budget,
                       (int64_t)6 * nsrc, (unsigned long long *)nullptr);
  const size_t lds = budget ? sizeof(double) * 6 * (size_t)nsrc : 0;
  int64_t nin = (int64_t)nsrc * (12ll << (2 * o.level0));
  int cur = 0;
  for (int level = o.level0; nin > 0 && level <= o.max_level; ++level) {
    const int nxt = cur ^ 1;
    if (ism_status s = art_list(ss, nxt, level < o.max_level ? 4 * nin : 0, stream)) return s;
    a.level = level;
    a.nin = nin;
    a.in = level == o.level0 ? nullptr : (ArtRay *)ss->art[cur];
    a.out = (ArtRay *)ss->art[nxt];
    a.nout = art_count;
    a.R2split = (12.0 * std::ldexp(1.0, 2 * level)) / (4.0 * M_PI * o.rays_per_cell);
    hipLaunchKernelGGL(art_zero_kernel, dim3(1), dim3(64), 0, stream, (double *)nullptr, (int64_t)0, art_count);
    const dim3 grid((unsigned)((nin + 255) / 256));
    if (prec == ISM_PREC_F64) {
      if (flux)
        hipLaunchKernelGGL((art_level_kernel<double, true>), grid, dim3(256), lds, stream, a);
      else
        hipLaunchKernelGGL((art_level_kernel<double, false>), grid, dim3(256), lds, stream, a);
    } else {
      if (flux)
        hipLaunchKernelGGL((art_level_kernel<float, true>), grid, dim3(256), lds, stream, a);
      else
        hipLaunchKernelGGL((art_level_kernel<float, false>), grid, dim3(256), lds, stream, a);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(ss->art_count_host, art_count, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           stream));
    HIP_TRY(hipStreamSynchronize(stream));
    nin = level < o.max_level ? (int64_t)*ss->art_count_host : 0;
    cur = nxt;
  }
  return ISM_OK;
}

ism_status ism_radiation_force(const ism_params *p, ism_precision prec, int64_t ncell, const double *n,
                               const double *T, const double *xH2, const double *xHp, const void *flux,
                               const ism_force_options *opt, void *f_rad, uint8_t *dust_off, double dt_s,
                               double *mom, double *etot, hipStream_t stream) {
  g_err.clear();
  if (ism_status s = check_params(p)) return s;
  if (prec != ISM_PREC_F64 && prec != ISM_PREC_MIXED) return fail(ISM_E_ARG, "invalid precision");
  if (ncell < 0) return fail(ISM_E_ARG, "ncell must be >= 0");
  ism_force_options o{1.0e6, 50.0};
  if (opt) o = *opt;
  if (!(o.T_destroy_K > 0.0)) return fail(ISM_E_ARG, "T_destroy_K must be > 0");
  if (!(o.prad_ratio_max > 0.0)) return fail(ISM_E_ARG, "prad_ratio_max must be > 0");
  if (!(dt_s >= 0.0) || !std::isfinite(dt_s)) return fail(ISM_E_ARG, "dt_s must be finite and >= 0");
  if (etot && !mom) return fail(ISM_E_ARG, "etot needs mom");
  if (ncell > (int64_t)0xFFFFFF00ll) return fail(ISM_E_ARG, "ncell must be in [0, 2^32 - 256]");
  if (ncell == 0) return ISM_OK;
  if (!n || !T || !xH2 || !xHp || !flux || !f_rad) return fail(ISM_E_ARG, "a required array is NULL");
  DevState *st;
  if (ism_status s = current_state(&st)) return s;
  const double Zd = p->Zd;
  ForceArgs a{};
  a.ncell = ncell;
  a.n = n; a.T = T; a.xH2 = xH2; a.xHp = xHp;
  a.flux = flux; a.f = f_rad; a.dust_off = dust_off; a.mom = mom; a.etot = etot;
  a.dt = dt_s;
  a.T_destroy = o.T_destroy_K;
  a.prad_ratio_max = o.prad_ratio_max;
  a.sPE = g_host_coef.sig_d_abs[2] * Zd;
  a.sLW = g_host_coef.sig_d_abs[1] * Zd;
  a.sdLyC = g_host_coef.sig_d_abs[0] * Zd;
  a.spiH = g_host_coef.sig_pi_H;
  a.spiH2 = g_host_coef.sig_pi_H2;
  a.hnu = g_host_coef.hnu_LyC_eV * EV;
  a.inv_c = 1.0 / C_LIGHT;
  a.two_kB = 2.0 * K_B;
  a.rho_per_n = (g_host_coef.muH0 - g_host_coef.muH_slope * (p->Zg - 1.0)) * M_H;
  const dim3 grid((unsigned)((ncell + 255) / 256));
  if (prec == ISM_PREC_F64)
    hipLaunchKernelGGL(radiation_force_kernel<double>, grid, dim3(256), 0, stream, a);
  else
    hipLaunchKernelGGL(radiation_force_kernel<float>, grid, dim3(256), 0, stream, a);
  HIP_TRY(hipGetLastError());
  return ISM_OK;
}

ism_status ism_surrogate_pairs(const ism_params *p, ism_precision prec, int64_t ncell, double dt_s, const double *n,
                               const double *T0, const double *xH2_0, const double *xHp_0, const void *chi_PE,
                               const void *phi_LyC, const void *xi_cr, const void *N_eff, const double *T1,
                               const double *xH2_1, const double *xHp_1, float *X, float *Y, hipStream_t stream) {
  g_err.clear();
  if (ism_status s = check_params(p)) return s;
  if (prec != ISM_PREC_F64 && prec != ISM_PREC_MIXED) return fail(ISM_E_ARG, "invalid precision");
  if (ncell < 0) return fail(ISM_E_ARG, "ncell must be >= 0");
  if (!(dt_s > 0.0) || !std::isfinite(dt_s)) return fail(ISM_E_ARG, "dt_s must be finite and > 0");
  if (ncell == 0) return ISM_OK;
  if (!n || !T0 || !xH2_0 || !xHp_0 || !chi_PE || !xi_cr || !N_eff || !X)
    return fail(ISM_E_ARG, "a required array is NULL");
  if (Y && (!T1 || !xH2_1 || !xHp_1)) return fail(ISM_E_ARG, "targets need T1, xH2_1 and xHp_1");
  DevState *st;
  if (ism_status s = current_state(&st)) return s;
  const float lZg = (float)std::log10(p->Zg), ldt = (float)std::log10(dt_s / 3.15576e7);
  const dim3 grid((unsigned)((ncell + 255) / 256));
  if (prec == ISM_PREC_F64) {
    mlp::CellIn<double> c{n, T0, xH2_0, xHp_0, (const double *)chi_PE, (const double *)phi_LyC,
                          (const double *)xi_cr, (const double *)N_eff, lZg, ldt};
    hipLaunchKernelGGL(mlp::mlp_pairs_kernel<double>, grid, dim3(256), 0, stream, c, ncell, T1, xH2_1, xHp_1, X, Y);
  } else {
    mlp::CellIn<float> c{n, T0, xH2_0, xHp_0, (const float *)chi_PE, (const float *)phi_LyC,
                         (const float *)xi_cr, (const float *)N_eff, lZg, ldt};
    hipLaunchKernelGGL(mlp::mlp_pairs_kernel<float>, grid, dim3(256), 0, stream, c, ncell, T1, xH2_1, xHp_1, X, Y);
  }
  HIP_TRY(hipGetLastError());
  return ISM_OK;
}

ism_status ism_chem_cool_step_surrogate(ism_surrogate *m, const ism_params *p, int64_t ncell, double dt_s,
                                        const double *n, double *T, double *xH2, double *xHp, const void *chi_PE,
                                        const void *chi_LW, const void *chi_H2, const void *chi_C,
                                        const void *phi_LyC, const void *xi_cr, const void *N_eff, void *xCp,
                                        void *xCO, void *xe, int32_t *nsub, uint8_t *status, double accept_tol,
                                        int64_t *n_fallback_dev, hipStream_t stream) {
  g_err.clear();
  if (m) {
    if (ism_status s = surr_check(m)) return s;
  }
  if (ism_status s = check_params(p)) return s;
  if (ncell < 0 || ncell > (int64_t)INT32_MAX) return fail(ISM_E_ARG, "ncell must be in [0, 2^31)");
  if (!(dt_s >= 0.0) || !std::isfinite(dt_s)) return fail(ISM_E_ARG, "dt_s must be finite and >= 0");
  if (!(accept_tol > 0.0 && accept_tol <= 1e-3)) return fail(ISM_E_ARG, "accept_tol must be in (0, 1e-3]");
  if (ncell == 0) {
    if (n_fallback_dev) hipLaunchKernelGGL(queue_init_kernel, dim3(1), dim3(1), 0, stream, n_fallback_dev, (int64_t)0);
    HIP_TRY(hipGetLastError());
    return ISM_OK;
  }
  if (!n || !T || !xH2 || !xHp || !chi_PE || !chi_LW || !chi_H2 || !chi_C || !xi_cr || !N_eff)
    return fail(ISM_E_ARG, "a required array is NULL");
  DevState *st;
  int dev = 0;
  if (ism_status s = current_state(&st, &dev)) return s;
  StreamScratch *ss = stream_scratch(dev, stream);
  // scratch: predictions (one per candidate), the chemistry-passing list, the candidate list,
  // the fallback list
  const size_t pred_bytes = m ? align256((size_t)ncell * 3 * sizeof(float)) : 0;
  const size_t list_bytes = align256((size_t)ncell * sizeof(int32_t));
  if (ism_status s = grow(&ss->surr, &ss->surr_b, pred_bytes + 3 * list_bytes, stream, "surrogate scratch")) return s;
  if (ism_status s = grow(&ss->ctl, &ss->ctl_b, 256, stream, "work-queue counter")) return s;
  if (p->order_cells)
    if (ism_status s = grow(&ss->ord, &ss->ord_b, order_bytes(ncell), stream, "order scratch")) return s;
  float *pred = m ? (float *)ss->surr : nullptr;
  int32_t *chem = (int32_t *)((uint8_t *)ss->surr + pred_bytes);
  int32_t *cand = (int32_t *)((uint8_t *)ss->surr + pred_bytes + list_bytes);
  int32_t *rej = (int32_t *)((uint8_t *)ss->surr + pred_bytes + 2 * list_bytes);
  int64_t *q = (int64_t *)ss->ctl;
  unsigned long long *nrej = (unsigned long long *)ss->ctl + 1;
  unsigned long long *ncand = (unsigned long long *)ss->ctl + 2;
  unsigned long long *nchem = (unsigned long long *)ss->ctl + 3;
  hipLaunchKernelGGL(counter_reset_kernel, dim3(1), dim3(1), 0, stream, nrej);
  hipLaunchKernelGGL(counter_reset_kernel, dim3(1), dim3(1), 0, stream, ncand);
  hipLaunchKernelGGL(counter_reset_kernel, dim3(1), dim3(1), 0, stream, nchem);
  const ParT<float> pr = make_par<float>(p, g_host_coef);
  const ParT<double> pd = make_par<double>(p, g_host_coef);
  constexpr double FAST = 20.0;  // dt times the slowest relaxation rate an accepted cell needs
  const int64_t lgrid = std::min<int64_t>((ncell + 255) / 256, (int64_t)std::max(st->num_cu, 1) * 4);
  // 1. the pre-test on the input state: chemical rates on every cell, then the thermal rate on
  //    the cells that passed; the others start the fallback list
  PreArgs pa{ncell, dt_s, n, T, xH2, xHp, (const float *)chi_PE, (const float *)chi_LW, (const float *)chi_H2,
             (const float *)chi_C, (const float *)phi_LyC, (const float *)xi_cr, (const float *)N_eff,
             st->tab32, pr, pd, FAST, nullptr, nullptr, chem, rej, nchem, nrej};
  hipLaunchKernelGGL(surr_pretest_kernel, dim3((unsigned)((ncell + PRETEST_THREADS - 1) / PRETEST_THREADS)),
                     dim3(PRETEST_THREADS), 0, stream, pa);
  pa.in = chem; pa.nin = nchem; pa.pass = cand; pa.npass = ncand;
  hipLaunchKernelGGL(surr_pretest_thermal_kernel, dim3((unsigned)lgrid), dim3(256), 0, stream, pa);
  // 2. the network on the candidates only (their count is read on the device)
  if (m) {
    mlp::FwdArgs fa{};
    fa.cin = mlp::CellIn<float>{n, T, xH2, xHp, (const float *)chi_PE, (const float *)phi_LyC,
                                (const float *)xi_cr, (const float *)N_eff, (float)std::log10(p->Zg),
                                (float)std::log10(std::max(dt_s, 1e-300) / 3.15576e7), cand};
    fa.B = ncell; fa.count = ncand; fa.fimg = m->fimg(); fa.norm = surr_norm(m); fa.Y = pred;
    hipLaunchKernelGGL(mlp::mlp_fwd_kernel<3>, dim3(fwd_grid(m, ncell)), dim3(mlp::FWD_THREADS), 0, stream, fa);
  }
  // 3. certification of the candidates; the rejected ones join the fallback list
  AcceptArgs aa{cand, ncand, dt_s, n, T, xH2, xHp, (const float *)chi_PE, (const float *)chi_LW,
                (const float *)chi_H2, (const float *)chi_C, (const float *)phi_LyC, (const float *)xi_cr,
                (const float *)N_eff, (float *)xCp, (float *)xCO, (float *)xe, nsub, status, pred, st->tab32, pr, pd,
                rej, nrej, FAST, accept_tol, 6, 1e-3};
  hipLaunchKernelGGL(accept_kernel, dim3((unsigned)lgrid), dim3(256), 0, stream, aa);
  // 4. the plain MIXED step on the fallback list, ordered by temperature
  int32_t *list = rej;
  if (p->order_cells) order_cells((uint8_t *)ss->ord, ncell, nrej, rej, T, nullptr, &list, stream);
  StepArgs<float> sa{ncell, dt_s, n, T, xH2, xHp, (const float *)chi_PE, (const float *)chi_LW,
                     (const float *)chi_H2, (const float *)chi_C, (const float *)phi_LyC,
                     (const float *)xi_cr, (const float *)N_eff, (float *)xCp, (float *)xCO, (float *)xe,
                     nsub, status, st->tab32, pr, pd, q, list, nrej, (uint32_t)ISM_ST_FALLBACK};
  const int64_t grid = std::min<int64_t>((ncell + 255) / 256, (int64_t)st->num_cu * std::max(st->occ32, 1));
  hipLaunchKernelGGL(queue_init_kernel, dim3(1), dim3(1), 0, stream, q, grid * 256);
  hipLaunchKernelGGL(step_queue_kernel<float>, dim3((unsigned)grid), dim3(256), 0, stream, sa);
  if (n_fallback_dev) hipLaunchKernelGGL(counter_copy_kernel, dim3(1), dim3(1), 0, stream, nrej, n_fallback_dev);
  HIP_TRY(hipGetLastError());
  return ISM_OK;
}

}  // extern "C"
