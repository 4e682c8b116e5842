/*
 * ism.h -- C ABI of the MI355X ISM photochemistry + heating/cooling source step.
 *
 * Method: Kim, Gong, Kim & Ostriker, "Photochemistry and Heating/Cooling of the
 * Multiphase Interstellar Medium with UV Radiative Transfer for Magnetohydrodynamic
 * Simulations" (arXiv:2210.08024).  Each entry point names the passage that defines
 * the operation it performs.
 *
 * Conventions (all entry points):
 *  - Pointers named as arrays are DEVICE pointers (hipMalloc / torch CUDA tensors),
 *    contiguous, owned by the caller, at least 8-byte aligned; the library never
 *    frees or retains them.  Scalars and structs are passed by host pointer.
 *  - Units are cgs: n [cm^-3], T [K], dt [s], dx [cm], chi in Draine-field units,
 *    phi_LyC [photons cm^-2 s^-1], xi_cr [s^-1], columns [cm^-2].
 *  - Grids are indexed idx = i + nx * (j + ny * k), x fastest.
 *  - ISM_PREC_F64: every floating array is double.  ISM_PREC_MIXED: the cell state
 *    (n, T, x_H2, x_H+) stays double; radiation inputs/outputs and the derived
 *    abundance outputs (x_C+, x_CO, x_e) are float.
 *  - Work is enqueued asynchronously on the given stream (NULL = default stream);
 *    nothing synchronises except where stated.
 *  - Argument errors are detected before anything is enqueued and return ISM_E_ARG;
 *    launch/runtime errors return ISM_E_DEVICE.  ism_last_error() gives the message
 *    (thread-local).  Per-cell numerical trouble never fails a call: it is reported
 *    in the per-cell status bits below and the call returns ISM_OK.
 *  - Scratch and thread safety: library scratch (tile sums, ordering keys, work-queue
 *    counters, the surrogate step's predictions, ray lists) belongs to the (device, stream)
 *    a call is enqueued on, so after ism_init every step and column entry point may run
 *    concurrently on different streams; calls on one stream are ordered by it (make them
 *    from one thread at a time).  Scratch grows with stream-ordered allocation
 *    (hipMallocAsync / hipFreeAsync on that stream) and is kept until ism_stream_release or
 *    ism_shutdown; nothing here synchronises the device.  The exceptions are stated at
 *    each call: the point-source entry points (ism_point_sources, ism_ray_trace) copy their
 *    sources into constant memory, so their calls on one device must not overlap in time,
 *    and ism_ray_trace waits for its stream after each level.
 */
#ifndef ISM_H
#define ISM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ISM_OK = 0,
  ISM_E_ARG = -1,     /* invalid argument (null, size, range)            */
  ISM_E_DEVICE = -2,  /* HIP runtime / launch failure                    */
  ISM_E_NOMEM = -3,   /* device allocation failed                        */
  ISM_E_STATE = -4,   /* library not initialised on this device          */
  ISM_E_TABLE = -5    /* coefficient file missing, unreadable or invalid */
} ism_status;

typedef enum { ISM_PREC_F64 = 0, ISM_PREC_MIXED = 1 } ism_precision;

/* Per-cell status bits written by the step entry points. */
enum {
  ISM_ST_SUBSTEP_CAP = 1,   /* max_substeps reached before t = dt                 */
  ISM_ST_NONFINITE = 2,     /* a non-finite value appeared; the cell stopped      */
  ISM_ST_T_FLOOR = 4,       /* the temperature floor was applied                  */
  ISM_ST_DENOM_GUARD = 8,   /* T-update denominator guard fired                   */
  ISM_ST_FALLBACK = 16,     /* surrogate rejected, plain solver used              */
  ISM_ST_TD_UNBRACKETED = 32 /* dust-temperature root not bracketed, T_d = 1e4 K  */
};

/* Uniform Cartesian grid (Sec. 5.2): nx*ny*nz cells of side dx_cm. */
typedef struct {
  int32_t nx, ny, nz;
  int32_t pad_;
  double dx_cm;
} ism_grid;

/* Parameters of the source step (Table t:param, Sec. 6.1, Sec. 7.1.2). */
typedef struct {
  double Zg;            /* scaled gas metallicity Z'_g (> 0)                              */
  double Zd;            /* scaled dust abundance Z'_d (> 0)                               */
  double chi0;          /* unattenuated FUV at the domain faces, Draine units (Sec. 5.2)  */
  double xi_cr0;        /* unattenuated primary CR ionisation rate [s^-1] (Sec. 2.4)      */
  double dvdr_kms_pc;   /* |dv/dr| for the CO LVG column (Sec. 4.6.2, default 1)          */
  double eps_sub;       /* substep limiter factor (Sec. 6.1, 0.1)                         */
  double fd_rel;        /* relative step of the forward difference dH/dT_mu (1e-3)        */
  double T_floor;       /* temperature floor [K] (1)                                       */
  double T_bb;          /* dust bath blackbody temperature [K] (Sec. 7.1.2, 6)            */
  double tau_opt_ratio; /* tau_PE,eff / tau_OPT (Sec. 7.1.2, 1.87)                        */
  int32_t cr_mode;      /* columns6: 0 xi = xi_cr0, 1 Eq. e:cratt on N_eff, 2 leave xi_cr  */
  int32_t kgr_const;    /* 1: k_gr = 3e-17 Z'_d (Sec. 7); 0: Eq. e:H2form                 */
  int32_t h2_rovib;     /* 1: include H2 ro-vibrational cooling                           */
  int32_t max_substeps; /* substep cap per cell (100000)                                   */
  int32_t order_cells;  /* step calls: 1 (default) process cells grouped by temperature (about
                           half a decade) and, within that, by slab of the grid, so that the lanes
                           of a wave stay in one regime and load nearby cells; 0 in index order;
                           2 (ism_chem_cool_step with an nsub array) grouped by the
                           substep counts nsub holds on entry, e.g. the previous step's
                           of the same cells, longest first (as 1 without nsub; the
                           surrogate step treats 2 as 1).  Results are identical in
                           every mode.                                                    */
  int32_t pad_;
} ism_params;

/* Fill *p with the defaults listed above (Z'_g = Z'_d = chi0 = 1, xi_cr0 = 2e-16). */
void ism_params_default(ism_params *p);

/* Initialise the library on HIP device `device`: parse the coefficient file
 * (JSON: printed constants, stand-in coefficients and tables) and upload it.
 * Must precede every other call on that device; may be called again to reload.
 * Returns ISM_E_TABLE if the file is missing or invalid, ISM_E_DEVICE on HIP errors. */
ism_status ism_init(int device, const char *coefficients_json_path);

/* Release the library's device memory on every initialised device (synchronises them). */
ism_status ism_shutdown(void);

/* Release the scratch the library holds for `stream` on the current device (stream-ordered:
 * the memory is returned after the work already queued on the stream).  For callers that
 * destroy streams; the next call on the stream allocates afresh. */
ism_status ism_stream_release(hipStream_t stream);

/* Message of the last error on the calling thread ("" if none).  Library-owned. */
const char *ism_last_error(void);

/* Number of per-cell diagnostics written by ism_rates, and the name of diagnostic k
 * (NULL if k is out of range).  Library-owned strings. */
int32_t ism_ndiag(void);
const char *ism_diag_name(int32_t k);

/* Six-ray diffuse-UV transfer (Secs. 5.1-5.3; Eqs. e:Erad, e:Erad_H2, e:fshld_H2_DB,
 * e:tau_eff, e:cratt).  For every cell, rays from the six faces give
 *   chi_b   = chi0/6 sum_d exp(-sigma_b N_in,d) (1 - exp(-dtau_b)) / dtau_b,  b = PE, LW
 *   chi_H2  = same LW sum weighted by f_shld,H2(N_H2,in,d + n x_H2 dx / 2)
 *   chi_C   = same LW sum weighted by f_shld,C(N_C,in,d + n x_C dx/2, N_H2 mid-cell)
 *   N_eff   = -ln(chi_PE / chi0) / (1e-21 Z'_d)   (0 when chi0 = 0)
 *   xi_cr   = per p->cr_mode (not written when cr_mode = 2)
 * with upstream columns accumulated in double.
 * In: n, xH2 (double, ncell), xC (double or NULL = 0).  Out: chi_PE, chi_LW, chi_H2,
 * chi_C, N_eff, xi_cr (double for F64, float for MIXED).  Requires 1 <= nx, ny, nz <= 2^24
 * and at most 2^40 cells.  Scratch: about 27 bytes per cell on the call's stream (tile sums
 * and their forward / backward offsets); ISM_E_NOMEM when it cannot grow. */
ism_status ism_columns6(const ism_grid *g, const ism_params *p, ism_precision prec,
                        const double *n, const double *xH2, const double *xC,
                        void *chi_PE, void *chi_LW, void *chi_H2, void *chi_C,
                        void *N_eff, void *xi_cr, hipStream_t stream);

/* A beam of surface intensity chi0 (params) entering every x row through the x = 0 face
 * along +x: the plane-parallel slab of Sec. 7.3.  Per cell the same terms as one six-ray
 * direction of ism_columns6 with weight chi0 instead of chi0/6: dust attenuation to the entry
 * face times the cell average, H2 and C shielding at mid-cell.  N_eff and xi_cr as in
 * ism_columns6.  Arguments and layout as ism_columns6 (no scratch). */
ism_status ism_columns_beam(const ism_grid *g, const ism_params *p, ism_precision prec,
                            const double *n, const double *xH2, const double *xC,
                            void *chi_PE, void *chi_LW, void *chi_H2, void *chi_C,
                            void *N_eff, void *xi_cr, hipStream_t stream);

/* Local shielding-length radiation (Sec. 7.1.2): a cell of density n and shielding length
 * L_cm (per cell) sees the background through N_shld = n L:
 *   chi_PE/LW = chi0 exp(-sigma_PE/LW Z'_d N_shld), chi_H2 = chi_LW f_shld,H2(0.5 x_H2 n L),
 *   chi_C = chi_LW f_shld,C(0.5 x_C n L, 0.5 x_H2 n L), N_eff = N_shld,
 *   xi_cr: cr_mode 0 xi_cr0, 1 Eq. e:cratt on N_eff, 2 left unchanged (may be NULL).
 * In: n, xH2, L_cm (double), xC (double or NULL = 0).  Out: double (F64) or float (MIXED). */
ism_status ism_local_shielding(const ism_params *p, ism_precision prec, int64_t ncell,
                               const double *n, const double *xH2, const double *xC,
                               const double *L_cm, void *chi_PE, void *chi_LW, void *chi_H2,
                               void *chi_C, void *N_eff, void *xi_cr, hipStream_t stream);

/* A point source: position (cm from the grid corner, inside the grid), ionising photon rate
 * Q [s^-1] and FUV luminosity L_FUV [erg s^-1]. */
typedef struct {
  double x_cm, y_cm, z_cm;
  double Q;
  double L_FUV;
} ism_source;

/* Point-source radiation by long characteristics: the many-ray limit of the ray tracing of
 * Sec. 5.1 (Eq. e:Erad) at cell centres.  For every cell and source, the straight segment
 * from the source to the cell centre gives the exact columns N_H, N_H2, N_C (sums of field x
 * length over the cells it crosses, in double), and the source adds
 *   chi_PE += chi_s exp(-sigma_PE N_H), chi_LW += chi_s exp(-sigma_LW N_H)   (sigma x Z'_d),
 *   chi_H2 += that LW term x f_shld,H2(N_H2)  (Eqs. e:chi_H2, e:fshld_H2_DB),
 *   chi_C  += that LW term x f_shld,C(N_C, N_H2),
 *   phi_LyC += Q exp(-sigma_LyC N_H) / (4 pi r^2) inside R_St = (3Q / (4 pi alpha_B(1e4 K)))^(1/3)
 *              (mean density 1 cm^-3), 0 beyond,
 * with chi_s = L_FUV / (16 pi^2 r^2 J^D_FUV) (Eq. e:chi_FUV; both bands get the same
 * normalised intensity) and r at least half a cell.  In: n, xH2 (double), xC (double or
 * NULL = 0); in/out: the five radiation arrays (double for F64, float for MIXED) -- the
 * contributions are added, so six-ray fields or other sources may already be there.
 * src is a host array of nsrc <= 256 sources, copied synchronously; calls on one device
 * must not overlap in time. */
ism_status ism_point_sources(const ism_grid *g, const ism_params *p, ism_precision prec,
                             int32_t nsrc, const ism_source *src, const double *n,
                             const double *xH2, const double *xC, void *chi_PE, void *chi_LW,
                             void *chi_H2, void *chi_C, void *phi_LyC, hipStream_t stream);

/* Options of the adaptive ray tracing (Sec. 5.1): packets start at HEALPix level level0
 * (12 4^level0 per source), split into four down to max_level (<= 13) while fewer than
 * rays_per_cell rays of a level would cross a cell, and stop once the optical depth from the
 * source exceeds tau_max in every band.  The paper's values: 4, (unbounded), 4, 30. */
typedef struct {
  int32_t level0;
  int32_t max_level;
  double rays_per_cell;
  double tau_max;
} ism_art_options;

/* Point-source radiation by adaptive ray tracing (Sec. 5.1, Eqs. e:Erad, e:Erad_H2, e:chi_H2).
 * Each source emits photon packets along the HEALPix directions (Gorski et al. 2005, nested
 * numbering); a packet crossing a cell over ds deposits, per band, L_in (1 - exp(-alpha ds)) /
 * alpha with L_in = L exp(-tau) / N_ray(level), tau from the source to the entry face:
 *   PE, LW: alpha = n sigma_d Z'_d, L = L_FUV, deposit / (4 pi dV J^D_FUV) added to chi_PE,
 *           chi_LW; the LW deposit times f_shld,H2(N_H2) to chi_H2 and times f_shld,C(N_C, N_H2)
 *           to chi_C, columns to the middle of the segment;
 *   LyC:    alpha = n (x_HI sigma_pi,H + x_H2 sigma_pi,H2 + Z'_d sigma_d,LyC),
 *           x_HI = max(0, 1 - 2 x_H2 - x_H+), L = Q, deposit / dV added to phi_LyC (photons
 *           cm^-2 s^-1).
 * A packet is split into its four children (same distance r, own directions, same columns)
 * before entering a cell where N_ray dx^2 / (4 pi r^2) < rays_per_cell, dropped where every
 * band's tau > tau_max, and lost through the grid faces (all open).
 * In: n, xH2, xHp (double, [nz][ny][nx], at most 2^31 - 1 cells), xC (double or NULL = 0);
 * src: host array of nsrc <= 256 sources inside the grid; opt: NULL for the defaults
 * {4, 13, 4.0, 30.0}.
 * In/out: the five radiation arrays (double for F64, float for MIXED): contributions are
 * added (atomically, so the last bits vary between runs).  flux: NULL, or 9 arrays of ncell
 * (the path's precision; band-major PE, LW, LyC, then x, y, z; component k of cell i at
 * flux + k * ncell + i) to which the flux vectors of Eq. e:Frad, F_j = sum dL_j n / alpha_j /
 * dV with n the packet's direction, are added: PE and LW as band energy fluxes in
 * erg cm^-2 s^-1 (a packet's L_FUV shared as J^D_PE : J^D_LW, the Draine field's shares), LyC
 * as a photon flux in photons cm^-2 s^-1.  budget: NULL, or a device array of
 * nsrc x 6 doubles that receives per source the luminosity lost through the faces (PE, LW in
 * erg s^-1, LyC in photons s^-1) and then the luminosity dropped at tau > tau_max.
 * The call returns when the work is done: it reads the number of packets of each level back
 * to the host.  The packet lists are scratch of the call's stream (48 bytes a packet; a level
 * may hold up to 4x the previous one); the sources sit in constant memory, so calls on one
 * device must not overlap in time.  ISM_E_NOMEM when a list cannot grow. */
ism_status ism_ray_trace(const ism_grid *g, const ism_params *p, ism_precision prec, int32_t nsrc,
                         const ism_source *src, const ism_art_options *opt, const double *n,
                         const double *xH2, const double *xHp, const double *xC, void *chi_PE,
                         void *chi_LW, void *chi_H2, void *chi_C, void *phi_LyC, void *flux,
                         double *budget, hipStream_t stream);

typedef struct {
  double T_destroy_K;     /* grains destroyed above this gas temperature (1e6) */
  double prad_ratio_max;  /* ... or where |F| / c exceeds this multiple of 2 n k_B T (50) */
} ism_force_options;

/* Radiation force per volume on the gas-dust mixture (Sec. 6.2): f = sum_j alpha_j F_j / c
 * over the traced bands with the opacities of ism_ray_trace (PE, LW: dust; LyC: dust, H and
 * H2), h nu_LyC per LyC photon.  Grain destruction (appendix on grain destruction): where
 * T > T_destroy_K or P_rad = |F_PE + F_LW + h nu F_LyC| / c > prad_ratio_max x 2 n k_B T
 * the dust part of every band is dropped and only LyC photoionisation of H and H2 pushes.
 * In: n, T, xH2, xHp (double, ncell each), flux (9 x ncell, the layout and precision that
 * ism_ray_trace writes); opt: NULL for {1e6, 50} (an infinite value turns a test off).
 * Out: f_rad (3 x ncell, the path's precision, dyn cm^-3: x, y, z at f_rad + q * ncell + i);
 * dust_off: NULL or ncell bytes, 1 where the grains count as destroyed.
 * Source-term update (optional): mom, NULL or 3 x ncell doubles of momentum density
 * (g cm^-2 s^-1, in/out), receives f dt_s; etot, NULL or ncell doubles of total energy
 * density (erg cm^-3, in/out, needs mom), receives the change of rho v^2 / 2 at
 * rho = mu_H m_H n (cells with n = 0 unchanged).  Arithmetic in double on both paths.
 * ISM_E_ARG for NULL required arrays, ncell outside [0, 2^32 - 256], NaN or non-positive
 * thresholds, dt_s negative or not finite, etot without mom. */
ism_status ism_radiation_force(const ism_params *p, ism_precision prec, int64_t ncell,
                               const double *n, const double *T, const double *xH2,
                               const double *xHp, const void *flux, const ism_force_options *opt,
                               void *f_rad, uint8_t *dust_off, double dt_s, double *mom,
                               double *etot, hipStream_t stream);

/* Per-cell diagnostics of the microphysics at the given state (Secs. 3-4): every rate
 * coefficient, heating and cooling term, T_d, the equilibrium x_C+, x_CO, x_e, the
 * net volumetric rate H = n Gamma - n^2 Lambda and C_H2, C_H+ (Eqs. e:HH, e:HII,
 * e:ODE1).  `out` is SoA: diagnostic k of cell i at out[k * ncell + i], ism_ndiag()
 * arrays of double (F64) or float (MIXED).  Radiation inputs as for the step;
 * phi_LyC may be NULL (= 0). */
ism_status ism_rates(const ism_params *p, ism_precision prec, int64_t ncell,
                     const double *n, const double *T, const double *xH2, const double *xHp,
                     const void *chi_PE, const void *chi_LW, const void *chi_H2, const void *chi_C,
                     const void *phi_LyC, const void *xi_cr, const void *N_eff,
                     void *out, hipStream_t stream);

/* The subcycled heating/cooling + chemistry source step (Sec. 6.1, Eqs. e:ODE1,
 * e:ODE2): advances every cell by dt_s with n and radiation fixed.  Per substep:
 * dt_sub = min(dt - t, eps e/|H|, eps/|C_H2|, eps/|C_H+|); semi-implicit T_mu update
 * with a forward-difference dH/dT_mu; backward-Euler update of (x_H2, x_H+) with rate
 * coefficients at the new temperature; equilibrium C/O/e closure (Secs. 3.2-3.3).
 * In/out: T, xH2, xHp (double).  In: n (double) and radiation (precision as above;
 * phi_LyC may be NULL = 0).  Optional outputs (NULL to skip): xCp, xCO, xe, nsub
 * (int32 substeps taken; with order_cells = 2 its entry values are also read, as the
 * ordering key, so it must then hold initialised counts), status (uint8 bits above).
 * F64 evaluates everything in
 * double; MIXED evaluates rates, heating, cooling and the closure in float and keeps
 * the net H, the T update and the abundance update in double. */
ism_status ism_chem_cool_step(const ism_params *p, ism_precision prec, int64_t ncell, double dt_s,
                              const double *n, double *T, double *xH2, double *xHp,
                              const void *chi_PE, const void *chi_LW, const void *chi_H2,
                              const void *chi_C, const void *phi_LyC, const void *xi_cr,
                              const void *N_eff, void *xCp, void *xCO, void *xe,
                              int32_t *nsub, uint8_t *status, hipStream_t stream);

/* ism_chem_cool_step for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments, results and
 * errors as ism_chem_cool_step, but the call allocates nothing: its scratch (work-queue counter
 * and cell-ordering keys) is a fixed ISM_NOALLOC_SCRATCH_BYTES array per device, created with
 * the library's code object and held until the process ends.  Every call on one device shares
 * that array, so calls that overlap in time on one device race (serialise them, e.g. one
 * stream).  Limit: with order_cells 1 or 2 ncell <= ISM_NOALLOC_MAX_ORDERED_CELLS (ISM_E_ARG
 * beyond); with order_cells 0 any ncell. */
#define ISM_NOALLOC_SCRATCH_BYTES (64u << 20)
#define ISM_NOALLOC_MAX_ORDERED_CELLS (1 << 23)
ism_status ism_chem_cool_step_noalloc(const ism_params *p, ism_precision prec, int64_t ncell,
                                      double dt_s, const double *n, double *T, double *xH2,
                                      double *xHp, const void *chi_PE, const void *chi_LW,
                                      const void *chi_H2, const void *chi_C, const void *phi_LyC,
                                      const void *xi_cr, const void *N_eff, void *xCp, void *xCO,
                                      void *xe, int32_t *nsub, uint8_t *status, hipStream_t stream);

/* ---------------------------------------------------------------- learned surrogate
 * A small MLP maps a cell's (state, radiation, dt) to its post-step (x_H2, x_H+, log10 T):
 * 10 inputs -> 128 -> 128 -> 128 -> 3 outputs, SiLU on the hidden layers.  The products
 * run on the matrix cores with BF16 operands (weights, layer inputs and, backward, the
 * error signal) and FP32 accumulation; the master weights and the Adam moments are FP32.
 * The surrogate is not part of the paper's method: the plain step above is its teacher,
 * its fallback and the reference its results are checked against.
 *
 * Parameters (flat FP32, ISM_SURR_NPARAM values, row-major W[out][in]):
 *   W1[128x10] b1[128] W2[128x128] b2[128] W3[128x128] b3[128] W4[3x128] b4[3].
 * Inputs are standardised inside the library, x_s = (x - mu_x) / sd_x, and outputs are
 * returned as y = y_s sd_y + mu_y; the loss is the mean over samples and the 3 outputs of
 * (y_s - (y_target - mu_y) / sd_y)^2.  Adam: beta1 0.9, beta2 0.999, eps 1e-8, bias
 * corrected, one step counter per surrogate.
 *
 * The object owns its device buffers on the device that was current at create; every
 * other call must be made with that device current.  Calls on one object are ordered by
 * the stream they are given; two streams using one object concurrently race. */
#define ISM_SURR_NIN 10
#define ISM_SURR_NOUT 3
#define ISM_SURR_NPARAM 34819
/* Checkpoint layout of get/set_params (floats): theta[NPARAM], adam_m[NPARAM],
 * adam_v[NPARAM], step, mu_x[10], sd_x[10], mu_y[3], sd_y[3]. */
#define ISM_SURR_STATE_FLOATS (3 * ISM_SURR_NPARAM + 1 + 26)

typedef struct ism_surrogate ism_surrogate;

/* Allocate a surrogate: He-uniform weights (bound sqrt(6/fan_in)) drawn from a counter-based
 * generator keyed by `seed`, zero biases, zero moments, identity standardisation.
 * Requires ism_init on the current device. */
ism_status ism_surrogate_create(ism_surrogate **out, uint64_t seed);
ism_status ism_surrogate_destroy(ism_surrogate *m);

/* Host arrays; sd values must be finite and > 0.  Held on the host and passed with every
 * later launch (no device work, no synchronisation). */
ism_status ism_surrogate_set_norm(ism_surrogate *m, const float *mu_x, const float *sd_x,
                                  const float *mu_y, const float *sd_y);

/* Inference: X [B][10] raw inputs -> Y [B][3] (device FP32, caller-owned).  B >= 0. */
ism_status ism_surrogate_forward(ism_surrogate *m, const float *X, float *Y, int64_t B,
                                 hipStream_t stream);

/* Gradient of sum_{b,o} dY[b][o] * y_s[b][o] with respect to the parameters, where y_s is
 * the standardised output: X [B][10], dY [B][3], grad [ISM_SURR_NPARAM] (device FP32,
 * caller-owned, overwritten).  B >= 1. */
ism_status ism_surrogate_backward(ism_surrogate *m, const float *X, const float *dY,
                                  float *grad, int64_t B, hipStream_t stream);

/* One training step on a batch: forward, MSE loss against Y [B][3] (raw targets),
 * backward, Adam with learning rate lr.  loss_dev (device float, nullable) receives the
 * batch loss before the update.  B >= 1, lr finite and >= 0. */
ism_status ism_surrogate_train_step(ism_surrogate *m, const float *X, const float *Y, int64_t B,
                                    float lr, float *loss_dev, hipStream_t stream);

/* Host checkpoint of the whole training state (layout above).  get copies on `stream` and
 * waits for that stream (the one synchronising call of the surrogate); set stages the host
 * values in the object's pinned buffer (waiting only for the previous set's copy out of it),
 * then copies and rebuilds the BF16 weight images on `stream`, without waiting. */
ism_status ism_surrogate_get_params(const ism_surrogate *m, float *flat, hipStream_t stream);
ism_status ism_surrogate_set_params(ism_surrogate *m, const float *flat, hipStream_t stream);

/* Training pairs for the surrogate: X [ncell][10] network inputs from the pre-step state
 * (n, T0, xH2_0, xHp_0), radiation (chi_PE, phi_LyC (nullable = 0), xi_cr, N_eff; double for
 * F64, float for MIXED), Z'_g and dt; Y [ncell][3] targets (x_H2, x_H+, log10 T) from the
 * post-step state (T1, xH2_1, xHp_1), skipped when Y is NULL.  Inputs, in order:
 * log10 n, log10 T, log10 max(chi_PE, 1e-10), log10 max(phi_LyC, 1), log10 max(xi_cr, 1e-30),
 * log10 Z'_g, x_H2, x_H+, log10 max(N_eff, 1e17 cm^-2), log10(dt / 1 yr).  dt_s > 0. */
ism_status ism_surrogate_pairs(const ism_params *p, ism_precision prec, int64_t ncell, double dt_s,
                               const double *n, const double *T0, const double *xH2_0,
                               const double *xHp_0, const void *chi_PE, const void *phi_LyC,
                               const void *xi_cr, const void *N_eff, const double *T1,
                               const double *xH2_1, const double *xHp_1, float *X, float *Y,
                               hipStream_t stream);

/* The source step with the surrogate in front of the plain solver (MIXED precision only:
 * radiation and x_C+, x_CO, x_e float).  Arguments as for ism_chem_cool_step.
 * A cell can stand in for the plain subcycled step (Sec. 6.1) only where that step's result no
 * longer depends on its substep path, so every cell first takes a pre-test at its input state:
 * both chemical relaxation rates fast, dt (2 k_gr n + D_H2) >= 10 and dt (I_H + R_H+) >= 10
 * (Eqs. e:HH, e:HII), and the thermal one too, -dt (dH/dT_mu) / K >= 10 (the forward difference
 * of Sec. 6.1, K = n mu_H k_B / (gamma - 1)).  For the cells that pass, the network predicts the
 * post-step (x_H2, x_H+, T), and the prediction seeds a Newton solve for the equilibrium of
 * (dT/dt, C_H2, C_H+) (Eqs. e:ODE1, e:HH, e:HII; Jacobian by forward differences).  The root is
 * accepted only where: Newton converged to accept_tol (relative); every eigenvalue of the
 * Jacobian at the root has real part below -20/dt; the root's T is within a factor e^0.1 of the
 * prediction; dT/dt keeps the sign of T_root - T along four temperatures from T to T_root; and
 * one plain substep of length dt, started at the root and at the root perturbed in each
 * variable, bounds the plain step's own end state to within accept_tol / 2 of the root.
 * Accepted cells return the root with equilibrium C/O/e there, nsub = 0, status = 0; every
 * other cell runs the plain MIXED step (ordered by temperature with order_cells 1 or 2) and has
 * ISM_ST_FALLBACK set; its outputs are those of ism_chem_cool_step(MIXED).  m may be NULL: the
 * seed is then the input state itself (the method without the network).  n_fallback_dev
 * (device int64, nullable) receives the number of plain-step cells.  accept_tol in (0, 1e-3];
 * ncell < 2^31.  Scratch (the candidate and fallback lists, predictions, ordering keys) on the
 * call's stream. */
ism_status ism_chem_cool_step_surrogate(ism_surrogate *m, const ism_params *p, int64_t ncell,
                                        double dt_s, const double *n, double *T, double *xH2,
                                        double *xHp, const void *chi_PE, const void *chi_LW,
                                        const void *chi_H2, const void *chi_C, const void *phi_LyC,
                                        const void *xi_cr, const void *N_eff, void *xCp, void *xCO,
                                        void *xe, int32_t *nsub, uint8_t *status, double accept_tol,
                                        int64_t *n_fallback_dev, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* ISM_H */
