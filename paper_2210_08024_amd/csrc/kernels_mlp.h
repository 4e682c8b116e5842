// Surrogate MLP on the CDNA4 matrix cores: 10 -> 128 -> 128 -> 128 -> 3, SiLU on the hidden
// layers, linear output.  Products take BF16 operands (weights, layer inputs and, backward, the
// error signal) and accumulate in FP32; master weights and Adam moments stay FP32.
//
// Formulation.  Every layer is computed transposed, Z^T = W * H^T: the weights are the MFMA A
// operand (rows = output neurons) and the samples run along the B/D column index.  A 16x16 MFMA
// result then leaves lane l holding output neurons 4(l/16)+j (j = 0..3) of sample l%16, which is
// already the lane layout of the next product's B operand (k index = neuron) -- no LDS transpose
// between layers.  The 16x16x32 instruction takes eight k values per lane; pairing the D tiles of
// neuron blocks 2s and 2s+1 gives lane group g the neurons {32s+4g+j} and {32s+16+4g+j}, so the
// weight image stores each row's columns in that same order (A and B only have to agree on the
// k order), and XOR-swizzles 16-byte chunks by row so the A-fragment reads are conflict-free.
//
// Parameter vector (flat FP32, 34,819 values): W1[128x10] b1 W2[128x128] b2 W3[128x128] b3
// W4[3x128] b4, W row-major [out][in].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ism {
namespace mlp {

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) short i16x4;
typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;

constexpr int NIN = 10, NH = 128, NOUT = 3, K1 = 16;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NH, OFF_W4 = OFF_B3 + NH,
              OFF_B4 = OFF_W4 + NOUT * NH, NPARAM = OFF_B4 + NOUT;
static_assert(NPARAM == 34819, "parameter count");

// Forward weight image (bytes), copied verbatim into LDS by the forward kernel.
constexpr int FI_W1 = 0;                      // [128][16] bf16, plain (cols 10..15 zero)
constexpr int FI_W2 = FI_W1 + NH * K1 * 2;    // [128][128] bf16, permuted + swizzled
constexpr int FI_W3 = FI_W2 + NH * NH * 2;
constexpr int FI_W4 = FI_W3 + NH * NH * 2;    // [16][128] bf16 (rows 3..15 zero)
constexpr int FI_B = FI_W4 + 16 * NH * 2;     // fp32 b1[128] b2[128] b3[128] b4[16]
constexpr int FI_BYTES = FI_B + (3 * NH + 16) * 4;
// Backward (transposed) weight image: A operands of the dX products.
constexpr int BI_W4T = 0;                     // [128][16] bf16: W4T[i][o] = W4[o][i], o >= 3 zero
constexpr int BI_W3T = BI_W4T + NH * 16 * 2;  // [128][128] bf16 W3^T, permuted + swizzled
constexpr int BI_W2T = BI_W3T + NH * NH * 2;
constexpr int BI_BYTES = BI_W2T + NH * NH * 2;
static_assert(FI_BYTES % 16 == 0 && BI_BYTES % 16 == 0, "image sizes");

// Standardisation block (device, fp32): mu_x[10] isd_x[10] mu_y[3] sd_y[3] isd_y[3].
constexpr int NRM_MUX = 0, NRM_ISDX = 10, NRM_MUY = 20, NRM_SDY = 23, NRM_ISDY = 26, NRM_FLOATS = 32;

// Position of logical column c (0..127) inside a permuted, swizzled 128-wide row r.
__host__ __device__ __forceinline__ int perm_pos(int r, int c) {
  const int s = c >> 5, w = c & 31;
  const int hi = w >> 4, g = (w & 15) >> 2, j = (w & 3) + 4 * hi;
  return ((((s << 2) + g) ^ (r & 15)) << 3) + j;
}

__device__ __forceinline__ float sigmoid_f(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

__device__ __forceinline__ i16x4 as_i16x4(bf16x4 v) { return __builtin_bit_cast(i16x4, v); }

__device__ __forceinline__ bf16x8 cat8(bf16x4 a, bf16x4 b) {
  return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// A per-iteration zero the compiler cannot see through: indexing LDS with it keeps the weight
// fragment loads inside the sample-tile loop instead of hoisting all of them into registers.
__device__ __forceinline__ int opaque_zero() {
  int z = 0;
  asm volatile("" : "+v"(z));
  return z;
}

constexpr int FWD_THREADS = 512, FWD_WAVES = FWD_THREADS / 64, NT = 4, WTILE = 16 * NT;

// Network inputs built from a cell's state, radiation and the step length (float logs):
//   0 log10 n, 1 log10 T, 2 log10 max(chi_PE, 1e-10), 3 log10 max(phi_LyC, 1),
//   4 log10 max(xi_cr, 1e-30), 5 log10 Z'_g, 6 x_H2, 7 x_H+, 8 log10 max(N_eff, 1e17),
//   9 log10 (dt / yr).  Outputs: post-step x_H2, x_H+, log10 T.
template <class R>
struct CellIn {
  const double *n, *T, *xH2, *xHp;
  const R *chiPE, *phi, *xi, *Neff;  // phi may be null (= 0)
  float lZg, ldt;
  const int32_t *idx;  // sample -> cell, or null (sample = cell)
};

template <class R>
__device__ __forceinline__ float cell_feature(const CellIn<R> &c, int64_t i, int k) {
  switch (k) {
    case 0: return log10f((float)c.n[i]);
    case 1: return log10f((float)c.T[i]);
    case 2: return log10f(fmaxf((float)c.chiPE[i], 1e-10f));
    case 3: return log10f(fmaxf(c.phi ? (float)c.phi[i] : 0.f, 1.f));
    case 4: return log10f(fmaxf((float)c.xi[i], 1e-30f));
    case 5: return c.lZg;
    case 6: return (float)c.xH2[i];
    case 7: return (float)c.xHp[i];
    case 8: return log10f(fmaxf((float)c.Neff[i], 1e17f));
    case 9: return c.ldt;
    default: return 0.f;
  }
}

// Standardisation of inputs and outputs, passed by value with each launch (NRM_* offsets).
struct Norm {
  float v[NRM_FLOATS];
};

struct FwdArgs {
  const float *X;  // [B][10] raw features (modes 0-2)
  CellIn<float> cin;  // mode 3: features built from the cell arrays
  int64_t B;
  const unsigned long long *count;  // mode 3: device sample count (<= B), or null (= B)
  const uint8_t *fimg;
  Norm norm;
  float *Y;        // modes 0, 3: [B][3] de-standardised predictions
  const float *Yt; // mode 2: [B][3] raw targets
  float dscale;    // mode 2: 2 / (3B)
  float *d4;       // mode 2: [B][3] dL/dy (standardised outputs)
  float *loss_part;  // mode 2: one partial sum of squared errors per wave of the grid
  uint16_t *h0;    // modes 1, 2: [B][16] bf16 standardised input
  float *z1, *z2, *z3;        // modes 1, 2: [B][128] pre-activations
  uint16_t *h1, *h2, *h3;     // modes 1, 2: [B][128] bf16 activations
};

// One hidden layer on a wave's NT sample tiles: hout = bf16(silu(W hin + b)).
template <int MODE>
__device__ __forceinline__ void fwd_hidden(const __bf16 *W, const float *b, const bf16x4 (&hin)[8][NT],
                                           bf16x4 (&hout)[8][NT], int r, int g, int64_t base, int64_t B,
                                           float *zst, uint16_t *hst) {
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const __bf16 *row = W + (16 * m + r) * NH;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bf16x8 w = *(const bf16x8 *)(row + ((((s << 2) + g) ^ r) << 3));
#pragma unroll
      for (int t = 0; t < NT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, cat8(hin[2 * s][t], hin[2 * s + 1][t]), acc[t],
                                                         0, 0, 0);
    }
    const f32x4 bb = *(const f32x4 *)(b + 16 * m + 4 * g);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const f32x4 z = acc[t] + bb;
      bf16x4 h;
      h.x = (__bf16)(z.x * sigmoid_f(z.x));
      h.y = (__bf16)(z.y * sigmoid_f(z.y));
      h.z = (__bf16)(z.z * sigmoid_f(z.z));
      h.w = (__bf16)(z.w * sigmoid_f(z.w));
      hout[m][t] = h;
      if (MODE == 1 || MODE == 2) {
        const int64_t n = base + 16 * t + r;
        if (n < B) {
          *(f32x4 *)(zst + n * NH + 16 * m + 4 * g) = z;
          *(bf16x4 *)(hst + n * NH + 16 * m + 4 * g) = h;
        }
      }
    }
  }
}

// MODE 0: inference (Y).  MODE 1: store activations for a backward pass.  MODE 2: also the loss
// against targets Yt and the output error signal d4.  MODE 3: inference on inputs built from
// cell arrays (CellIn).
template <int MODE>
__global__ __launch_bounds__(FWD_THREADS) void mlp_fwd_kernel(FwdArgs a) {
  __shared__ __align__(16) uint8_t smem[FI_BYTES];
  for (int i = threadIdx.x; i < FI_BYTES / 16; i += FWD_THREADS)
    ((uint4 *)smem)[i] = ((const uint4 *)a.fimg)[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  float mux[4], isdx[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = 4 * g + j;
    mux[j] = k < NIN ? a.norm.v[NRM_MUX + k] : 0.f;
    isdx[j] = k < NIN ? a.norm.v[NRM_ISDX + k] : 0.f;
  }
  float lossacc = 0.f;
  int64_t B = a.B;
  if (MODE == 3 && a.count) B = (int64_t)*a.count < B ? (int64_t)*a.count : B;
  const int64_t stride = (int64_t)gridDim.x * FWD_WAVES * WTILE;
  for (int64_t base = ((int64_t)wave * gridDim.x + blockIdx.x) * WTILE; base < B; base += stride) {
    const uint8_t *sm = smem + opaque_zero();
    const __bf16 *W1 = (const __bf16 *)(sm + FI_W1);
    const __bf16 *W2 = (const __bf16 *)(sm + FI_W2);
    const __bf16 *W3 = (const __bf16 *)(sm + FI_W3);
    const __bf16 *W4 = (const __bf16 *)(sm + FI_W4);
    const float *bias = (const float *)(sm + FI_B);
    i16x4 x[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int64_t n = base + 16 * t + r;
      const int64_t cn = (MODE == 3 && a.cin.idx && n < B) ? (int64_t)a.cin.idx[n] : n;
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 4 * g + j;
        float raw = 0.f;
        if (n < B && k < NIN) raw = MODE == 3 ? cell_feature(a.cin, cn, k) : a.X[n * NIN + k];
        v[j] = (n < B && k < NIN) ? (raw - mux[j]) * isdx[j] : 0.f;
      }
      bf16x4 h;
      h.x = (__bf16)v[0];
      h.y = (__bf16)v[1];
      h.z = (__bf16)v[2];
      h.w = (__bf16)v[3];
      x[t] = as_i16x4(h);
      if ((MODE == 1 || MODE == 2) && n < B) *(bf16x4 *)(a.h0 + n * K1 + 4 * g) = h;
    }
    bf16x4 ha[8][NT], hb[8][NT];
    // layer 1 (K = 16, one 16x16x16 product per neuron block)
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const i16x4 w = *(const i16x4 *)(W1 + (16 * m + r) * K1 + 4 * g);
      const f32x4 bb = *(const f32x4 *)(bias + 16 * m + 4 * g);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const f32x4 z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w, x[t], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0) + bb;
        bf16x4 h;
        h.x = (__bf16)(z.x * sigmoid_f(z.x));
        h.y = (__bf16)(z.y * sigmoid_f(z.y));
        h.z = (__bf16)(z.z * sigmoid_f(z.z));
        h.w = (__bf16)(z.w * sigmoid_f(z.w));
        ha[m][t] = h;
        if (MODE == 1 || MODE == 2) {
          const int64_t n = base + 16 * t + r;
          if (n < B) {
            *(f32x4 *)(a.z1 + n * NH + 16 * m + 4 * g) = z;
            *(bf16x4 *)(a.h1 + n * NH + 16 * m + 4 * g) = h;
          }
        }
      }
    }
    fwd_hidden<MODE>(W2, bias + NH, ha, hb, r, g, base, B, a.z2, a.h2);
    fwd_hidden<MODE>(W3, bias + 2 * NH, hb, ha, r, g, base, B, a.z3, a.h3);
    // output layer: rows 0..2 of a 16-row tile
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bf16x8 w = *(const bf16x8 *)(W4 + r * NH + ((((s << 2) + g) ^ r) << 3));
#pragma unroll
      for (int t = 0; t < NT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, cat8(ha[2 * s][t], ha[2 * s + 1][t]), acc[t], 0, 0, 0);
    }
    if (g == 0) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int64_t n = base + 16 * t + r;
        if (n < B) {
#pragma unroll
          for (int j = 0; j < NOUT; ++j) {
            const float y = acc[t][j] + bias[3 * NH + j];
            if (MODE == 0 || MODE == 3) a.Y[n * NOUT + j] = y * a.norm.v[NRM_SDY + j] + a.norm.v[NRM_MUY + j];
            if (MODE == 2) {
              const float e = y - (a.Yt[n * NOUT + j] - a.norm.v[NRM_MUY + j]) * a.norm.v[NRM_ISDY + j];
              a.d4[n * NOUT + j] = e * a.dscale;
              lossacc += e * e;
            }
          }
        }
      }
    }
  }
  if (MODE == 2) {
    lossacc = wave_sum(lossacc);
    if (lane == 0) a.loss_part[blockIdx.x * FWD_WAVES + wave] = lossacc;
  }
}

struct BwdArgs {
  int64_t B;
  const uint8_t *bimg;
  const float *d4;          // [B][3] dL/dy
  float *z1, *z2, *z3;      // in: pre-activations; out: dL/dz of the same layer (in place)
};

// d = (W^T bf16(dnext)) * silu'(z) for one hidden layer, stored over z; dout = bf16(d).
__device__ __forceinline__ void bwd_finish(const f32x4 &acc, float *zd, int64_t n, int64_t B, int m, int g,
                                           bf16x4 &dout) {
  f32x4 z = f32x4{0.f, 0.f, 0.f, 0.f};
  float *p = zd + n * NH + 16 * m + 4 * g;
  if (n < B) z = *(const f32x4 *)p;
  f32x4 d;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float s = sigmoid_f(z[j]);
    d[j] = acc[j] * (s * (1.f + z[j] * (1.f - s)));
  }
  if (n < B) *(f32x4 *)p = d;
  dout.x = (__bf16)d.x;
  dout.y = (__bf16)d.y;
  dout.z = (__bf16)d.z;
  dout.w = (__bf16)d.w;
}

__device__ __forceinline__ void bwd_hidden(const __bf16 *Wt, const bf16x4 (&din)[8][NT], bf16x4 (&dout)[8][NT],
                                           float *zd, int r, int g, int64_t base, int64_t B) {
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    f32x4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const __bf16 *row = Wt + (16 * m + r) * NH;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bf16x8 w = *(const bf16x8 *)(row + ((((s << 2) + g) ^ r) << 3));
#pragma unroll
      for (int t = 0; t < NT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, cat8(din[2 * s][t], din[2 * s + 1][t]), acc[t],
                                                         0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) bwd_finish(acc[t], zd, base + 16 * t + r, B, m, g, dout[m][t]);
  }
}

// Error signal back through layers 4, 3, 2 (the input layer needs no dX).
__global__ __launch_bounds__(FWD_THREADS) void mlp_bwd_kernel(BwdArgs a) {
  __shared__ __align__(16) uint8_t smem[BI_BYTES];
  for (int i = threadIdx.x; i < BI_BYTES / 16; i += FWD_THREADS)
    ((uint4 *)smem)[i] = ((const uint4 *)a.bimg)[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int64_t stride = (int64_t)gridDim.x * FWD_WAVES * WTILE;
  for (int64_t base = ((int64_t)wave * gridDim.x + blockIdx.x) * WTILE; base < a.B; base += stride) {
    const uint8_t *sm = smem + opaque_zero();
    const __bf16 *W4t = (const __bf16 *)(sm + BI_W4T);
    const __bf16 *W3t = (const __bf16 *)(sm + BI_W3T);
    const __bf16 *W2t = (const __bf16 *)(sm + BI_W2T);
    i16x4 dy[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int64_t n = base + 16 * t + r;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (g == 0 && n < a.B) {
#pragma unroll
        for (int j = 0; j < NOUT; ++j) v[j] = a.d4[n * NOUT + j];
      }
      bf16x4 h;
      h.x = (__bf16)v[0];
      h.y = (__bf16)v[1];
      h.z = (__bf16)v[2];
      h.w = (__bf16)v[3];
      dy[t] = as_i16x4(h);
    }
    bf16x4 da[8][NT], db[8][NT];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      const i16x4 w = *(const i16x4 *)(W4t + (16 * m + r) * 16 + 4 * g);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w, dy[t], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        bwd_finish(acc, a.z3, base + 16 * t + r, a.B, m, g, da[m][t]);
      }
    }
    bwd_hidden(W3t, da, db, a.z2, r, g, base, a.B);
    bwd_hidden(W2t, db, da, a.z1, r, g, base, a.B);
  }
}

constexpr int DW_THREADS = 256, DW_SUB = 64, DW_LROW = DW_SUB + 8;

struct DwArgs {
  int64_t B, chunk;
  const uint16_t *h0, *h1, *h2, *h3;  // layer inputs, bf16
  const float *d1, *d2, *d3, *d4;     // error signals dL/dz, fp32
  float *part;                        // [nchunk][NPARAM]
};

// Stage a 64-sample slice of a [B][WSRC] array into LDS as [feature][sample] bf16, features
// 0..ROWS-1 (zero beyond WSRC or past the chunk end).  Each thread takes a sample pair and
// ROWS/8 features; FP32 sources also accumulate the per-feature sums (bias gradient).
template <int ROWS, int WSRC, typename T>
__device__ __forceinline__ void dw_stage(__bf16 *dst, const T *src, int64_t s0, int64_t s1, float (&bsum)[ROWS / 8]) {
  const int p = threadIdx.x & 31, q = threadIdx.x >> 5;
  const int64_t na = s0 + 2 * p, nb = na + 1;
  constexpr int PER = ROWS / 8;
  typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
  constexpr bool VEC = WSRC == ROWS && PER % (16 / (int)sizeof(T)) == 0;
  if constexpr (VEC) {
    // the thread's PER features of a sample are contiguous (16-byte aligned): 16-byte loads
    constexpr int EPV = 16 / (int)sizeof(T), NV = PER / EPV;
    T ra[PER], rb[PER];
    const uint4 *pa = reinterpret_cast<const uint4 *>(src + na * WSRC + q * PER);
    const uint4 *pb = reinterpret_cast<const uint4 *>(src + nb * WSRC + q * PER);
#pragma unroll
    for (int w = 0; w < NV; ++w) {
      const uint4 xa = na < s1 ? pa[w] : make_uint4(0u, 0u, 0u, 0u);
      const uint4 xb = nb < s1 ? pb[w] : make_uint4(0u, 0u, 0u, 0u);
      __builtin_memcpy(ra + EPV * w, &xa, 16);
      __builtin_memcpy(rb + EPV * w, &xb, 16);
    }
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      bf16x2 v;
      if constexpr (sizeof(T) == 4) {
        bsum[e] += (float)ra[e] + (float)rb[e];
        v.x = (__bf16)(float)ra[e];
        v.y = (__bf16)(float)rb[e];
      } else {
        v.x = __builtin_bit_cast(__bf16, (uint16_t)ra[e]);
        v.y = __builtin_bit_cast(__bf16, (uint16_t)rb[e]);
      }
      *(bf16x2 *)(dst + (q * PER + e) * DW_LROW + 2 * p) = v;
    }
    return;
  }
#pragma unroll
  for (int e = 0; e < ROWS / 8; ++e) {
    const int f = q * (ROWS / 8) + e;
    __bf16 ba = (__bf16)0.f, bb = (__bf16)0.f;
    if (f < WSRC) {
      if constexpr (sizeof(T) == 4) {
        const float va = na < s1 ? (float)src[na * WSRC + f] : 0.f;
        const float vb = nb < s1 ? (float)src[nb * WSRC + f] : 0.f;
        bsum[e] += va + vb;
        ba = (__bf16)va;
        bb = (__bf16)vb;
      } else {
        if (na < s1) ba = __builtin_bit_cast(__bf16, (uint16_t)src[na * WSRC + f]);
        if (nb < s1) bb = __builtin_bit_cast(__bf16, (uint16_t)src[nb * WSRC + f]);
      }
    }
    bf16x2 v;
    v.x = ba;
    v.y = bb;
    *(bf16x2 *)(dst + f * DW_LROW + 2 * p) = v;
  }
}

// Partial dW = sum over the block's sample chunk of bf16(d)^T bf16(h), and db = sum of d.
// RD/RH: rows of the staged d / h slices (padded widths), WD/WH: source widths, OUTR/INR: the
// real layer shape.
template <int RD, int RH, int WD, int WH, int OUTR, int INR>
__device__ __forceinline__ void dw_layer(const DwArgs &a, const float *D, const uint16_t *H, int offw, int offb,
                                         __bf16 *sD, __bf16 *sH) {
  constexpr int TO = RD / 16, TI = RH / 16;
  constexpr int NO = TO >= 4 ? TO / 4 : 1, NI = TO >= 4 ? TI : TI / 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int ob0 = TO >= 4 ? wave * NO : 0, ib0 = TO >= 4 ? 0 : wave * NI;
  const int64_t s_begin = (int64_t)blockIdx.x * a.chunk;
  const int64_t s_end = s_begin + a.chunk < a.B ? s_begin + a.chunk : a.B;
  f32x4 acc[NO][NI];
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int k = 0; k < NI; ++k) acc[i][k] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum[RD / 8], hdummy[RH / 8];
#pragma unroll
  for (int e = 0; e < RD / 8; ++e) bsum[e] = 0.f;
  for (int64_t s0 = s_begin; s0 < s_end; s0 += DW_SUB) {
    __syncthreads();
    dw_stage<RD, WD>(sD, D, s0, s_end, bsum);
    dw_stage<RH, WH>(sH, H, s0, s_end, hdummy);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < DW_SUB / 32; ++ks) {
      bf16x8 av[NO], bv[NI];
#pragma unroll
      for (int i = 0; i < NO; ++i) av[i] = *(const bf16x8 *)(sD + (16 * (ob0 + i) + r) * DW_LROW + 32 * ks + 8 * g);
#pragma unroll
      for (int k = 0; k < NI; ++k) bv[k] = *(const bf16x8 *)(sH + (16 * (ib0 + k) + r) * DW_LROW + 32 * ks + 8 * g);
#pragma unroll
      for (int i = 0; i < NO; ++i)
#pragma unroll
        for (int k = 0; k < NI; ++k) acc[i][k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[k], acc[i][k], 0, 0, 0);
    }
  }
  float *part = a.part + (int64_t)blockIdx.x * NPARAM;
#pragma unroll
  for (int i = 0; i < NO; ++i)
#pragma unroll
    for (int k = 0; k < NI; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int o = 16 * (ob0 + i) + 4 * g + j, in = 16 * (ib0 + k) + r;
        if (o < OUTR && in < INR) part[offw + o * INR + in] = acc[i][k][j];
      }
  // bias: reduce the per-thread sums over the 32 lanes that share a feature group
  const int p = threadIdx.x & 31, q = threadIdx.x >> 5;
#pragma unroll
  for (int e = 0; e < RD / 8; ++e) {
    float v = bsum[e];
#pragma unroll
    for (int o = 16; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    const int f = q * (RD / 8) + e;
    if (p == 0 && f < OUTR) part[offb + f] = v;
  }
}

__global__ __launch_bounds__(DW_THREADS) void mlp_dw_kernel(DwArgs a) {
  __shared__ __align__(16) __bf16 sD[NH * DW_LROW];
  __shared__ __align__(16) __bf16 sH[NH * DW_LROW];
  switch (blockIdx.y) {
    case 0: dw_layer<NH, K1, NH, K1, NH, NIN>(a, a.d1, a.h0, OFF_W1, OFF_B1, sD, sH); break;
    case 1: dw_layer<NH, NH, NH, NH, NH, NH>(a, a.d2, a.h1, OFF_W2, OFF_B2, sD, sH); break;
    case 2: dw_layer<NH, NH, NH, NH, NH, NH>(a, a.d3, a.h2, OFF_W3, OFF_B3, sD, sH); break;
    default: dw_layer<16, NH, NOUT, NH, NOUT, NH>(a, a.d4, a.h3, OFF_W4, OFF_B4, sD, sH); break;
  }
}

// Write one master parameter into the BF16 forward/backward images (biases stay FP32).
__device__ __forceinline__ void put_param(int p, float val, uint8_t *fimg, uint8_t *bimg) {
  const __bf16 hv = (__bf16)val;
  __bf16 *fw = (__bf16 *)fimg;
  __bf16 *bw = (__bf16 *)bimg;
  float *fb = (float *)(fimg + FI_B);
  if (p < OFF_B1) {
    const int o = p / NIN, i = p % NIN;
    fw[FI_W1 / 2 + o * K1 + i] = hv;
  } else if (p < OFF_W2) {
    fb[p - OFF_B1] = val;
  } else if (p < OFF_B2) {
    const int q = p - OFF_W2, o = q / NH, i = q % NH;
    fw[FI_W2 / 2 + o * NH + perm_pos(o, i)] = hv;
    bw[BI_W2T / 2 + i * NH + perm_pos(i, o)] = hv;
  } else if (p < OFF_W3) {
    fb[NH + p - OFF_B2] = val;
  } else if (p < OFF_B3) {
    const int q = p - OFF_W3, o = q / NH, i = q % NH;
    fw[FI_W3 / 2 + o * NH + perm_pos(o, i)] = hv;
    bw[BI_W3T / 2 + i * NH + perm_pos(i, o)] = hv;
  } else if (p < OFF_W4) {
    fb[2 * NH + p - OFF_B3] = val;
  } else if (p < OFF_B4) {
    const int q = p - OFF_W4, o = q / NH, i = q % NH;
    fw[FI_W4 / 2 + o * NH + perm_pos(o, i)] = hv;
    bw[BI_W4T / 2 + i * 16 + o] = hv;
  } else {
    fb[3 * NH + p - OFF_B4] = val;
  }
}

// Training pairs: inputs from a cell's pre-step state, targets from its post-step state.
template <class R>
__global__ void mlp_pairs_kernel(CellIn<R> c, int64_t N, const double *T1, const double *xH2_1,
                                 const double *xHp_1, float *X, float *Y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
#pragma unroll
  for (int k = 0; k < NIN; ++k) X[i * NIN + k] = cell_feature(c, i, k);
  if (Y) {
    Y[i * NOUT + 0] = (float)xH2_1[i];
    Y[i * NOUT + 1] = (float)xHp_1[i];
    Y[i * NOUT + 2] = log10f((float)T1[i]);
  }
}

__global__ void mlp_pack_kernel(const float *theta, uint8_t *fimg, uint8_t *bimg) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NPARAM) put_param(p, theta[p], fimg, bimg);
}

struct AdamArgs {
  const float *part;
  int nchunk;
  float *grad;   // gradient output when adam == 0
  float *theta, *m, *v;
  uint8_t *fimg, *bimg;
  float lr, b1, b2, eps, bc1, bc2;
  int adam;
};

// Sum the per-chunk partial gradients: four threads per parameter each take every fourth
// chunk, and the four sums are added in a fixed order (the result is the same on every run);
// then either store the gradient or take one Adam step on the FP32 master parameter and
// refresh its BF16 image entries.  Blocks of 256 threads cover 64 parameters.
constexpr int RA_PARAMS = 64;
__global__ __launch_bounds__(256) void mlp_reduce_adam_kernel(AdamArgs a) {
  __shared__ float s[256];
  const int t = threadIdx.x, j = t & (RA_PARAMS - 1), q = t / RA_PARAMS;
  const int p = blockIdx.x * RA_PARAMS + j;
  float part = 0.f;
  if (p < NPARAM)
    for (int c = q; c < a.nchunk; c += 4) part += a.part[(int64_t)c * NPARAM + p];
  s[t] = part;
  __syncthreads();
  if (q != 0 || p >= NPARAM) return;
  const float gsum = (s[j] + s[j + RA_PARAMS]) + (s[j + 2 * RA_PARAMS] + s[j + 3 * RA_PARAMS]);
  if (!a.adam) {
    a.grad[p] = gsum;
    return;
  }
  const float m = a.b1 * a.m[p] + (1.f - a.b1) * gsum;
  const float v = a.b2 * a.v[p] + (1.f - a.b2) * gsum * gsum;
  const float th = a.theta[p] - a.lr * (m / a.bc1) / (sqrtf(v / a.bc2) + a.eps);
  a.m[p] = m;
  a.v[p] = v;
  a.theta[p] = th;
  put_param(p, th, a.fimg, a.bimg);
}

// loss = (sum of the per-wave partials, in order) / (3B), one block.
__global__ __launch_bounds__(256) void mlp_loss_kernel(const float *part, int nparts, double inv_count, float *loss) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) acc += (double)part[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(s[0] * inv_count);
}

}  // namespace mlp
}  // namespace ism
