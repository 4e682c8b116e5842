// Processing order for the persistent step kernels.
//
// A cell's result does not depend on when it is processed, but the speed of a wave does: its
// lanes run the same instruction stream, so lanes whose cells sit in different temperature
// regimes execute both sides of every regime branch, and lanes whose cells need different
// numbers of substeps refill at different times.  Grouping cells with similar input
// temperature into the same waves removes most of that divergence, and taking the cells of a
// group slab by slab through the grid keeps a wave's loads on nearby lines.  When the caller holds the
// substep counts of the previous step of the same cells, they are the better key: cells are
// grouped by how long they will run, longest first.  The order is a
// counting sort on a 12-bit key: a per-block LDS histogram, an exclusive scan of the 4096
// bins, and a scatter that reserves one range per (block, bin) with a single global atomic.
// A block takes ORDER_PER items per thread (16,384 items), so that zeroing and flushing its
// 4096 bins, and its global atomics, are spread over many items.  Within a bin the order depends
// on atomic timing; results do not.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ism {

constexpr int ORDER_BITS = 12, ORDER_BINS = 1 << ORDER_BITS, ORDER_THREADS = 1024, ORDER_PER = 16;
constexpr int64_t ORDER_CHUNK = (int64_t)ORDER_THREADS * ORDER_PER;  // items per block (key, scatter)

__device__ __forceinline__ uint32_t order_quant(float x, float lo, float hi, int bits) {
  float u = (x - lo) / (hi - lo);
  u = fminf(fmaxf(u, 0.f), 1.f);  // NaN maps to 0
  return (uint32_t)(u * (float)((1 << bits) - 1) + 0.5f);
}

// Key of one cell: log10 T over [0, 8] rounded to 16 levels, about half a decade apart (the top
// 4 of the 12 bits),
// with the cell's place in the grid below it (its index's top 8 bits: 256 slabs), or, with
// previous substep counts, log2 of the count in [0, 17] on 12 bits.  Keys are visited from high
// to low (hot to cold, long to short).  The temperature bins are coarse on purpose: the lanes of
// a wave then take cells of one slab, near each other, and share the lines of their loads; with
// 4096 temperature bins the runs of one bin and block are a few cells long and every lane's
// load pulls its own line.  The slab bits keep that grouping also for item lists in no
// particular order (the surrogate step's fallback list).
constexpr int ORDER_T_BITS = 4;
__device__ __forceinline__ uint32_t order_key(const double *T, const int32_t *nsub, int64_t cell, int cshift) {
  if (nsub) {
    const int32_t c = nsub[cell];
    return (uint32_t)(ORDER_BINS - 1) - order_quant(log2f((float)(c > 1 ? c : 1)), 0.f, 17.f, ORDER_BITS);
  }
  return (uint32_t)(ORDER_BINS - 1) -
         ((order_quant(log10f((float)T[cell]), 0.f, 8.f, ORDER_T_BITS) << (ORDER_BITS - ORDER_T_BITS)) |
          ((uint32_t)(cell >> cshift) & ((1u << (ORDER_BITS - ORDER_T_BITS)) - 1u)));
}

struct OrderArgs {
  int64_t n;                          // items (upper bound when count is set)
  const unsigned long long *count;    // device item count, or null (= n)
  const int32_t *items;               // item -> cell, or null (item = cell)
  const double *T;
  const int32_t *nsub;                // previous substep counts per cell, or null
  uint16_t *key;                      // per item
  uint32_t *hist;                     // ORDER_BINS counts
  uint32_t *cursor;                   // ORDER_BINS running offsets
  int32_t *out;                       // ordered cells
  int32_t cshift;                     // cell index >> cshift: the slab (top 8 bits of the index)
};

__global__ __launch_bounds__(ORDER_THREADS) void order_zero_kernel(uint32_t *hist) {
  for (int b = threadIdx.x; b < ORDER_BINS; b += ORDER_THREADS) hist[b] = 0u;
}

__global__ __launch_bounds__(ORDER_THREADS) void order_key_kernel(OrderArgs a) {
  __shared__ uint32_t h[ORDER_BINS];
  for (int b = threadIdx.x; b < ORDER_BINS; b += ORDER_THREADS) h[b] = 0u;
  __syncthreads();
  const int64_t nitem = a.count ? (int64_t)*a.count : a.n;
  const int64_t i0 = (int64_t)blockIdx.x * ORDER_CHUNK + threadIdx.x;
#pragma unroll 4
  for (int j = 0; j < ORDER_PER; ++j) {
    const int64_t i = i0 + (int64_t)j * ORDER_THREADS;
    if (i < nitem) {
      const int64_t cell = a.items ? (int64_t)a.items[i] : i;
      const uint32_t k = order_key(a.T, a.nsub, cell, a.cshift);
      a.key[i] = (uint16_t)k;
      atomicAdd(&h[k], 1u);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < ORDER_BINS; b += ORDER_THREADS)
    if (h[b]) atomicAdd(&a.hist[b], h[b]);
}

// Exclusive scan of the histogram into cursor (one block; four bins per thread).
__global__ __launch_bounds__(ORDER_THREADS) void order_scan_kernel(OrderArgs a) {
  __shared__ uint32_t s[ORDER_THREADS];
  constexpr int PER = ORDER_BINS / ORDER_THREADS;
  uint32_t v[PER], sum = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    v[j] = a.hist[threadIdx.x * PER + j];
    sum += v[j];
  }
  s[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < ORDER_THREADS; off <<= 1) {
    const uint32_t t = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  uint32_t run = s[threadIdx.x] - sum;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    a.cursor[threadIdx.x * PER + j] = run;
    run += v[j];
  }
}

__global__ __launch_bounds__(ORDER_THREADS) void order_scatter_kernel(OrderArgs a) {
  __shared__ uint32_t cnt[ORDER_BINS];
  __shared__ uint32_t base[ORDER_BINS];
  for (int b = threadIdx.x; b < ORDER_BINS; b += ORDER_THREADS) cnt[b] = 0u;
  __syncthreads();
  const int64_t nitem = a.count ? (int64_t)*a.count : a.n;
  const int64_t i0 = (int64_t)blockIdx.x * ORDER_CHUNK + threadIdx.x;
  uint32_t k[ORDER_PER], rank[ORDER_PER];
#pragma unroll
  for (int j = 0; j < ORDER_PER; ++j) {
    const int64_t i = i0 + (int64_t)j * ORDER_THREADS;
    k[j] = 0u;
    rank[j] = 0u;
    if (i < nitem) {
      k[j] = a.key[i];
      rank[j] = atomicAdd(&cnt[k[j]], 1u);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < ORDER_BINS; b += ORDER_THREADS)
    if (cnt[b]) base[b] = atomicAdd(&a.cursor[b], cnt[b]);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < ORDER_PER; ++j) {
    const int64_t i = i0 + (int64_t)j * ORDER_THREADS;
    if (i < nitem) a.out[base[k[j]] + rank[j]] = a.items ? a.items[i] : (int32_t)i;
  }
}

}  // namespace ism
