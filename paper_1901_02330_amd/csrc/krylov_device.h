// Device helpers shared by the Krylov kernels (krylov.hip) and the inner pipelined CG
// (pcg.hip): wavefront and block reductions without atomics or fences, the XCD-aware
// row order of the inner-CG kernels, and the SELL-64 row product.
#pragma once

#include <type_traits>

#include "vem_internal.h"

namespace vem {
namespace {

constexpr int kThreads = kRedThreads;
constexpr int kMaxWaves = 16;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Workgroups are dealt round-robin to the eight XCDs, each with its own L2.  The
// inner-CG kernels take their rows from this logical block number instead: XCD x
// runs chunks x, x+8, x+16, ... of C consecutive blocks (C blocks = 16384 rows), so
// that the vector entries gathered around a chunk are fetched into one L2, while all
// eight XCDs still advance through the rows together.  Blocks past the last whole
// round of 8 chunks keep their own number.  (Measured on the 64^3 cube: 1.5% off the
// A_gamma iteration, 3.5% off the S iteration.  The saddle SpMV keeps the hardware
// order: its flux and pressure rows differ in cost, and contiguous bands per XCD
// left it 10% slower.)
__device__ inline int64_t xcd_block_of(int block) {
  const int b = blockIdx.x, P = gridDim.x;
  const int C = (16384 / block) > 0 ? (16384 / block) : 1;
  const int full = P / (8 * C) * (8 * C);
  const int x = b & 7, i = b >> 3, j = i / C, off = i % C;
  const int64_t mapped = (int64_t)(j * 8 + x) * C + off;
  return b >= full ? (int64_t)b : mapped;  // a select, not a branch: the kernel's loads stay in one block
}
__device__ inline int64_t xcd_block() { return xcd_block_of((int)blockDim.x); }
// The same for a kernel whose block size is the compile-time constant kBlock.  Kernels use the
// constant rather than blockDim.x where they know it: reading blockDim.x for arithmetic such as the
// divisions above costs a vector load of the dispatch's 16-bit block size at the start of the
// kernel, ahead of every other load (on the 64^3 Chebyshev product about 0.6 us of 5.7 us).
template <int kBlock>
__device__ inline int64_t xcd_block_n() { return xcd_block_of(kBlock); }

// Block-reduce K accumulators and store this block's partial sums at
// partials[blockIdx.x * K + k].  No atomics and no fences: the consumer is a
// later kernel on the same stream, and the kernel boundary makes the partials
// visible to every XCD.  kBlock: the launch's block size (these helpers take it as a constant).
template <int K, int kBlock>
__device__ inline void block_partials(const double (&acc)[K], double* partials) {
  static_assert(kBlock % 64 == 0 && kBlock / 64 <= kMaxWaves, "block size");
  __shared__ double sh[kMaxWaves][K];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = kBlock >> 6;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double v = wave_sum(acc[i]);
    if (lane == 0) sh[wid][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[w][threadIdx.x];
    partials[(size_t)blockIdx.x * K + threadIdx.x] = s;
  }
}

// Sum of nparts partials (stride K, component k) by the whole block, in a fixed
// order: every block that calls it obtains the same bits.
// Each thread's share of the partials is loaded kSumLoads at a time, all in flight at once (a loop
// that adds as it loads waits for every load in turn), and added in the same order as such a loop:
// the same bits.  Slots past nparts load partial 0 and add nothing.
constexpr int kSumLoads = 8;
template <int kBlock>
__device__ inline double block_sum_partials(const double* __restrict__ partials, int nparts, int K, int k) {
  __shared__ double sh[kMaxWaves];
  __shared__ double total;
  double s = 0.0;
  for (int b0 = threadIdx.x; b0 < nparts; b0 += kSumLoads * kBlock) {
    double v[kSumLoads];
#pragma unroll
    for (int u = 0; u < kSumLoads; ++u) {
      const int b = b0 + u * kBlock;
      v[u] = partials[(size_t)(b < nparts ? b : 0) * K + k];
    }
#pragma unroll
    for (int u = 0; u < kSumLoads; ++u)
      if (b0 + u * kBlock < nparts) s += v[u];
  }
  s = wave_sum(s);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = kBlock >> 6;
  if (lane == 0) sh[wid] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += sh[w];
    total = t;
  }
  __syncthreads();
  double r = total;
  __syncthreads();
  return r;
}

// Both components of nparts (gamma, delta) partial pairs, summed by the whole block
// in one pass, in a fixed order (every block obtains the same bits).
template <int kBlock>
__device__ inline void block_sum_partials2(const double* __restrict__ partials, int nparts, double (&out)[2]) {
  __shared__ double sh[kMaxWaves][2];
  __shared__ double total[2];
  double g = 0.0, d = 0.0;
  for (int b0 = threadIdx.x; b0 < nparts; b0 += kSumLoads * kBlock) {
    double vg[kSumLoads], vd[kSumLoads];
#pragma unroll
    for (int u = 0; u < kSumLoads; ++u) {
      const int b = b0 + u * kBlock, c = b < nparts ? b : 0;
      vg[u] = partials[2 * (size_t)c];
      vd[u] = partials[2 * (size_t)c + 1];
    }
#pragma unroll
    for (int u = 0; u < kSumLoads; ++u)
      if (b0 + u * kBlock < nparts) {
        g += vg[u];
        d += vd[u];
      }
  }
  g = wave_sum(g);
  d = wave_sum(d);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = kBlock >> 6;
  if (lane == 0) {
    sh[wid][0] = g;
    sh[wid][1] = d;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += sh[w][threadIdx.x];
    total[threadIdx.x] = t;
  }
  __syncthreads();
  out[0] = total[0];
  out[1] = total[1];
}

// ---- SELL-64: one thread per row -----------------------------------------------------------
template <typename T>
struct SellViewT {
  int64_t rows;
  const int* __restrict__ slice_ptr;
  const int* __restrict__ slice_len;
  const int* __restrict__ col;
  const T* __restrict__ val;
};
using SellView = SellViewT<double>;

inline SellView view(const Sell& A) { return {A.rows, A.slice_ptr, A.slice_len, A.col, A.val}; }

// Whole waves share a slice because every block size here is a multiple of 64 and every kernel
// gives a wave 64 consecutive rows from a multiple of 64.  The slice index is therefore the same on
// all lanes: taken from the first active lane it sits in scalar registers, and the slice's offset and
// length arrive through scalar loads, ahead of the vector loads that depend on them.
__device__ inline int64_t wave_uniform(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// The product is formed in the matrix's precision T from x of type X.
template <typename T, typename X>
__device__ inline T sell_dot(const SellViewT<T>& A, int64_t row, const X* __restrict__ x) {
  const int64_t s = wave_uniform(row >> 6);
  const int64_t base = A.slice_ptr[s] + (row & 63);
  const int len = A.slice_len[s];
  T acc = T(0);
#pragma unroll 4
  for (int k = 0; k < len; ++k) acc += A.val[base + 64 * k] * (T)x[A.col[base + 64 * k]];
  return acc;
}

// The same product for slices of at most kShortRow entries: all column and value loads are
// issued first, then all gathers, so a row costs two memory round trips instead of a chain
// per entry.  The loads take no branches (slots past the slice's length reload its first slot,
// a cache hit, so every address is valid), which lets every load of the row be in flight at
// once; only the sum skips those slots, in the same order as the loop above (same bits).
constexpr int kShortRow = 8;
template <typename T, typename X>
__device__ inline T sell_dot_short(const SellViewT<T>& A, int64_t row, const X* __restrict__ x) {
  const int64_t s = wave_uniform(row >> 6);
  const int64_t base = A.slice_ptr[s] + (row & 63);
  const int len = A.slice_len[s];
  int c[kShortRow];
  T v[kShortRow];
#pragma unroll
  for (int u = 0; u < kShortRow; ++u) {
    const int64_t at = base + 64 * (u < len ? u : 0);
    c[u] = A.col[at];
    v[u] = A.val[at];
  }
  X g[kShortRow];
#pragma unroll
  for (int u = 0; u < kShortRow; ++u) g[u] = x[c[u]];
  T acc = T(0);
#pragma unroll
  for (int u = 0; u < kShortRow; ++u)
    if (u < len) acc += v[u] * (T)g[u];
  return acc;
}

// The same product where every slice holds exactly N entries per row (a matrix of short rows whose
// slices were all padded to one length): N loads of each kind at fixed offsets and no masks, the
// same sum (padding entries add +0).  On the 64^3 cube's S (N = 7) a Chebyshev product took 4.8 us
// against 5.2-5.4 us with the masked form (stand-alone, per-launch events).
template <int N, typename T, typename X>
__device__ inline T sell_dot_fixed(const SellViewT<T>& A, int64_t row, const X* __restrict__ x) {
  // every slice holds 64 N slots, so slice s starts at 64 N s: no slice offset to load
  const int64_t base = (row >> 6) * (64 * N) + (row & 63);
  int c[N];
  T v[N];
#pragma unroll
  for (int u = 0; u < N; ++u) {
    c[u] = A.col[base + 64 * u];
    v[u] = A.val[base + 64 * u];
  }
  X g[N];
#pragma unroll
  for (int u = 0; u < N; ++u) g[u] = x[c[u]];
  T acc = T(0);
#pragma unroll
  for (int u = 0; u < N; ++u) acc += v[u] * (T)g[u];
  return acc;
}

// Row forms of the one-thread-per-row products: any length (loop), at most kShortRow entries
// (masked), or exactly N > 0 entries in every slice.
constexpr int kRowAny = 0, kRowShort = -1;
template <int kRow, typename T, typename X>
__device__ inline T sell_row(const SellViewT<T>& A, int64_t row, const X* __restrict__ x) {
  if constexpr (kRow == kRowShort)
    return sell_dot_short(A, row, x);
  else if constexpr (kRow > 0)
    return sell_dot_fixed<kRow>(A, row, x);
  else
    return sell_dot(A, row, x);
}

// The row form of a matrix: the fixed count 7 where every slice was padded to 7 entries per row (S
// of a hexahedral mesh at the lowest order; other fixed counts keep the masked form, which is
// correct for any padding), else the masked form for rows of at most kShortRow entries, else the
// loop.
inline int row_form(const Sell& A) {
  if (A.fixed_len == 7) return 7;
  return A.max_len <= kShortRow ? kRowShort : kRowAny;
}

// Calls f(std::integral_constant<int, form>) for a row form.
template <typename F>
inline void with_row_form(int form, F&& f) {
  switch (form) {
    case 7: f(std::integral_constant<int, 7>{}); break;
    case kRowShort: f(std::integral_constant<int, kRowShort>{}); break;
    default: f(std::integral_constant<int, kRowAny>{}); break;
  }
}

static SellView view_cs(const Sell& A) { return {A.rows, A.slice_ptr, A.slice_len, A.col, A.val_cs}; }
static SellViewT<float> view32(const Sell& A) { return {A.rows, A.slice_ptr, A.slice_len, A.col, A.val32}; }
static SellViewT<float> view_cs32(const Sell& A) {
  return {A.rows, A.slice_ptr, A.slice_len, A.col, A.val32_cs};
}

// Grid of the inner-CG kernels: one resident round at most (kPcgMaxThreads threads);
// larger systems loop over rows.
inline int pcg_grid(int64_t n, int block = kPcgThreads) {
  const int64_t cap = kPcgMaxThreads / block;
  int64_t b = (n + block - 1) / block;
  return (int)(b < cap ? (b < 1 ? 1 : b) : cap);
}

}  // namespace
}  // namespace vem
