// Sparse matrix-vector products, the vector kernels of flexible GMRES, and the
// classical FP32 conjugate gradients of mixed-precision inner solves (the pipelined
// FP64 inner CG is in pcg.hip).
//
// Reductions are deterministic and use neither atomics nor fences: every block
// writes its partial sums, and a later kernel on the same stream adds them in
// block order (a one-block finalize kernel, or every block of the consumer
// kernel itself for the inner CG).  Every kernel here is bandwidth bound.
#include <algorithm>

#include "krylov_device.h"

namespace vem {
namespace {

// out[k] = sum over nparts partials; block k handles component k.  hout (or null): a copy in pinned
// host memory (its device address), which the host reads once the stream has passed this kernel.
__global__ void __launch_bounds__(kThreads) k_finalize(int nparts, int K, const double* __restrict__ partials,
                                                       double* __restrict__ out, double* __restrict__ hout) {
  const int k = blockIdx.x;
  double v = block_sum_partials<kThreads>(partials, nparts, K, k);
  if (threadIdx.x == 0) {
    out[k] = v;
    if (hout) hout[k] = v;
  }
}

inline int red_grid(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  return (int)(b < kRedBlocks ? (b < 1 ? 1 : b) : kRedBlocks);
}

// ---- SELL-64 SpMV: one thread per row -------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_spmv(SellView A, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t row = (int64_t)blockIdx.x * kThreads + threadIdx.x; row < A.rows;
       row += (int64_t)gridDim.x * kThreads)
    y[row] = sell_dot(A, row, x);
}

// r = b - A x and per-block partials of ||r||^2
__global__ void __launch_bounds__(kThreads) k_residual(SellView A, const double* __restrict__ x,
                                                       const double* __restrict__ b, double* __restrict__ r,
                                                       double* partials) {
  double acc[1] = {0.0};
  for (int64_t row = (int64_t)blockIdx.x * kThreads + threadIdx.x; row < A.rows;
       row += (int64_t)gridDim.x * kThreads) {
    double ri = b[row] - sell_dot(A, row, x);
    r[row] = ri;
    acc[0] += ri * ri;
  }
  block_partials<1, kThreads>(acc, partials);
}

// ---- Gram-Schmidt kernels ------------------------------------------------------------------
// partials of V_k . w.  Up to 4 waves per SIMD: with the default budget of 8 (64 VGPRs) the K
// accumulators leave room for few loads in flight; this pass reads V from HBM (measured: the
// Block-Schur solve 22.5 -> 22.3 ms at 64^3).
template <int K>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 4))) k_dots(int64_t n, const double* __restrict__ V, int64_t ldv,
                                                   const double* __restrict__ w, double* partials) {
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    double wi = w[i];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += V[k * ldv + i] * wi;
  }
  block_partials<K, kThreads>(acc, partials);
}

// First Gram-Schmidt pass of Arnoldi step j (K = j + 1 >= 2 basis vectors) with the previous
// step's second pass folded in.  V[K-1] still holds w' of step j-1 (after its first projection,
// neither re-orthogonalised nor normalised), and hp holds that step's V^T w' (K-1 values) and
// ||w'||^2.  With V orthonormal, ||w' - V hp||^2 = ||w'||^2 - |hp|^2, so the pass finishes the
// basis vector v = (w' - V hp) / sqrt(||w'||^2 - |hp|^2) (written back, zeros if the difference
// is <= 0), then forms the partials of V_k . w with the finished vectors.  V[0..K-2] are read once
// for both jobs.
template <int K>
__device__ inline void dots_fix_body(int64_t n, double* __restrict__ V, int64_t ldv, const double* __restrict__ hp,
                                     const double* __restrict__ w, double* partials) {
  double hk[K - 1];
  double hh = 0.0;
#pragma unroll
  for (int k = 0; k < K - 1; ++k) {
    hk[k] = hp[k];
    hh += hk[k] * hk[k];
  }
  const double nn = hp[K - 1] - hh;
  const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const double wi = w[i];
    double t = V[(K - 1) * ldv + i];
#pragma unroll
    for (int k = 0; k < K - 1; ++k) {
      const double vk = V[k * ldv + i];
      t -= vk * hk[k];
      acc[k] += vk * wi;
    }
    t *= inv;
    V[(K - 1) * ldv + i] = t;
    acc[K - 1] += t * wi;
  }
  block_partials<K, kThreads>(acc, partials);
}
template <int K>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 4))) k_dots_fix(int64_t n, double* __restrict__ V, int64_t ldv,
                                                       const double* __restrict__ hp, const double* __restrict__ w,
                                                       double* partials) {
  dots_fix_body<K>(n, V, ldv, hp, w, partials);
}
// The same pass for K >= 29 basis vectors, with the register budget of two waves per SIMD: at four,
// the K - 1 coefficients and K accumulators did not fit, and the basis loads were issued one at a
// time (85 us against 53 us at K = 29, 64^3).
template <int K>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 2))) k_dots_fix_wide(int64_t n, double* __restrict__ V, int64_t ldv,
                                                       const double* __restrict__ hp, const double* __restrict__ w,
                                                       double* partials) {
  dots_fix_body<K>(n, V, ldv, hp, w, partials);
}

// w -= V h; partials of V_k . w (k < K) and of ||w||^2 (component K)
template <int K>
__global__ void __launch_bounds__(kThreads) k_update_dots(int64_t n, const double* __restrict__ V, int64_t ldv,
                                                          const double* __restrict__ h, double* __restrict__ w,
                                                          double* partials) {
  double hk[K], acc[K + 1];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    hk[k] = h[k];
    acc[k] = 0.0;
  }
  acc[K] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    double v[K];
    double wi = w[i];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      v[k] = V[k * ldv + i];
      wi -= v[k] * hk[k];
    }
    w[i] = wi;
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += v[k] * wi;
    acc[K] += wi * wi;
  }
  block_partials<K + 1, kThreads>(acc, partials);
}

// out = x - v (dot * inv_vv): x without its component along v (dot = v . x on the device)
__global__ void __launch_bounds__(kThreads) k_project(int64_t n, const double* x, const double* __restrict__ v, const double* __restrict__ dot,
                          double inv_vv, double* out) {
  const double c = *dot * inv_vv;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    out[i] = x[i] - v[i] * c;
}

// x += sum_k Z_k y_k
template <int K>
__global__ void __launch_bounds__(kThreads) k_combine(int64_t n, const double* __restrict__ Z, int64_t ldz,
                                                      const double* __restrict__ y, double* __restrict__ x) {
  double yk[K];
#pragma unroll
  for (int k = 0; k < K; ++k) yk[k] = y[k];
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    double s = x[i];
#pragma unroll
    for (int k = 0; k < K; ++k) s += Z[k * ldz + i] * yk[k];
    x[i] = s;
  }
}

__global__ void __launch_bounds__(kThreads) k_scale_to(int64_t n, const double* __restrict__ w, const double* __restrict__ norm2,
                           double* __restrict__ dst) {
  double inv = 1.0 / sqrt(norm2[0]);
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    dst[i] = w[i] * inv;
}

__global__ void __launch_bounds__(kThreads) k_scale_by(int64_t n, const double* __restrict__ x, const double* __restrict__ d, double c,
                           double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    y[i] = d ? c * d[i] * x[i] : c * x[i];
}

__global__ void __launch_bounds__(kThreads) k_fill(int64_t n, double v, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    y[i] = v;
}

__global__ void __launch_bounds__(kThreads) k_sum(int64_t n, const double* __restrict__ x, double* partials) {
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    acc[0] += x[i];
  block_partials<1, kThreads>(acc, partials);
}

// ---- classical Jacobi-PCG in FP32 (mixed-precision inner solves) --------------------------
// alpha = rho / p.Ap stays positive for an SPD matrix, which the pipelined
// recurrences do not guarantee once FP32 rounding meets an ill-conditioned
// operator.  Two kernels per iteration; the direction update p = z + beta p
// is fused into the product through two p buffers, and every kernel sums the
// partials the previous one left.  Vectors and matrix values in T (FP32 for mixed
// precision, FP64 for the classical inner form), dot products and scalars in FP64.
//   [spmv]   rho_k, beta = rho_k / rho_{k-1}; stop test; p_k = z + beta p_{k-1}; q = A p_k; partials p_k.q
//   [update] alpha = rho_k / p_k.q; x += alpha p_k; r -= alpha q; z = D^{-1} r; partials rho_{k+1}
template <typename T>
__global__ void __launch_bounds__(kPcgThreads) k_cg_init(int64_t n, const double* __restrict__ b,
                                                         const T* __restrict__ dinv, T* __restrict__ x,
                                                         T* __restrict__ r, T* __restrict__ z, PcgState* st,
                                                         double tol2, double* __restrict__ prho0) {
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * kPcgThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kPcgThreads) {
    const T bi = (T)b[i], zi = dinv[i] * bi;
    x[i] = T(0);
    r[i] = bi;
    z[i] = zi;
    acc[0] += (double)bi * (double)zi;
  }
  block_partials<1, kPcgThreads>(acc, prho0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->gamma[0] = st->gamma[1] = 0.0;
    st->gamma0 = 0.0;
    st->tol2 = tol2;
    st->count = 0;
    st->done = 0;
  }
}

template <typename T>
__global__ void __launch_bounds__(kPcgThreads) k_cg_spmv(int k, SellViewT<T> A, const T* __restrict__ z,
                                                         const T* __restrict__ pold, T* __restrict__ pnew,
                                                         T* __restrict__ q, PcgState* st,
                                                         const double* __restrict__ prho, double* __restrict__ ppq) {
  if (st->done) return;
  const int P = gridDim.x;
  const int cur = k & 1;
  const double rho = block_sum_partials<kPcgThreads>(prho + (size_t)cur * P, P, 1, 0);
  const double rho0 = k == 0 ? rho : st->gamma0;
  const double beta = k == 0 ? 0.0 : rho / st->gamma[1 - cur];
  const bool done = !(rho > st->tol2 * rho0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (k == 0) st->gamma0 = rho0;
    st->gamma[cur] = rho;
    if (done) st->done = 1;
  }
  if (done) return;
  const T bt = (T)beta;
  double acc[1] = {0.0};
  for (int64_t row = xcd_block_n<kPcgThreads>() * kPcgThreads + threadIdx.x; row < A.rows;
       row += (int64_t)gridDim.x * kPcgThreads) {
    const int64_t sl = row >> 6;
    const int64_t base = A.slice_ptr[sl] + (row & 63);
    const int len = A.slice_len[sl];
    T s = T(0), pn;
    if (k == 0) {
#pragma unroll 4
      for (int j = 0; j < len; ++j) s += A.val[base + 64 * j] * z[A.col[base + 64 * j]];
      pn = z[row];
    } else {
#pragma unroll 4
      for (int j = 0; j < len; ++j) {
        const int c = A.col[base + 64 * j];
        s += A.val[base + 64 * j] * (z[c] + bt * pold[c]);
      }
      pn = z[row] + bt * pold[row];
    }
    pnew[row] = pn;
    q[row] = s;
    acc[0] += (double)pn * (double)s;
  }
  block_partials<1, kPcgThreads>(acc, ppq);
}

template <typename T>
__global__ void __launch_bounds__(kPcgThreads) k_cg_update(int k, int64_t n, T* __restrict__ x, T* __restrict__ r,
                                                           T* __restrict__ z, const T* __restrict__ q,
                                                           const T* __restrict__ p, const T* __restrict__ dinv,
                                                           PcgState* st, double* __restrict__ prho,
                                                           const double* __restrict__ ppq) {
  if (st->done) return;
  const int P = gridDim.x;
  const int cur = k & 1;
  const double rho = block_sum_partials<kPcgThreads>(prho + (size_t)cur * P, P, 1, 0);
  const double pq = block_sum_partials<kPcgThreads>(ppq, P, 1, 0);
  if (!(pq > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st->done = 2;
    return;
  }
  const T a = (T)(rho / pq);
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * kPcgThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kPcgThreads) {
    x[i] += a * p[i];
    const T ri = r[i] - a * q[i];
    r[i] = ri;
    const T zi = dinv[i] * ri;
    z[i] = zi;
    acc[0] += (double)ri * (double)zi;
  }
  block_partials<1, kPcgThreads>(acc, prho + (size_t)(1 - cur) * P);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->count += 1;
    st->total += 1;
  }
}

// ---- face blocks: one thread per DOF row of an order-k face system ---------------------------
// Row (f, i) reads, per block j of face f, its NFD entries (contiguous) and the NFD entries of the
// gathered vector at face bcol (contiguous), as pairs when NFD is even (both runs start at a
// multiple of NFD elements of a 256-byte aligned allocation).  The sum runs over the columns in
// ascending order, as the SELL-64 product does.
template <typename T, int NFD>
struct BlockViewT {
  int64_t rows;
  const int* __restrict__ bptr;
  const int* __restrict__ bcol;
  const T* __restrict__ val;
};

template <int N, typename E>
__device__ inline void load_run(const E* __restrict__ p, E (&out)[N]) {
  if constexpr (N % 2 == 0) {
    typedef E pair_t __attribute__((ext_vector_type(2)));
    const pair_t* q = reinterpret_cast<const pair_t*>(p);
#pragma unroll
    for (int u = 0; u < N / 2; ++u) {
      const pair_t t = q[u];
      out[2 * u] = t.x;
      out[2 * u + 1] = t.y;
    }
  } else {
#pragma unroll
    for (int u = 0; u < N; ++u) out[u] = p[u];
  }
}

template <typename T, int NFD, typename X>
__device__ inline T mat_row(const BlockViewT<T, NFD>& A, int64_t row, const X* __restrict__ x) {
  const int64_t f = row / NFD;
  const int i = (int)(row - f * NFD);
  const int b1 = A.bptr[f + 1];
  T acc = T(0);
  // two (FP64) or four (FP32) blocks' loads in flight per thread: measured fastest at 6 face DOFs
  constexpr int kUnroll = sizeof(T) == 4 ? 4 : 2;
#pragma unroll kUnroll
  for (int b = A.bptr[f]; b < b1; ++b) {
    T v[NFD];
    X g[NFD];
    load_run<NFD>(A.val + ((int64_t)b * NFD + i) * NFD, v);
    load_run<NFD>(x + (int64_t)A.bcol[b] * NFD, g);
#pragma unroll
    for (int c = 0; c < NFD; ++c) acc += v[c] * (T)g[c];
  }
  return acc;
}

template <typename T, typename X>
__device__ inline T mat_row(const SellViewT<T>& A, int64_t row, const X* __restrict__ x) {
  return sell_dot(A, row, x);
}

// ---- CG on the face system F with the edge-patch Schwarz operator P (Block-Reg) -------------
// Two kernels per iteration, each one sparse product with a single gathered vector.  The products
// F p and P r are carried by recurrences, as F p_new = F z + beta F p_old and
// P r_new = P r_old - alpha P q: the product kernel gathers only z and the update kernel only q
// (gathering z and p, or r and q, doubled the gathers per matrix entry).  Every vector is then read
// and written at its own row only, except the gathered one, which the kernel does not write, so no
// vector needs a second buffer.  The recurrences equal the direct products in exact arithmetic;
// over the few dozen iterations of one inner solve their rounding stays far below the inner
// tolerance, and the outer flexible GMRES accepts any inner result.
//   [init]    z = P r0; x = 0; partials r0.z
//   [product] rho, beta = rho / rho_old; stop test; p = z + beta p; q = F z + beta q; partials p.q
//   [update]  alpha = rho / p.q; x += alpha p; r -= alpha q; z -= alpha P q; partials r.z
// Each kernel issues its row's product (which does not depend on this iteration's scalars) before
// it sums the previous kernel's partials, so the product's loads are in flight during that prologue.
// Block size: 1024 threads when every row has a thread, 256 when threads loop over rows.  V: the
// matrices' storage (SELL-64, or face blocks at order k).
template <typename T, int kBlock, typename V>
__global__ void __launch_bounds__(kBlock) k_scg_init(V P, const T* __restrict__ r0, T* __restrict__ x,
                                                     T* __restrict__ z, PcgState* st, double tol2,
                                                     double* __restrict__ prho0) {
  double acc[1] = {0.0};
  for (int64_t row = xcd_block_n<kBlock>() * kBlock + threadIdx.x; row < P.rows;
       row += (int64_t)gridDim.x * kBlock) {
    const T zi = mat_row(P, row, r0);
    z[row] = zi;
    x[row] = T(0);
    acc[0] += (double)r0[row] * (double)zi;
  }
  block_partials<1, kBlock>(acc, prho0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->gamma[0] = st->gamma[1] = 0.0;
    st->gamma0 = 0.0;
    st->tol2 = tol2;
    st->count = 0;
    st->done = 0;
  }
}

template <typename T, int kBlock, typename V>
__global__ void __launch_bounds__(kBlock) k_scg_prod(int k, int early, V F, const T* __restrict__ z,
                                                     T* __restrict__ p, T* __restrict__ q, PcgState* st,
                                                     const double* __restrict__ prho, double* __restrict__ ppq) {
  if (early && st->done) return;
  const int G = gridDim.x;
  const int cur = k & 1;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  int64_t row = xcd_block_n<kBlock>() * kBlock + threadIdx.x;
  T fz = T(0), zi = T(0), po = T(0), qo = T(0);
  auto load = [&](int64_t i) {
    zi = z[i];
    if (k > 0) {
      po = p[i];
      qo = q[i];
    }
    fz = mat_row(F, i, z);
  };
  if (row < F.rows) load(row);
  const int was_done = st->done;
  const double rho = block_sum_partials<kBlock>(prho + (size_t)cur * G, G, 1, 0);
  if (was_done) return;
  const double rho0 = k == 0 ? rho : st->gamma0;
  const double beta = k == 0 ? 0.0 : rho / st->gamma[1 - cur];
  const bool done = !(rho > st->tol2 * rho0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (k == 0) st->gamma0 = rho0;
    st->gamma[cur] = rho;
    if (done) st->done = 1;
  }
  if (done) return;
  const T bt = (T)beta;
  double acc[1] = {0.0};
  while (row < F.rows) {
    const T pn = k == 0 ? zi : zi + bt * po;
    const T qn = k == 0 ? fz : fz + bt * qo;
    p[row] = pn;
    q[row] = qn;
    acc[0] += (double)pn * (double)qn;
    row += stride;
    if (row < F.rows) load(row);
  }
  block_partials<1, kBlock>(acc, ppq);
}

template <typename T, int kBlock, typename V>
__global__ void __launch_bounds__(kBlock) k_scg_update(int k, int early, V P, T* __restrict__ x,
                                                       T* __restrict__ r, T* __restrict__ z,
                                                       const T* __restrict__ q, const T* __restrict__ p,
                                                       PcgState* st, double* __restrict__ prho,
                                                       const double* __restrict__ ppq) {
  if (early && st->done) return;
  const int G = gridDim.x;
  const int cur = k & 1;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  int64_t row = xcd_block_n<kBlock>() * kBlock + threadIdx.x;
  T pq_r = T(0), qi = T(0), ri = T(0), zi = T(0), xi = T(0), pi = T(0);
  auto load = [&](int64_t i) {
    qi = q[i];
    ri = r[i];
    zi = z[i];
    xi = x[i];
    pi = p[i];
    pq_r = mat_row(P, i, q);
  };
  if (row < P.rows) load(row);
  const int was_done = st->done;
  const double rho = block_sum_partials<kBlock>(prho + (size_t)cur * G, G, 1, 0);
  const double pq = block_sum_partials<kBlock>(ppq, G, 1, 0);
  if (was_done) return;
  if (!(pq > 0.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st->done = 2;
    return;
  }
  const T a = (T)(rho / pq);
  double acc[1] = {0.0};
  while (row < P.rows) {
    const T rn = ri - a * qi;
    const T zn = zi - a * pq_r;
    r[row] = rn;
    z[row] = zn;
    x[row] = xi + a * pi;
    acc[0] += (double)rn * (double)zn;
    row += stride;
    if (row < P.rows) load(row);
  }
  block_partials<1, kBlock>(acc, prho + (size_t)(1 - cur) * G);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->count += 1;
    st->total += 1;
  }
}

template <typename T>
SellViewT<T> values_view(const Sell& A);
template <>
SellViewT<double> values_view<double>(const Sell& A) {
  return view(A);
}
template <>
SellViewT<float> values_view<float>(const Sell& A) {
  return view32(A);
}

__global__ void __launch_bounds__(kThreads) k_to_f32(int64_t n, const double* __restrict__ x, float* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    y[i] = (float)x[i];
}

__global__ void __launch_bounds__(kThreads) k_to_f64(int64_t n, const float* __restrict__ x, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    y[i] = (double)x[i];
}

__global__ void __launch_bounds__(kThreads) k_col_scale(int64_t n, const int* __restrict__ col, const double* __restrict__ val,
                            const double* __restrict__ dinv, double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    out[i] = val[i] * dinv[col[i]];
}

inline int stream_grid(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  const int64_t cap = 4096;
  return (int)(b < cap ? (b < 1 ? 1 : b) : cap);
}

#define VEM_K_CASES_FROM2(X) \
  X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20) \
  X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)
#define VEM_K_CASES(X) X(1) VEM_K_CASES_FROM2(X)

template <int K>
void dots_fix_launch(hipStream_t s, int grid, int64_t n, double* V, int64_t ldv, const double* hp, const double* w,
                     double* partials) {
  if constexpr (K >= 29)
    k_dots_fix_wide<K><<<grid, kThreads, 0, s>>>(n, V, ldv, hp, w, partials);
  else
    k_dots_fix<K><<<grid, kThreads, 0, s>>>(n, V, ldv, hp, w, partials);
}

void finalize(hipStream_t s, int nparts, int K, const double* partials, double* out, double* hout = nullptr) {
  k_finalize<<<K, kThreads, 0, s>>>(nparts, K, partials, out, hout);
}

}  // namespace

void launch_spmv(hipStream_t s, const Sell& A, const double* x, double* y) {
  if (A.rows <= 0) return;
  int64_t blocks = (A.rows + kThreads - 1) / kThreads;
  k_spmv<<<(int)(blocks < 65536 ? blocks : 65536), kThreads, 0, s>>>(view(A), x, y);
}

void launch_residual(hipStream_t s, const Sell& A, const double* x, const double* b, double* r, double* partials,
                     double* out) {
  int grid = red_grid(A.rows);
  k_residual<<<grid, kThreads, 0, s>>>(view(A), x, b, r, partials);
  finalize(s, grid, 1, partials, out);
}

void launch_dots(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* w, double* partials,
                 double* out, double* hout) {
  int grid = red_grid(n);
  switch (k) {
#define X(K) \
  case K: k_dots<K><<<grid, kThreads, 0, s>>>(n, V, ldv, w, partials); break;
    VEM_K_CASES(X)
#undef X
    default: throw Error{VEM_EINVAL, "too many basis vectors"};
  }
  finalize(s, grid, k, partials, out, hout);
}

void launch_update_dots(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* h, double* w,
                        double* partials, double* out, double* hout) {
  int grid = red_grid(n);
  switch (k) {
#define X(K) \
  case K: k_update_dots<K><<<grid, kThreads, 0, s>>>(n, V, ldv, h, w, partials); break;
    VEM_K_CASES(X)
#undef X
    default: throw Error{VEM_EINVAL, "too many basis vectors"};
  }
  finalize(s, grid, k + 1, partials, out, hout);
}

void launch_dots_fix(hipStream_t s, int64_t n, int k, double* V, int64_t ldv, const double* hp, const double* w,
                     double* partials, double* out, double* hout) {
  int grid = red_grid(n);
  switch (k) {
#define X(K) \
  case K: dots_fix_launch<K>(s, grid, n, V, ldv, hp, w, partials); break;
    VEM_K_CASES_FROM2(X)
#undef X
    default: throw Error{VEM_EINVAL, "the folded first pass needs 2 to 32 basis vectors"};
  }
  finalize(s, grid, k, partials, out, hout);
}

void launch_project(hipStream_t s, int64_t n, const double* x, const double* v, const double* dot, double inv_vv,
                    double* out) {
  if (n > 0) k_project<<<stream_grid(n), kThreads, 0, s>>>(n, x, v, dot, inv_vv, out);
}

void launch_combine(hipStream_t s, int64_t n, int k, const double* Z, int64_t ldz, const double* y, double* x) {
  int grid = stream_grid(n);
  switch (k) {
#define X(K) \
  case K: k_combine<K><<<grid, kThreads, 0, s>>>(n, Z, ldz, y, x); break;
    VEM_K_CASES(X)
#undef X
    default: throw Error{VEM_EINVAL, "too many basis vectors"};
  }
}

void launch_scale_to(hipStream_t s, int64_t n, const double* w, const double* norm2, double* dst) {
  k_scale_to<<<stream_grid(n), kThreads, 0, s>>>(n, w, norm2, dst);
}
void launch_scale_by(hipStream_t s, int64_t n, const double* x, const double* d, double c, double* y) {
  if (n > 0) k_scale_by<<<stream_grid(n), kThreads, 0, s>>>(n, x, d, c, y);
}
void launch_copy(hipStream_t s, int64_t n, const double* x, double* y) {
  if (n > 0) VEM_HIP(hipMemcpyAsync(y, x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
}
void launch_fill(hipStream_t s, int64_t n, double v, double* y) {
  if (n > 0) k_fill<<<stream_grid(n), kThreads, 0, s>>>(n, v, y);
}
void launch_sum(hipStream_t s, int64_t n, const double* x, double* partials, double* out) {
  int grid = red_grid(n);
  k_sum<<<grid, kThreads, 0, s>>>(n, x, partials);
  finalize(s, grid, 1, partials, out);
}

void launch_col_scale(hipStream_t s, Sell& A, const double* dinv) {
  if (A.nnz <= 0) return;
  A.val_cs.alloc(A.nnz);
  VEM_REQUIRE(A.val_cs.p && A.val.p && A.col.p, VEM_EINVAL, "column scaling of an unbuilt matrix");
  k_col_scale<<<stream_grid(A.nnz), kThreads, 0, s>>>(A.nnz, A.col, A.val, dinv, A.val_cs);
}


void launch_col_scale32(hipStream_t s, Sell& A, const double* dinv, float* dinv32) {
  if (A.nnz <= 0) return;
  A.val32.alloc(A.nnz);
  A.val32_cs.alloc(A.nnz);
  k_to_f32<<<stream_grid(A.nnz), kThreads, 0, s>>>(A.nnz, A.val, A.val32);
  k_to_f32<<<stream_grid(A.nnz), kThreads, 0, s>>>(A.nnz, A.val_cs, A.val32_cs);
  k_to_f32<<<stream_grid(A.rows), kThreads, 0, s>>>(A.rows, dinv, dinv32);
}

void launch_to_f64(hipStream_t s, int64_t n, const float* x, double* y) {
  if (n > 0) k_to_f64<<<stream_grid(n), kThreads, 0, s>>>(n, x, y);
}

void launch_pcg_init32(hipStream_t s, const Sell& A, const PcgWork32& w, const double* b, PcgState* st, double tol,
                       int maxit, double* part) {
  (void)maxit;
  k_cg_init<float><<<pcg_grid(A.rows), kPcgThreads, 0, s>>>(A.rows, b, w.dinv, w.x, w.r, w.z, st, tol * tol, part);
}

// The classical iteration in FP64 on the unscaled values (same work layout as the FP32 one below)
void launch_pcg_init64c(hipStream_t s, const Sell& A, const PcgWork& w, const double* b, PcgState* st, double tol,
                        double* part) {
  k_cg_init<double><<<pcg_grid(A.rows), kPcgThreads, 0, s>>>(A.rows, b, w.dinv, w.x, w.r, w.z, st, tol * tol, part);
}

void launch_pcg_iter64c(hipStream_t s, int i, const Sell& A, const PcgWork& w, PcgState* st, double* part) {
  const int P = pcg_grid(A.rows);
  double* prho = part;  // 2 x P slots
  double* ppq = part + 2 * (size_t)P;
  double* pold = (i & 1) ? w.p : w.s;
  double* pnew = (i & 1) ? w.s : w.p;
  k_cg_spmv<double><<<P, kPcgThreads, 0, s>>>(i, view(A), w.z, pold, pnew, w.w0, st, prho, ppq);
  k_cg_update<double><<<P, kPcgThreads, 0, s>>>(i, A.rows, w.x, w.r, w.z, w.w0, pnew, w.dinv, st, prho, ppq);
}

// FP32 work layout: r, z as named; s and p hold the two direction buffers, w0 holds A p
void launch_pcg_iter32(hipStream_t s, int i, const Sell& A, const PcgWork32& w, PcgState* st, double* part) {
  const int P = pcg_grid(A.rows);
  double* prho = part;  // 2 x P slots
  double* ppq = part + 2 * (size_t)P;
  float* pold = (i & 1) ? w.p : w.s;
  float* pnew = (i & 1) ? w.s : w.p;
  k_cg_spmv<float><<<P, kPcgThreads, 0, s>>>(i, view32(A), w.z, pold, pnew, w.w0, st, prho, ppq);
  k_cg_update<float><<<P, kPcgThreads, 0, s>>>(i, A.rows, w.x, w.r, w.z, w.w0, pnew, w.dinv, st, prho, ppq);
}

template <typename T>
const T* block_values(const FaceBlocks& B);
template <>
const double* block_values<double>(const FaceBlocks& B) {
  return B.val.p;
}
template <>
const float* block_values<float>(const FaceBlocks& B) {
  return B.val32.p;
}
template <typename T, int NFD>
BlockViewT<T, NFD> block_view(const FaceBlocks& B) {
  return {B.nf * NFD, B.bptr.p, B.bcol.p, block_values<T>(B)};
}

// Grid of the Schwarz-CG kernels: at most the blocks that are resident at once (the fewest over
// the three kernels of a form, from their register use), since the threads loop over the rows and
// blocks beyond one resident round would run as a second, partly filled round.  The init and the
// iteration kernels take the same grid, so the partial sums match.
template <typename T, int kBlock, typename V>
int scg_grid(int64_t rows) {
  static const int resident = [] {
    int dev = 0, ncu = 0, a = 0, b = 0, c = 0;
    VEM_HIP(hipGetDevice(&dev));
    VEM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    VEM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_scg_init<T, kBlock, V>, kBlock, 0));
    VEM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_scg_prod<T, kBlock, V>, kBlock, 0));
    VEM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&c, k_scg_update<T, kBlock, V>, kBlock, 0));
    const int m = std::min(a, std::min(b, c));
    return std::max(1, m) * std::max(1, ncu);
  }();
  return std::min(pcg_grid(rows, kBlock), resident);
}

template <typename T, typename V>
void scg_init_as(hipStream_t s, const V& P, const PcgWorkT<T>& w, PcgState* st, double tol, double* part) {
  if (P.rows > kPcgMaxThreads)
    k_scg_init<T, 256><<<scg_grid<T, 256, V>(P.rows), 256, 0, s>>>(P, w.r, w.x, w.z, st, tol * tol, part);
  else
    k_scg_init<T, 1024><<<scg_grid<T, 1024, V>(P.rows), 1024, 0, s>>>(P, w.r, w.x, w.z, st, tol * tol, part);
}

// work layout: x, r, z, p as named, w0 = q (s and w1 unused); the init's grid (same rows, same
// block size) leaves the partials the first product kernel sums
template <typename T, typename V>
void scg_iter_as(hipStream_t s, int i, const V& F, const V& P, const PcgWorkT<T>& w, PcgState* st, double* part,
                 int early) {
  if (F.rows > kPcgMaxThreads) {
    const int G = scg_grid<T, 256, V>(F.rows);
    double* prho = part;  // 2 x G slots
    double* ppq = part + 2 * (size_t)G;
    k_scg_prod<T, 256><<<G, 256, 0, s>>>(i, early, F, w.z, w.p, w.w0, st, prho, ppq);
    k_scg_update<T, 256><<<G, 256, 0, s>>>(i, early, P, w.x, w.r, w.z, w.w0, w.p, st, prho, ppq);
  } else {
    const int G = scg_grid<T, 1024, V>(F.rows);
    double* prho = part;
    double* ppq = part + 2 * (size_t)G;
    k_scg_prod<T, 1024><<<G, 1024, 0, s>>>(i, early, F, w.z, w.p, w.w0, st, prho, ppq);
    k_scg_update<T, 1024><<<G, 1024, 0, s>>>(i, early, P, w.x, w.r, w.z, w.w0, w.p, st, prho, ppq);
  }
}

template <typename T>
void launch_scg_init(hipStream_t s, const Schwarz& X, const PcgWorkT<T>& w, PcgState* st, double tol, double* part) {
  if (!X.blocked) return scg_init_as<T>(s, values_view<T>(X.Ps), w, st, tol, part);
  switch (X.Pb.nfd) {
    case 3: return scg_init_as<T>(s, block_view<T, 3>(X.Pb), w, st, tol, part);
    case 6: return scg_init_as<T>(s, block_view<T, 6>(X.Pb), w, st, tol, part);
    case 10: return scg_init_as<T>(s, block_view<T, 10>(X.Pb), w, st, tol, part);
    default: throw Error{VEM_EINVAL, "face blocks of an unsupported size"};
  }
}

template <typename T>
void launch_scg_iter(hipStream_t s, int i, const Sell& F, const Schwarz& X, const PcgWorkT<T>& w, PcgState* st,
                     double* part, bool early_exit) {
  const int e = early_exit ? 1 : 0;
  if (!X.blocked) return scg_iter_as<T>(s, i, values_view<T>(F), values_view<T>(X.Ps), w, st, part, e);
  switch (X.Pb.nfd) {
    case 3: return scg_iter_as<T>(s, i, block_view<T, 3>(X.Fb), block_view<T, 3>(X.Pb), w, st, part, e);
    case 6: return scg_iter_as<T>(s, i, block_view<T, 6>(X.Fb), block_view<T, 6>(X.Pb), w, st, part, e);
    case 10: return scg_iter_as<T>(s, i, block_view<T, 10>(X.Fb), block_view<T, 10>(X.Pb), w, st, part, e);
    default: throw Error{VEM_EINVAL, "face blocks of an unsupported size"};
  }
}

template void launch_scg_init<double>(hipStream_t, const Schwarz&, const PcgWorkT<double>&, PcgState*, double,
                                      double*);
template void launch_scg_init<float>(hipStream_t, const Schwarz&, const PcgWorkT<float>&, PcgState*, double,
                                     double*);
template void launch_scg_iter<double>(hipStream_t, int, const Sell&, const Schwarz&, const PcgWorkT<double>&,
                                      PcgState*, double*, bool);
template void launch_scg_iter<float>(hipStream_t, int, const Sell&, const Schwarz&, const PcgWorkT<float>&,
                                     PcgState*, double*, bool);

}  // namespace vem
