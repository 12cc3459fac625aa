// Sparse matrix-vector products and the vector kernels of flexible GMRES and
// of the inner Jacobi-preconditioned conjugate gradients.
//
// Reductions are deterministic: every block writes its partial sums, the last
// block to arrive (atomic ticket) adds the partials in block order and, where
// the solver needs it, updates the device-resident scalar state.  The flux
// and pressure vectors are HBM-streamed; every kernel here is bandwidth bound.
#include "vem_internal.h"

namespace vem {
namespace {

constexpr int kThreads = kRedThreads;
constexpr int kWaves = kThreads / 64;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Block-reduce K accumulators, publish per-block partials, and let the last
// block sum them in block order into res[] (shared).  Returns true in the
// last block (all its threads), where res[] holds the grid totals.
template <int K>
__device__ inline bool grid_reduce(const double (&acc)[K], double* partials, unsigned* counter, double* res) {
  __shared__ double sh[kWaves][K];
  __shared__ int last;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double v = wave_sum(acc[i]);
    if (lane == 0) sh[wid][i] = v;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += sh[w][threadIdx.x];
    partials[(size_t)blockIdx.x * K + threadIdx.x] = s;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = (atomicAdd(counter, 1u) == gridDim.x - 1) ? 1 : 0;
  __syncthreads();
  if (!last) return false;
  __threadfence();
  for (int i = 0; i < K; ++i) {
    double s = 0.0;
    for (unsigned b = threadIdx.x; b < gridDim.x; b += blockDim.x) s += partials[(size_t)b * K + i];
    s = wave_sum(s);
    if (lane == 0) sh[wid][0] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kWaves; ++w) t += sh[w][0];
      res[i] = t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *counter = 0u;
  return true;
}

inline int red_grid(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  return (int)(b < kRedBlocks ? (b < 1 ? 1 : b) : kRedBlocks);
}

// ---- SpMV: L lanes per row, rows in consecutive groups -------------------------------------
template <int L>
__device__ inline double row_dot(int64_t row, int lane, const int* __restrict__ rowptr, const int* __restrict__ col,
                                 const double* __restrict__ val, const double* __restrict__ x) {
  double s = 0.0;
  int e = rowptr[row + 1];
  for (int j = rowptr[row] + lane; j < e; j += L) s += val[j] * x[col[j]];
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, L);
  return s;
}

template <int L>
__global__ void __launch_bounds__(kThreads) k_spmv(int64_t rows, const int* __restrict__ rowptr,
                                                   const int* __restrict__ col, const double* __restrict__ val,
                                                   const double* __restrict__ x, double* __restrict__ y) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t row = g / L;
  int lane = (int)(g & (L - 1));
  if (row >= rows) return;
  double s = row_dot<L>(row, lane, rowptr, col, val, x);
  if (lane == 0) y[row] = s;
}

// r = b - A x and ||r||^2 (grid-stride over row groups)
template <int L>
__global__ void __launch_bounds__(kThreads) k_residual(int64_t rows, const int* __restrict__ rowptr,
                                                       const int* __restrict__ col, const double* __restrict__ val,
                                                       const double* __restrict__ x, const double* __restrict__ b,
                                                       double* __restrict__ r, double* partials, unsigned* counter,
                                                       double* out) {
  const int lane = threadIdx.x & (L - 1);
  const int64_t groups_per_grid = (int64_t)gridDim.x * blockDim.x / L;
  double acc[1] = {0.0};
  for (int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L; row < rows; row += groups_per_grid) {
    double s = row_dot<L>(row, lane, rowptr, col, val, x);
    if (lane == 0) {
      double ri = b[row] - s;
      r[row] = ri;
      acc[0] += ri * ri;
    }
  }
  __shared__ double res[1];
  if (grid_reduce<1>(acc, partials, counter, res) && threadIdx.x == 0) out[0] = res[0];
}

// ---- Gram-Schmidt kernels ------------------------------------------------------------------
// out[k] = V_k . w
template <int K>
__global__ void __launch_bounds__(kThreads) k_dots(int64_t n, const double* __restrict__ V, int64_t ldv,
                                                   const double* __restrict__ w, double* partials,
                                                   unsigned* counter, double* out) {
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double wi = w[i];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += V[k * ldv + i] * wi;
  }
  __shared__ double res[K];
  if (grid_reduce<K>(acc, partials, counter, res) && threadIdx.x == 0)
    for (int k = 0; k < K; ++k) out[k] = res[k];
}

// w -= V h; out[k] = V_k . w (k < K), out[K] = ||w||^2
template <int K>
__global__ void __launch_bounds__(kThreads) k_update_dots(int64_t n, const double* __restrict__ V, int64_t ldv,
                                                          const double* __restrict__ h, double* __restrict__ w,
                                                          double* partials, unsigned* counter, double* out) {
  double hk[K], acc[K + 1];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    hk[k] = h[k];
    acc[k] = 0.0;
  }
  acc[K] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
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
  __shared__ double res[K + 1];
  if (grid_reduce<K + 1>(acc, partials, counter, res) && threadIdx.x == 0)
    for (int k = 0; k <= K; ++k) out[k] = res[k];
}

// w -= V h; out[0] = ||w||^2
template <int K>
__global__ void __launch_bounds__(kThreads) k_update_norm(int64_t n, const double* __restrict__ V, int64_t ldv,
                                                          const double* __restrict__ h, double* __restrict__ w,
                                                          double* partials, unsigned* counter, double* out) {
  double hk[K];
#pragma unroll
  for (int k = 0; k < K; ++k) hk[k] = h[k];
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double wi = w[i];
#pragma unroll
    for (int k = 0; k < K; ++k) wi -= V[k * ldv + i] * hk[k];
    w[i] = wi;
    acc[0] += wi * wi;
  }
  __shared__ double res[1];
  if (grid_reduce<1>(acc, partials, counter, res) && threadIdx.x == 0) out[0] = res[0];
}

// x += sum_k Z_k y_k
template <int K>
__global__ void __launch_bounds__(kThreads) k_combine(int64_t n, const double* __restrict__ Z, int64_t ldz,
                                                      const double* __restrict__ y, double* __restrict__ x) {
  double yk[K];
#pragma unroll
  for (int k = 0; k < K; ++k) yk[k] = y[k];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = x[i];
#pragma unroll
    for (int k = 0; k < K; ++k) s += Z[k * ldz + i] * yk[k];
    x[i] = s;
  }
}

__global__ void k_scale_to(int64_t n, const double* __restrict__ w, const double* __restrict__ norm2,
                           double* __restrict__ dst) {
  double inv = 1.0 / sqrt(norm2[0]);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = w[i] * inv;
}

__global__ void k_scale_by(int64_t n, const double* __restrict__ x, const double* __restrict__ d, double c,
                           double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = d ? c * d[i] * x[i] : c * x[i];
}

__global__ void k_fill(int64_t n, double v, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = v;
}

__global__ void k_sum(int64_t n, const double* __restrict__ x, double* partials, unsigned* counter, double* out) {
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc[0] += x[i];
  __shared__ double res[1];
  if (grid_reduce<1>(acc, partials, counter, res) && threadIdx.x == 0) out[0] = res[0];
}

// ---- inner Jacobi-preconditioned CG, state kept on the device -----------------------------
// x = 0, r = b, z = D^{-1} b, p = z, rho0 = r.z
__global__ void __launch_bounds__(kThreads) k_pcg_init(int64_t n, const double* __restrict__ b,
                                                       const double* __restrict__ dinv, double* __restrict__ x,
                                                       double* __restrict__ r, double* __restrict__ z,
                                                       double* __restrict__ p, PcgState* st, double tol2, int maxit,
                                                       double* partials, unsigned* counter) {
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double bi = b[i], zi = dinv[i] * bi;
    x[i] = 0.0;
    r[i] = bi;
    z[i] = zi;
    p[i] = zi;
    acc[0] += bi * zi;
  }
  __shared__ double res[1];
  if (grid_reduce<1>(acc, partials, counter, res) && threadIdx.x == 0) {
    st->rho = res[0];
    st->rho0 = res[0];
    st->alpha = 0.0;
    st->beta = 0.0;
    st->tol2 = tol2;
    st->it = 0;
    st->maxit = maxit;
    st->done = (!(res[0] > 0.0) || maxit <= 0) ? 1 : 0;
  }
}

// q = A p, alpha = rho / (p.q)
template <int L>
__global__ void __launch_bounds__(kThreads) k_pcg_spmv(int64_t rows, const int* __restrict__ rowptr,
                                                       const int* __restrict__ col, const double* __restrict__ val,
                                                       const double* __restrict__ p, double* __restrict__ q,
                                                       PcgState* st, double* partials, unsigned* counter) {
  if (st->done) return;
  const int lane = threadIdx.x & (L - 1);
  const int64_t groups_per_grid = (int64_t)gridDim.x * blockDim.x / L;
  double acc[1] = {0.0};
  for (int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L; row < rows; row += groups_per_grid) {
    double s = row_dot<L>(row, lane, rowptr, col, val, p);
    if (lane == 0) {
      q[row] = s;
      acc[0] += s * p[row];
    }
  }
  __shared__ double res[1];
  if (grid_reduce<1>(acc, partials, counter, res) && threadIdx.x == 0) {
    double pq = res[0];
    if (pq > 0.0) {
      st->alpha = st->rho / pq;
    } else {
      st->alpha = 0.0;
      st->done = 2;  // loss of positivity: stop with the current iterate
    }
  }
}

// x += alpha p, r -= alpha q, z = D^{-1} r, rho' = r.z, beta = rho'/rho
__global__ void __launch_bounds__(kThreads) k_pcg_update(int64_t n, double* __restrict__ x, double* __restrict__ r,
                                                         double* __restrict__ z, const double* __restrict__ q,
                                                         const double* __restrict__ p,
                                                         const double* __restrict__ dinv, PcgState* st,
                                                         double* partials, unsigned* counter) {
  if (st->done) return;
  const double alpha = st->alpha;
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    double ri = r[i] - alpha * q[i];
    r[i] = ri;
    double zi = dinv[i] * ri;
    z[i] = zi;
    acc[0] += ri * zi;
  }
  __shared__ double res[1];
  if (grid_reduce<1>(acc, partials, counter, res) && threadIdx.x == 0) {
    double rn = res[0];
    st->beta = rn / st->rho;
    st->rho = rn;
    st->it += 1;
    if (rn <= st->tol2 * st->rho0 || st->it >= st->maxit || !(rn == rn)) st->done = 1;
  }
}

// p = z + beta p
__global__ void __launch_bounds__(kThreads) k_pcg_dir(int64_t n, const double* __restrict__ z,
                                                      double* __restrict__ p, const PcgState* st) {
  if (st->done) return;
  const double beta = st->beta;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z[i] + beta * p[i];
}

inline int stream_grid(int64_t n) {
  int64_t b = (n + kThreads - 1) / kThreads;
  const int64_t cap = 4096;
  return (int)(b < cap ? (b < 1 ? 1 : b) : cap);
}

#define VEM_K_CASES(X) \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20) \
  X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)

}  // namespace

int spmv_lanes(double avg_row) {
  int L = 1;
  while (L < 64 && 2 * L <= avg_row) L *= 2;
  if (L < 2) L = 2;
  return L;
}

void launch_spmv(hipStream_t s, int lanes, int64_t rows, const int* rowptr, const int* col, const double* val,
                 const double* x, double* y) {
  if (rows <= 0) return;
  int64_t threads = rows * lanes;
  int grid = (int)((threads + kThreads - 1) / kThreads);
  switch (lanes) {
#define X(L) \
  case L: k_spmv<L><<<grid, kThreads, 0, s>>>(rows, rowptr, col, val, x, y); break;
    X(2) X(4) X(8) X(16) X(32) X(64)
#undef X
    default: throw Error{VEM_EINVAL, "bad lanes per row"};
  }
}

void launch_residual(hipStream_t s, int lanes, int64_t rows, const int* rowptr, const int* col, const double* val,
                     const double* x, const double* b, double* r, double* partials, unsigned* counter,
                     double* out) {
  int grid = red_grid(rows * lanes);
  switch (lanes) {
#define X(L) \
  case L: k_residual<L><<<grid, kThreads, 0, s>>>(rows, rowptr, col, val, x, b, r, partials, counter, out); break;
    X(2) X(4) X(8) X(16) X(32) X(64)
#undef X
    default: throw Error{VEM_EINVAL, "bad lanes per row"};
  }
}

void launch_dots(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* w, double* partials,
                 unsigned* counter, double* out) {
  int grid = red_grid(n);
  switch (k) {
#define X(K) \
  case K: k_dots<K><<<grid, kThreads, 0, s>>>(n, V, ldv, w, partials, counter, out); break;
    VEM_K_CASES(X)
#undef X
    default: throw Error{VEM_EINVAL, "too many basis vectors"};
  }
}

void launch_update_dots(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* h, double* w,
                        double* partials, unsigned* counter, double* out) {
  int grid = red_grid(n);
  switch (k) {
#define X(K) \
  case K: k_update_dots<K><<<grid, kThreads, 0, s>>>(n, V, ldv, h, w, partials, counter, out); break;
    VEM_K_CASES(X)
#undef X
    default: throw Error{VEM_EINVAL, "too many basis vectors"};
  }
}

void launch_update_norm(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* h, double* w,
                        double* partials, unsigned* counter, double* out) {
  int grid = red_grid(n);
  switch (k) {
#define X(K) \
  case K: k_update_norm<K><<<grid, kThreads, 0, s>>>(n, V, ldv, h, w, partials, counter, out); break;
    VEM_K_CASES(X)
#undef X
    default: throw Error{VEM_EINVAL, "too many basis vectors"};
  }
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
void launch_sum(hipStream_t s, int64_t n, const double* x, double* partials, unsigned* counter, double* out) {
  k_sum<<<red_grid(n), kThreads, 0, s>>>(n, x, partials, counter, out);
}

void launch_pcg_init(hipStream_t s, int64_t n, const double* b, const double* dinv, double* x, double* r, double* z,
                     double* p, PcgState* st, double tol, int maxit, double* partials, unsigned* counter) {
  k_pcg_init<<<red_grid(n), kThreads, 0, s>>>(n, b, dinv, x, r, z, p, st, tol * tol, maxit, partials, counter);
}

void launch_pcg_iter(hipStream_t s, int lanes, int64_t n, const int* rowptr, const int* col, const double* val,
                     const double* dinv, double* x, double* r, double* z, double* p, double* q, PcgState* st,
                     double* partials, unsigned* counter) {
  int grid_spmv = red_grid(n * lanes);
  switch (lanes) {
#define X(L)                                                                                                     \
  case L:                                                                                                        \
    k_pcg_spmv<L><<<grid_spmv, kThreads, 0, s>>>(n, rowptr, col, val, p, q, st, partials, counter);              \
    break;
    X(2) X(4) X(8) X(16) X(32) X(64)
#undef X
    default: throw Error{VEM_EINVAL, "bad lanes per row"};
  }
  k_pcg_update<<<red_grid(n), kThreads, 0, s>>>(n, x, r, z, q, p, dinv, st, partials, counter);
  k_pcg_dir<<<stream_grid(n), kThreads, 0, s>>>(n, z, p, st);
}

}  // namespace vem
