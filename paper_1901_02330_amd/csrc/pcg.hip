// The inner Jacobi-preconditioned conjugate gradients of the block preconditioners,
// pipelined so that one kernel performs one iteration.
#include <algorithm>
#include <type_traits>

#include <hip/hip_ext.h>

#include <vector>

#include "krylov_device.h"

namespace vem {
namespace {

// ---- inner Jacobi-preconditioned CG, pipelined: one kernel per iteration ------------------
// Pipelined CG (Ghysels & Vanroose) overlaps the two dot products of an
// iteration with its matrix-vector product, so one kernel per iteration
// suffices: it sums the dot-product partials that the previous kernel left
// (every block in the same order, hence the same scalars everywhere), forms
// alpha and beta, performs the product and every vector update, and writes
// the partials of the next iteration's dots.  With the Jacobi preconditioner
// D^{-1} the preconditioned vectors are diagonal scalings (u = D^{-1} r,
// q = D^{-1} s, m = D^{-1} w), and the product A D^{-1} w uses the
// column-scaled copy A D^{-1}, so only r, w, s, z, p, x are stored; w
// alternates between two buffers because neighbours read it while its owner
// updates it.  Iteration i, with gamma = r.D^{-1}r, delta = w.D^{-1}r:
//   beta = gamma_i / gamma_{i-1},  alpha = gamma_i / (delta - beta gamma_i / alpha_{i-1})
//   n = (A D^{-1}) w,  z = n + beta z,  s = w + beta s,  p = D^{-1} r + beta p,
//   x += alpha p,  r -= alpha s,  w -= alpha z.
// The stopping test is gamma_i <= tol^2 gamma_0, as for the plain algorithm.
template <typename T>
struct PcgViewT {
  T* __restrict__ x;
  T* __restrict__ r;
  T* __restrict__ z;
  T* __restrict__ s;
  T* __restrict__ p;
  T* __restrict__ w0;
  T* __restrict__ w1;
  const T* __restrict__ dinv;
};

// w = (A D^{-1}) b, x = 0, r = b; partials of gamma_0, delta_0 (slot 0).  b is FP64 and is
// rounded to T element by element (also where it is gathered).
template <typename T, int kBlock, int kRow>
__global__ void __launch_bounds__(kBlock) k_ppcg_init(SellViewT<T> Ac, PcgViewT<T> v,
                                                           const double* __restrict__ b, PcgState* st, double tol2,
                                                           int maxit, double* __restrict__ part) {
  double acc[2] = {0.0, 0.0};
  for (int64_t row = xcd_block_n<kBlock>() * kBlock + threadIdx.x; row < Ac.rows;
       row += (int64_t)gridDim.x * kBlock) {
    const T bi = (T)b[row], di = v.dinv[row];
    const T wi = sell_row<kRow>(Ac, row, b);
    v.x[row] = T(0);
    v.r[row] = bi;
    v.w0[row] = wi;
    acc[0] += (double)bi * (double)bi * (double)di;
    acc[1] += (double)wi * (double)bi * (double)di;
  }
  block_partials<2, kBlock>(acc, part);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->gamma[0] = st->gamma[1] = 0.0;
    st->alpha[0] = st->alpha[1] = 0.0;
    st->gamma0 = 0.0;
    st->tol2 = tol2;
    st->count = 0;
    st->maxit = maxit;
    st->done = maxit <= 0 ? 1 : 0;
  }
}

// One pipelined CG iteration.  Vectors and matrix values in T; scalars and dot products in FP64.
template <typename T, bool kFirst, int kBlock, int kRow>
__global__ void __launch_bounds__(kBlock) k_ppcg_iter(int parity, SellViewT<T> Ac, PcgViewT<T> v, PcgState* st,
                                                           double* __restrict__ part) {
  const int P = gridDim.x;
  const int cur = parity;
  const T* __restrict__ win = cur ? v.w1 : v.w0;
  T* __restrict__ wout = cur ? v.w0 : v.w1;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  int64_t row = xcd_block_n<kBlock>() * kBlock + threadIdx.x;
  // The product and the old vector entries do not depend on this iteration's
  // scalars: their loads are issued first and are in flight while the block sums
  // the partials of gamma and delta left by the previous iteration.
  T n = T(0), wi = T(0), di = T(0), ri = T(0), zo = T(0), so = T(0), po = T(0), xo = T(0);
  auto load = [&](int64_t i) {
    n = sell_row<kRow>(Ac, i, win);
    wi = win[i];
    di = v.dinv[i];
    ri = v.r[i];
    xo = v.x[i];
    if (!kFirst) {
      zo = v.z[i];
      so = v.s[i];
      po = v.p[i];
    }
  };
  if (row < Ac.rows) load(row);
  const int was_done = st->done;
  double gd[2];
  block_sum_partials2<kBlock>(part + (size_t)cur * 2 * P, P, gd);
  if (was_done) return;
  const double gamma = gd[0], delta = gd[1];
  double gamma0, beta, alpha;
  if (kFirst) {
    gamma0 = gamma;
    beta = 0.0;
    alpha = gamma / delta;
  } else {
    gamma0 = st->gamma0;
    beta = gamma / st->gamma[1 - cur];
    alpha = gamma / (delta - beta * gamma / st->alpha[1 - cur]);
  }
  int done = 0;
  if (!(gamma > st->tol2 * gamma0)) done = 1;
  else if (!(alpha > 0.0) || !isfinite(alpha)) done = 2;  // loss of positivity: keep the iterate
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (kFirst) st->gamma0 = gamma0;
    st->gamma[cur] = gamma;
    st->alpha[cur] = alpha;
    if (done) st->done = done;
  }
  if (done) return;
  const T a = (T)alpha, bt = (T)beta;
  double acc[2] = {0.0, 0.0};
  while (row < Ac.rows) {
    T zz, ss, pp;
    if (kFirst) {
      zz = n;
      ss = wi;
      pp = di * ri;
    } else {
      zz = n + bt * zo;
      ss = wi + bt * so;
      pp = di * ri + bt * po;
    }
    v.z[row] = zz;
    v.s[row] = ss;
    v.p[row] = pp;
    v.x[row] = xo + a * pp;
    const T rn = ri - a * ss;
    const T wn = wi - a * zz;
    v.r[row] = rn;
    wout[row] = wn;
    acc[0] += (double)rn * (double)rn * (double)di;
    acc[1] += (double)wn * (double)rn * (double)di;
    row += stride;
    if (row < Ac.rows) load(row);
  }
  block_partials<2, kBlock>(acc, part + (size_t)(1 - cur) * 2 * P);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->count += 1;
    st->total += 1;
  }
}

template <typename T>
PcgViewT<T> pview(const PcgWorkT<T>& w) {
  return {w.x, w.r, w.z, w.s, w.p, w.w0, w.w1, w.dinv};
}

template <typename T, int kBlock, int kRow>
void pcg_init_as(hipStream_t s, SellViewT<T> Av, const PcgWorkT<T>& w, const double* b, PcgState* st, double tol,
                 int maxit, double* part) {
  k_ppcg_init<T, kBlock, kRow><<<pcg_grid(Av.rows, kBlock), kBlock, 0, s>>>(Av, pview(w), b, st, tol * tol, maxit,
                                                                              part);
}

template <typename T, int kBlock, int kRow>
void pcg_iter_as(hipStream_t s, int i, SellViewT<T> Av, const PcgWorkT<T>& w, PcgState* st, double* part) {
  const int P = pcg_grid(Av.rows, kBlock);
  if (i == 0)
    k_ppcg_iter<T, true, kBlock, kRow><<<P, kBlock, 0, s>>>(0, Av, pview(w), st, part);
  else
    k_ppcg_iter<T, false, kBlock, kRow><<<P, kBlock, 0, s>>>(i & 1, Av, pview(w), st, part);
}

// Launch shape: 1024-thread blocks when every row has a thread, 256-thread blocks when threads
// loop over rows (their barriers hold fewer waves).  One-row-per-thread launches take the
// short-row product when no slice is longer than kShortRow (measured on the 64^3 cube: S, 7 per
// row, 10.95 -> 10.53 us per iteration; rows of 11-13 entries were slower with it, 31.5 ->
// 33.9 us for A_gamma, so longer rows keep the plain loop), and its fixed-count form where every
// slice was padded to one length.
template <typename T>
void pcg_init_sel(hipStream_t s, const Sell& A, SellViewT<T> Av, const PcgWorkT<T>& w, const double* b,
                  PcgState* st, double tol, int maxit, double* part) {
  if (A.rows > kPcgMaxThreads)  // threads loop over rows
    pcg_init_as<T, 256, kRowAny>(s, Av, w, b, st, tol, maxit, part);
  else
    with_row_form(row_form(A), [&](auto R) { pcg_init_as<T, 1024, decltype(R)::value>(s, Av, w, b, st, tol, maxit, part); });
}

template <typename T>
void pcg_iter_sel(hipStream_t s, int i, const Sell& A, SellViewT<T> Av, const PcgWorkT<T>& w, PcgState* st,
                  double* part) {
  if (A.rows > kPcgMaxThreads)
    pcg_iter_as<T, 256, kRowAny>(s, i, Av, w, st, part);
  else
    with_row_form(row_form(A), [&](auto R) { pcg_iter_as<T, 1024, decltype(R)::value>(s, i, Av, w, st, part); });
}

// ---- inner Chebyshev-Jacobi: a fixed polynomial in D^{-1}A, no reductions ----------------------
// Chebyshev iteration for D^{-1}A x = D^{-1}b on [lo, hi] = [c hi, hi], from x = 0: with
// theta = (hi + lo) / 2, delta = (hi - lo) / 2, sigma = theta / delta, rho_0 = 1 / sigma and
// rho_{k+1} = 1 / (2 sigma - rho_k), the iterates satisfy x_1 = D^{-1}b / theta and
//   x_{k+2} = x_{k+1} + rho_{k+1} rho_k (x_{k+1} - x_k) + (2 rho_{k+1} / delta) D^{-1}(b - A x_{k+1}).
// The kernels run it in y = D x, on the column-scaled values A D^{-1} (the same spectrum):
//   y_1 = b / theta,  y_{k+2} = y_{k+1} + c1_k (y_{k+1} - y_k) + c2_k (b - A D^{-1} y_{k+1}),
// and the last product writes x = D^{-1} y.  A product gathers one vector (y_{k+1}) and reads y_k and
// b at its own row; y_{k+2} overwrites y_k (each row reads and writes only its own entry of that
// buffer), so the two iterates alternate between two buffers, and D^{-1} is read by the last product
// only.  The residual is formed from the iterate at every step rather than carried.  The rho_k
// depend on c only, so the host forms every coefficient in units of 1/hi, and the kernels scale them
// by the device-resident 1/hi (the Gershgorin bound of D^{-1}A, taken when the values are built):
// nothing is read back.  m products give x_{m+1}, a polynomial of degree m in D^{-1}A applied to
// D^{-1}b.  The first product also sets the inner-solve counters (no separate start kernel).
constexpr int kChebBlock = 1024;  // the Chebyshev products' block size (every launch)
template <typename T, int kRow, bool kFirst, bool kLast>
__global__ void __launch_bounds__(kChebBlock) k_cheb_iter(SellViewT<T> Acs, const T* __restrict__ dinv,
                                                    const double* __restrict__ b, T* __restrict__ bT,
                                                    const T* __restrict__ ycur, T* yprev, T* yout,
                                                    T* __restrict__ x,
                                                    const double* __restrict__ inv_hi, double c0u, double c1,
                                                    double c2u, PcgState* st, int m, ScaleJob side) {
  const T t1 = (T)c1;
  if (kFirst && blockIdx.x == 0 && threadIdx.x == 0) {
    st->count = m;
    st->total += m;
    st->done = 0;
  }
  // The side job's first kSide entries per thread are loaded before the product's rows, so that their
  // loads are in flight while the rows' dependent loads proceed; they are stored after the rows.  The
  // block size is the launch's constant kChebBlock (not read from the dispatch: a vector load of it
  // would be ordered behind those loads).
  constexpr int kSide = 4;
  const int64_t tid = (int64_t)blockIdx.x * kChebBlock + threadIdx.x, nthr = (int64_t)gridDim.x * kChebBlock;
  double sx[kSide], sd[kSide];
  if constexpr (kFirst) {
    if (side.n > 0) {  // the same on every thread; the loads take no branch (slots past n reload entry n - 1)
#pragma unroll
      for (int u = 0; u < kSide; ++u) {
        const int64_t i = tid + u * nthr, j = i < side.n ? i : side.n - 1;
        sx[u] = side.x[j];
        sd[u] = side.d[j];
      }
    }
  }
  auto one_row = [&](int64_t row) {
    T yn;
    if constexpr (kFirst) {
      // y_1 = c0 b and y_0 = 0, with A D^{-1} y_1 = c0 (A D^{-1} b)
      const T bi = (T)b[row];
      const T ab = sell_row<kRow>(Acs, row, b);
      const double ih = inv_hi[0];
      const T c0 = (T)(c0u * ih), c2 = (T)(c2u * ih);
      const T y1 = c0 * bi;
      yn = y1 + t1 * y1 + c2 * (bi - c0 * ab);
      if (!kLast) {
        yprev[row] = y1;
        if (bT) bT[row] = bi;
      }
    } else {
      // the row's own entries first: their loads overlap the product's
      const T yj = ycur[row], yp = yprev[row];
      const T bi = bT ? bT[row] : (T)b[row];
      const T ay = sell_row<kRow>(Acs, row, ycur);
      const T c2 = (T)(c2u * inv_hi[0]);
      yn = yj + t1 * (yj - yp) + c2 * (bi - ay);
    }
    if constexpr (kLast)
      x[row] = dinv[row] * yn;
    else
      yout[row] = yn;
  };
  const int64_t row0 = xcd_block_of(kChebBlock) * kChebBlock + threadIdx.x;
  if constexpr (kRow == kRowAny) {
    for (int64_t row = row0; row < Acs.rows; row += nthr) one_row(row);
  } else if (row0 < Acs.rows) {
    // the short-row forms are launched with a thread for every row: no loop, so that nothing is
    // hoisted ahead of the row's first loads
    one_row(row0);
  }
  if constexpr (kFirst) {
#pragma unroll
    for (int u = 0; u < kSide; ++u) {
      const int64_t i = tid + u * nthr;
      if (i < side.n) side.y[i] = sd[u] * sx[u];
    }
    for (int64_t i = tid + kSide * nthr; i < side.n; i += nthr) side.y[i] = side.d[i] * side.x[i];
  }
}

// Gershgorin bound of D^{-1}A (max over rows of sum_j |a_ij| / a_ii): block maxima, then their
// maximum; out[0] = 1 / bound.
__global__ void __launch_bounds__(256) k_gersh(SellView A, const double* __restrict__ dinv,
                                               double* __restrict__ part) {
  __shared__ double sh[4];
  double m = 0.0;
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < A.rows;
       row += (int64_t)gridDim.x * blockDim.x) {
    const int64_t sl = row >> 6, base = A.slice_ptr[sl] + (row & 63);
    double t = 0.0;
    for (int k = 0; k < A.slice_len[sl]; ++k) t += fabs(A.val[base + 64 * k]);
    t *= fabs(dinv[row]);
    m = t > m ? t : m;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double q = __shfl_down(m, o, 64);
    m = q > m ? q : m;
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = sh[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = sh[w] > b ? sh[w] : b;
    part[blockIdx.x] = b;
  }
}

// one 256-thread block: the maximum of the block maxima (a single thread walking 1024 partials took
// 88 us)
__global__ void __launch_bounds__(256) k_gersh_final(int nparts, const double* __restrict__ part,
                                                     double* __restrict__ out) {
  __shared__ double sh[4];
  double m = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) m = part[i] > m ? part[i] : m;
  for (int o = 32; o > 0; o >>= 1) {
    const double q = __shfl_down(m, o, 64);
    m = q > m ? q : m;
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = sh[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = sh[w] > b ? sh[w] : b;
    out[0] = b > 0.0 ? 1.0 / b : 0.0;
  }
}

template <typename T, int kRow>
void cheb_iter_as(hipStream_t s, int k, int m, SellViewT<T> Acs, const T* dinv, const double* b, T* bT,
                  const T* ycur, T* yprev, T* yout, T* x, const double* inv_hi, double c0u, double c1, double c2u,
                  PcgState* st, const ScaleJob& side) {
  const int G = pcg_grid(Acs.rows, kChebBlock);
  const bool first = k == 0, last = k == m - 1;
  if (first && last)
    k_cheb_iter<T, kRow, true, true><<<G, kChebBlock, 0, s>>>(Acs, dinv, b, bT, ycur, yprev, yout, x, inv_hi, c0u, c1,
                                                          c2u, st, m, side);
  else if (first)
    k_cheb_iter<T, kRow, true, false><<<G, kChebBlock, 0, s>>>(Acs, dinv, b, bT, ycur, yprev, yout, x, inv_hi, c0u, c1,
                                                           c2u, st, m, side);
  else if (last)
    k_cheb_iter<T, kRow, false, true><<<G, kChebBlock, 0, s>>>(Acs, dinv, b, bT, ycur, yprev, yout, x, inv_hi, c0u, c1,
                                                           c2u, st, m, side);
  else
    k_cheb_iter<T, kRow, false, false><<<G, kChebBlock, 0, s>>>(Acs, dinv, b, bT, ycur, yprev, yout, x, inv_hi, c0u,
                                                            c1, c2u, st, m, side);
}

}  // namespace

template <typename T>
void launch_cheb(hipStream_t s, const Sell& A, const PcgWorkT<T>& w, const double* b, const double* inv_hi,
                 double c, int m, PcgState* st, const ScaleJob& side) {
  VEM_REQUIRE(c > 0.0 && c < 1.0 && m >= 1, VEM_EINVAL, "Chebyshev interval or degree out of range");
  const T* vcs = std::is_same<T, float>::value ? (const T*)(const void*)A.val32_cs.p : (const T*)(const void*)A.val_cs.p;
  VEM_REQUIRE(vcs != nullptr, VEM_EINVAL, "Chebyshev inner solve without the column-scaled values");
  const SellViewT<T> Acs{A.rows, A.slice_ptr, A.slice_len, A.col, vcs};
  // b rounded to T once (FP32), or read in FP64 where T is double
  T* bT = std::is_same<T, float>::value ? w.r : nullptr;
  const double sigma = (1.0 + c) / (1.0 - c);
  const double c0u = 2.0 / (1.0 + c);  // 1 / theta, theta = hi (1 + c) / 2
  double rho = 1.0 / sigma;
  T* ybuf[2] = {w.p, w.s};
  const int form = A.rows <= kPcgMaxThreads ? row_form(A) : kRowAny;
  for (int k = 0; k < m; ++k) {
    const double rho1 = 1.0 / (2.0 * sigma - rho);
    const double c1 = rho1 * rho, c2u = 4.0 * rho1 / (1.0 - c);  // 2 rho_{k+1} / delta, delta = hi (1 - c) / 2
    // after product k, y_{k+2} is in ybuf[k & 1] and y_{k+1} in ybuf[(k + 1) & 1]
    const T* ycur = k == 0 ? nullptr : ybuf[(k + 1) & 1];
    T* yprev = k == 0 ? ybuf[1] : ybuf[k & 1];
    T* yout = ybuf[k & 1];
    with_row_form(form, [&](auto R) {
      cheb_iter_as<T, decltype(R)::value>(s, k, m, Acs, w.dinv, b, bT, ycur, yprev, yout, w.x, inv_hi, c0u, c1, c2u,
                                          st, k == 0 ? side : ScaleJob{});
    });
    rho = rho1;
  }
}
// Mean duration (ms) of `reps` Chebyshev products of the middle form (the form of every product of a
// solve but its first and last), each launched with start and stop events of its own: the kernels'
// own time, without the dispatch gaps between back-to-back launches.  A degree-2 solve sets up the
// two iterates first; the timed products continue its recurrence.
template <typename T>
double time_cheb_products(hipStream_t s, const Sell& A, const PcgWorkT<T>& w, const double* b,
                          const double* inv_hi, double c, int reps, PcgState* st) {
  VEM_REQUIRE(reps >= 1, VEM_EINVAL, "at least one timed product");
  launch_cheb<T>(s, A, w, b, inv_hi, c, 2, st);
  const T* vcs = std::is_same<T, float>::value ? (const T*)(const void*)A.val32_cs.p : (const T*)(const void*)A.val_cs.p;
  const SellViewT<T> Acs{A.rows, A.slice_ptr, A.slice_len, A.col, vcs};
  T* bT = std::is_same<T, float>::value ? w.r : nullptr;
  const double sigma = (1.0 + c) / (1.0 - c), c0u = 2.0 / (1.0 + c);
  double rho = 1.0 / sigma;
  rho = 1.0 / (2.0 * sigma - rho);  // the degree-2 solve's two steps
  rho = 1.0 / (2.0 * sigma - rho);
  const int form = A.rows <= kPcgMaxThreads ? row_form(A) : kRowAny;
  const int G = pcg_grid(Acs.rows, kChebBlock);
  std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
  double total = 0.0;
  try {
    for (auto& e : ev) VEM_HIP(hipEventCreate(&e));
    T* ybuf[2] = {w.p, w.s};
    for (int r = 0; r < reps; ++r) {
      const int k = r + 1;  // after the set-up, y_2 is in ybuf[0] and y_1 in ybuf[1]
      const double rho1 = 1.0 / (2.0 * sigma - rho);
      const double c1 = rho1 * rho, c2u = 4.0 * rho1 / (1.0 - c);
      rho = rho1;
      const T* ycur = ybuf[(k + 1) & 1];
      T* ynext = ybuf[k & 1];
      with_row_form(form, [&](auto R) {
        hipExtLaunchKernelGGL(k_cheb_iter<T, decltype(R)::value, false, false>, dim3(G), dim3(kChebBlock), 0, s, ev[2 * r],
                              ev[2 * r + 1], 0, Acs, (const T*)w.dinv, b, bT, ycur, ynext, ynext, w.x, inv_hi, c0u,
                              c1, c2u, st, reps, ScaleJob{});
      });
      VEM_HIP(hipGetLastError());
    }
    VEM_HIP(hipEventSynchronize(ev.back()));
    for (int r = 0; r < reps; ++r) {
      float ms = 0.f;
      VEM_HIP(hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]));
      total += ms;
    }
  } catch (...) {
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
    throw;
  }
  for (auto e : ev) (void)hipEventDestroy(e);
  return total / reps;
}
template double time_cheb_products<double>(hipStream_t, const Sell&, const PcgWorkT<double>&, const double*,
                                           const double*, double, int, PcgState*);
template double time_cheb_products<float>(hipStream_t, const Sell&, const PcgWorkT<float>&, const double*,
                                          const double*, double, int, PcgState*);

template void launch_cheb<double>(hipStream_t, const Sell&, const PcgWorkT<double>&, const double*, const double*,
                                  double, int, PcgState*, const ScaleJob&);
template void launch_cheb<float>(hipStream_t, const Sell&, const PcgWorkT<float>&, const double*, const double*,
                                 double, int, PcgState*, const ScaleJob&);

void launch_gershgorin(hipStream_t s, const Sell& A, const double* dinv, double* part, double* inv_hi) {
  const int G = (int)std::min<int64_t>(1024, (A.rows + 255) / 256);
  k_gersh<<<G > 0 ? G : 1, 256, 0, s>>>(view(A), dinv, part);
  k_gersh_final<<<1, 256, 0, s>>>(G > 0 ? G : 1, part, inv_hi);
}

void launch_pcg_init(hipStream_t s, const Sell& A, const PcgWork& w, const double* b, PcgState* st, double tol,
                     int maxit, double* part) {
  pcg_init_sel<double>(s, A, view_cs(A), w, b, st, tol, maxit, part);
}

void launch_pcg_iter(hipStream_t s, int i, const Sell& A, const PcgWork& w, PcgState* st, double* part) {
  pcg_iter_sel<double>(s, i, A, view_cs(A), w, st, part);
}

void launch_pcg_init32p(hipStream_t s, const Sell& A, const PcgWork32& w, const double* b, PcgState* st, double tol,
                        int maxit, double* part) {
  pcg_init_sel<float>(s, A, view_cs32(A), w, b, st, tol, maxit, part);
}

void launch_pcg_iter32p(hipStream_t s, int i, const Sell& A, const PcgWork32& w, PcgState* st, double* part) {
  pcg_iter_sel<float>(s, i, A, view_cs32(A), w, st, part);
}

}  // namespace vem
