// Edge-patch additive Schwarz preconditioner for the regularised block of Block-Reg
// (Section 5, eq. block_diag: A_gamma = M + B^T B / gamma).
//
// gamma^{-1} B^T B dominates A_gamma (B^T B / gamma ~ h^2 against M ~ h^3 per entry), and it
// vanishes on divergence-free fluxes, so the small eigenvalues of A_gamma belong to fluxes that
// circulate.  A flux through the faces around one mesh edge, turning about the edge, is
// divergence-free in every cell it touches: the patches of faces that share an edge carry these
// local circulations, and a Jacobi scaling (one DOF at a time) never sees them.
//
// Set-up (this file):
//  - the mesh edges, as the distinct vertex pairs of the face loops (a stable radix sort of the
//    pair keys; each edge lists its faces in ascending order);
//  - order k: the interior DOFs of a cell couple only to that cell's DOFs (A_gamma is a sum of
//    cell matrices), so they are condensed cell by cell: F = A_ff - A_fi A_ii^{-1} A_if on the
//    face DOFs, with W = A_fi A_ii^{-1} and A_ii^{-1} kept for the right-hand side and the
//    back-substitution.  At the lowest order there are no interior DOFs and F = A_gamma;
//  - per edge e, the inverse of F restricted to the DOFs of its faces (dense, Gauss-Jordan in
//    LDS, one wavefront per edge);
//  - P = sum_e R_e^T F_e^{-1} R_e assembled by gathering: each row sums the inverses of the
//    edges of its face, in the face loop's order (no atomics, same bits every run).
// The CG on F preconditioned by P is in krylov.hip.
#include <hipcub/hipcub.hpp>

#include <climits>

#include "vem_internal.h"

namespace vem {
namespace {

constexpr int kT = 256;
inline int grid(int64_t n) { return (int)((n + kT - 1) / kT); }
// faces that share an edge with one face (its own included); more is rejected
constexpr int kMaxNb = 160;
// DOFs of one edge patch (faces around the edge times face DOFs); more is rejected
constexpr int kMaxPatchDof = 80;
// LDS of the per-cell staged kernels of the inner solve's right-hand side and back-substitution;
// cells too large for it take the unstaged kernels
constexpr size_t kCellStageLds = 48 * 1024;

__global__ void k_inc_face(int nf, const int* __restrict__ fptr, int* __restrict__ inc_face) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  for (int i = fptr[f]; i < fptr[f + 1]; ++i) inc_face[i] = f;
}

// key of the loop edge (v_a, v_{a+1}) of every face-loop incidence: min * nv + max
__global__ void k_loop_keys(int nf, int nv, const int* __restrict__ fptr, const int* __restrict__ fvtx,
                            unsigned long long* __restrict__ keys, int* __restrict__ vals) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int b = fptr[f], n = fptr[f + 1] - b;
  for (int a = 0; a < n; ++a) {
    const int v = fvtx[b + a], w = fvtx[b + (a + 1 == n ? 0 : a + 1)];
    const unsigned long long lo = v < w ? v : w, hi = v < w ? w : v;
    keys[b + a] = lo * (unsigned long long)nv + hi;
    vals[b + a] = b + a;
  }
}

__global__ void k_edge_flags(int64_t n, const unsigned long long* __restrict__ keys, int* __restrict__ flag) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) flag[j] = (j == 0 || keys[j] != keys[j - 1]) ? 1 : 0;
}

// edge ids from the flags' exclusive sum; faces of each edge; edge of each incidence
__global__ void k_edge_lists(int64_t n, const int* __restrict__ flag, const int* __restrict__ pos,
                             const int* __restrict__ vals, const int* __restrict__ inc_face, int* __restrict__ edge_ptr,
                             int* __restrict__ edge_face, int* __restrict__ face_edge, int ne) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int e = pos[j] + flag[j] - 1;
  if (flag[j]) edge_ptr[e] = (int)j;
  const int i = vals[j];
  edge_face[j] = inc_face[i];
  face_edge[i] = e;
  if (j == n - 1) edge_ptr[ne] = (int)n;
}

__global__ void k_max_patch(int ne, const int* __restrict__ edge_ptr, int* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  int m = e < ne ? edge_ptr[e + 1] - edge_ptr[e] : 0;
  for (int o = 32; o > 0; o >>= 1) {
    const int t = __shfl_xor(m, o, 64);
    m = t > m ? t : m;
  }
  if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(out, m);
}

// Faces sharing an edge with face f (f included), ascending and unique; returns the count, or -1
// past kMaxNb.
__device__ inline int face_nbrs(int f, const int* __restrict__ fptr, const int* __restrict__ face_edge,
                                const int* __restrict__ edge_ptr, const int* __restrict__ edge_face, int* nb) {
  int n = 0;
  for (int i = fptr[f]; i < fptr[f + 1]; ++i) {
    const int e = face_edge[i];
    for (int j = edge_ptr[e]; j < edge_ptr[e + 1]; ++j) {
      const int g = edge_face[j];
      int k = n;
      bool dup = false;
      for (int q = 0; q < n; ++q)
        if (nb[q] == g) dup = true;
      if (dup) continue;
      if (n == kMaxNb) return -1;
      while (k > 0 && nb[k - 1] > g) {
        nb[k] = nb[k - 1];
        --k;
      }
      nb[k] = g;
      ++n;
    }
  }
  return n;
}

__global__ void k_p_rowlen(int nf, int nfd, const int* __restrict__ fptr, const int* __restrict__ face_edge,
                           const int* __restrict__ edge_ptr, const int* __restrict__ edge_face, int* __restrict__ len,
                           int* __restrict__ err) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int nb[kMaxNb];
  const int n = face_nbrs(f, fptr, face_edge, edge_ptr, edge_face, nb);
  if (n < 0) *err = 1;
  for (int b = 0; b < nfd; ++b) len[(int64_t)f * nfd + b] = n < 0 ? 0 : n * nfd;
}

__global__ void k_p_cols(int nf, int nfd, const int* __restrict__ fptr, const int* __restrict__ face_edge,
                         const int* __restrict__ edge_ptr, const int* __restrict__ edge_face,
                         const int* __restrict__ rowptr, int* __restrict__ col) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int nb[kMaxNb];
  const int n = face_nbrs(f, fptr, face_edge, edge_ptr, edge_face, nb);
  if (n < 0) return;
  for (int b = 0; b < nfd; ++b) {
    int o = rowptr[(int64_t)f * nfd + b];
    for (int t = 0; t < n; ++t)
      for (int c = 0; c < nfd; ++c) col[o++] = nb[t] * nfd + c;
  }
}

__global__ void k_patch_size(int ne, int nfd, const int* __restrict__ edge_ptr, int64_t* __restrict__ sz) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int64_t n = (int64_t)(edge_ptr[e + 1] - edge_ptr[e]) * nfd;
  sz[e] = n * n;
}

// face system pattern (order k): the face-DOF columns of A_gamma's face-DOF rows (interior DOFs are
// numbered after every face DOF, so they end each row)
__device__ inline int lower_bound_i32(const int* __restrict__ a, int n, int v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ void k_fc_rowlen(int64_t nF, const int* __restrict__ Aptr, const int* __restrict__ Acol,
                            int* __restrict__ len) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nF) return;
  len[r] = lower_bound_i32(Acol + Aptr[r], Aptr[r + 1] - Aptr[r], (int)nF);
}

__global__ void k_fc_cols(int64_t nF, const int* __restrict__ Aptr, const int* __restrict__ Acol,
                          const int* __restrict__ Fptr, int* __restrict__ Fcol) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nF) return;
  const int n = Fptr[r + 1] - Fptr[r];
  for (int k = 0; k < n; ++k) Fcol[Fptr[r] + k] = Acol[Aptr[r] + k];
}

// ---- values ----------------------------------------------------------------------------------

__device__ inline bool fixed_face_dof(const int* bnd, int nfd, int64_t gid) { return bnd && bnd[gid / nfd]; }

// Storage position of the k-th entry (in column order) of row r: SELL-64 slots, or face blocks
// (the columns of an order-k face row come in whole faces, nfd at a time, so entry k lies in block
// k / nfd at column c = k mod nfd).
struct Slots {
  const int* slice_ptr;  // SELL-64 (bptr null)
  const int* bptr;       // face blocks
  int nfd;
  __device__ int64_t at(int64_t r, int k) const {
    if (bptr) {
      const int64_t f = r / nfd;
      const int i = (int)(r - f * nfd), j = k / nfd, c = k - j * nfd;
      return (((int64_t)bptr[f] + j) * nfd + i) * nfd + c;
    }
    return (int64_t)slice_ptr[r >> 6] + (r & 63) + 64 * (int64_t)k;
  }
};
inline Slots slots_of(const Sell& S) { return {S.slice_ptr.p, nullptr, 1}; }
inline Slots slots_of(const FaceBlocks& B) { return {nullptr, B.bptr.p, B.nfd}; }

// Local A_gamma entry (i, j) of cell P in the cell's outward orientation:
// nu_P M1_P[i][j] + gamma^{-1} sum_q B_P[q][i] B_P[q][j].
__device__ inline double local_a(const double* __restrict__ M, const double* __restrict__ Bp, int nd, int npd,
                                 double nu, double ig, int i, int j) {
  double t = 0.0;
  for (int q = 0; q < npd; ++q) t += Bp[q * nd + i] * Bp[q * nd + j];
  return nu * M[(int64_t)i * nd + j] + ig * t;
}

// In-place inverse of the SPD n x n matrix a (row-major, in LDS) by Gauss-Jordan elimination
// without pivoting; rk, ck: scratch rows of n.  All threads of the block take part.
__device__ inline void gj_invert(double* a, double* rk, double* ck, int n) {
  for (int k = 0; k < n; ++k) {
    __syncthreads();
    const double p = 1.0 / a[k * n + k];
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
      rk[t] = a[k * n + t] * p;
      ck[t] = a[t * n + k];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
      const int i = t / n, j = t - i * n;
      if (i == k && j == k)
        a[t] = p;
      else if (i == k)
        a[t] = rk[j];
      else if (j == k)
        a[t] = -ck[i] * p;
      else
        a[t] -= ck[i] * rk[j];
    }
  }
  __syncthreads();
}

// Per cell (one block): A_ii^{-1} and W = A_fi A_ii^{-1} (rows of prescribed face DOFs zero: A_gamma
// holds identity rows and columns there); with Sp, also the condensed cell matrix
// S_P = A_ff - W A_if (Fn x Fn, row-major at sp_ptr[P]), A_if and W staged in LDS.  Each S_P entry is
// formed as the face system's gather formed it from the local matrices (the same operands in the
// same order), so the face system is the same either way.
// LDS: nint^2 + 2 nint doubles, plus 2 nint fn_max with Sp.
__global__ void k_cell_condense(DofLayout L, const int* __restrict__ cptr, const int* __restrict__ cface,
                                const int64_t* __restrict__ lmat_ptr, const double* __restrict__ M1,
                                const int64_t* __restrict__ lb_ptr, const double* __restrict__ Bdiv1,
                                const double* __restrict__ nu, double ig, const int* __restrict__ bnd,
                                const int* __restrict__ ldof_ptr, double* __restrict__ Aiinv,
                                double* __restrict__ W, int fn_max, const int64_t* __restrict__ sp_ptr,
                                double* __restrict__ Sp) {
  extern __shared__ double sh[];
  const int P = blockIdx.x;
  const int ni = L.nint;
  double* a = sh;
  double* rk = sh + ni * ni;
  double* ck = rk + ni;
  double* aif = ck + ni;              // A_if[c][m] = A(m, interior c), nint x Fn (with Sp)
  double* wl = aif + ni * fn_max;     // W[l][c], Fn x nint (with Sp)
  const int F = cptr[P + 1] - cptr[P], Fn = F * L.nfd, nd = Fn + ni;
  const double* M = M1 + lmat_ptr[P];
  const double* Bp = Bdiv1 + lb_ptr[P];
  const double nuP = nu[P];
  for (int t = threadIdx.x; t < ni * ni; t += blockDim.x) {
    const int i = t / ni, j = t - i * ni;
    a[t] = local_a(M, Bp, nd, L.npd, nuP, ig, Fn + i, Fn + j);
  }
  if (Sp)
    for (int t = threadIdx.x; t < ni * Fn; t += blockDim.x) {
      const int c = t / Fn, m = t - c * Fn;
      aif[t] = local_a(M, Bp, nd, L.npd, nuP, ig, m, Fn + c);
    }
  gj_invert(a, rk, ck, ni);
  for (int t = threadIdx.x; t < ni * ni; t += blockDim.x) Aiinv[(int64_t)P * ni * ni + t] = a[t];
  const int64_t wo = ((int64_t)ldof_ptr[P] - (int64_t)P * ni) * ni;
  for (int l = threadIdx.x; l < Fn; l += blockDim.x) {
    const int j = l / L.nfd;
    const bool fixed = bnd && bnd[cface[cptr[P] + j]];
    double af[64];
    for (int b = 0; b < ni; ++b) af[b] = fixed ? 0.0 : local_a(M, Bp, nd, L.npd, nuP, ig, l, Fn + b);
    for (int c = 0; c < ni; ++c) {
      double t = 0.0;
      for (int b = 0; b < ni; ++b) t += af[b] * a[b * ni + c];
      W[wo + (int64_t)l * ni + c] = t;
      if (Sp) wl[l * ni + c] = t;
    }
  }
  if (!Sp) return;
  __syncthreads();
  double* out = Sp + sp_ptr[P];
  for (int t = threadIdx.x; t < Fn * Fn; t += blockDim.x) {
    const int l = t / Fn, m = t - l * Fn;
    double v = local_a(M, Bp, nd, L.npd, nuP, ig, l, m);
    for (int c = 0; c < ni; ++c) v -= wl[l * ni + c] * aif[c * Fn + m];
    out[t] = v;
  }
}

__global__ void k_cell_fn2(int nc, int nfd, const int* __restrict__ cptr, int64_t* __restrict__ len,
                           int* __restrict__ fmax) {
  const int P = blockIdx.x * blockDim.x + threadIdx.x;
  int f = 0;
  if (P < nc) {
    f = (cptr[P + 1] - cptr[P]) * nfd;
    len[P] = (int64_t)f * f;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const int t = __shfl_xor(f, o, 64);
    f = t > f ? t : f;
  }
  if ((threadIdx.x & 63) == 0 && f > 0) atomicMax(fmax, f);
}

// Face system values (order k): row r (face DOF) of F = sum over its cells of
// sigma_r sigma_g (A_ff - W A_if)[l_r][l_g], written to the SELL slots in column order.
__global__ void k_fc_values(DofLayout L, const int* __restrict__ cptr, const int* __restrict__ cface,
                            const int8_t* __restrict__ csign, const int* __restrict__ ldof_ptr,
                            const int* __restrict__ sorted_gid, const int* __restrict__ sorted_l,
                            const int* __restrict__ face_cell, const int* __restrict__ face_lidx,
                            const int64_t* __restrict__ lmat_ptr, const double* __restrict__ M1,
                            const int64_t* __restrict__ lb_ptr, const double* __restrict__ Bdiv1,
                            const double* __restrict__ nu, double ig, const int* __restrict__ bnd,
                            const double* __restrict__ W, const int64_t* __restrict__ sp_ptr,
                            const double* __restrict__ Sp, Slots Fs, double* __restrict__ Fval) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nF = (int64_t)L.nf * L.nfd;
  if (r >= nF) return;
  const int f = (int)(r / L.nfd), beta = (int)(r - (int64_t)f * L.nfd);
  const bool fixed_row = bnd && bnd[f];
  int P[2], lr[2], n = 0;
  for (int side = 0; side < 2; ++side) {
    const int c = face_cell[2 * f + side];
    if (c >= 0) {
      P[n] = c;
      lr[n] = face_lidx[2 * f + side] * L.nfd + beta;
      ++n;
    }
  }
  if (n == 2 && P[0] > P[1]) {
    int t = P[0];
    P[0] = P[1];
    P[1] = t;
    t = lr[0];
    lr[0] = lr[1];
    lr[1] = t;
  }
  int nd[2], Fn[2], na[2];
  double sr[2];
  const int* gl[2];
  const int* ll[2];
  int64_t wo[2];
  for (int c = 0; c < n; ++c) {
    const int F = cptr[P[c] + 1] - cptr[P[c]];
    Fn[c] = F * L.nfd;
    nd[c] = Fn[c] + L.nint;
    sr[c] = (double)csign[cptr[P[c]] + lr[c] / L.nfd];
    gl[c] = sorted_gid + ldof_ptr[P[c]];
    ll[c] = sorted_l + ldof_ptr[P[c]];
    na[c] = Fn[c];  // the face DOFs come first in the sorted list
    wo[c] = ((int64_t)ldof_ptr[P[c]] - (int64_t)P[c] * L.nint) * L.nint;
  }
  int k = 0, ia = 0, ib = 0;
  const int nb = n == 2 ? na[1] : 0;
  while (ia < na[0] || ib < nb) {
    const int ga = ia < na[0] ? gl[0][ia] : INT_MAX, gb = ib < nb ? gl[1][ib] : INT_MAX;
    const int g = ga < gb ? ga : gb;
    double v = 0.0;
    for (int c = 0; c < n; ++c) {
      int idx;
      if (c == 0) {
        if (ga != g) continue;
        idx = ia;
      } else {
        if (gb != g) continue;
        idx = ib;
      }
      const int lg = ll[c][idx];
      const double sg = (double)csign[cptr[P[c]] + lg / L.nfd];
      double t;
      if (Sp) {
        t = Sp[sp_ptr[P[c]] + (int64_t)lr[c] * Fn[c] + lg];
      } else {
        const double* M = M1 + lmat_ptr[P[c]];
        const double* Bp = Bdiv1 + lb_ptr[P[c]];
        const double nuP = nu[P[c]];
        t = local_a(M, Bp, nd[c], L.npd, nuP, ig, lr[c], lg);
        const bool fixed_col = bnd && bnd[g / L.nfd];
        if (!fixed_row && !fixed_col) {
          const double* Wr = W + wo[c] + (int64_t)lr[c] * L.nint;
          for (int a = 0; a < L.nint; ++a) t -= Wr[a] * local_a(M, Bp, nd[c], L.npd, nuP, ig, lg, Fn[c] + a);
        }
      }
      v += sr[c] * sg * t;
    }
    if (ga == g) ++ia;
    if (gb == g) ++ib;
    if (fixed_row || (bnd && bnd[g / L.nfd])) v = (g == r) ? 1.0 : 0.0;
    Fval[Fs.at(r, k++)] = v;
  }
}

// Entry (r, c) of a matrix given by its CSR pattern (sorted columns) and its stored values; 0 where
// the pattern has none.
__device__ inline double csr_entry(const int* __restrict__ rowptr, const int* __restrict__ col, Slots S,
                                   const double* __restrict__ val, int64_t r, int c) {
  const int b = rowptr[r], n = rowptr[r + 1] - b;
  const int k = lower_bound_i32(col + b, n, c);
  if (k >= n || col[b + k] != c) return 0.0;
  return val[S.at(r, k)];
}

// One block per edge: the face system restricted to the DOFs of the edge's faces, inverted.
__global__ void k_edge_inv(int ne, int nfd, const int* __restrict__ edge_ptr, const int* __restrict__ edge_face,
                           const int* __restrict__ Fptr, const int* __restrict__ Fcol, Slots Fs,
                           const double* __restrict__ Fval,
                           const int64_t* __restrict__ einv_ptr, double* __restrict__ einv) {
  extern __shared__ double sh[];
  const int e = blockIdx.x;
  if (e >= ne) return;
  const int m = edge_ptr[e + 1] - edge_ptr[e], n = m * nfd;
  const int* fe = edge_face + edge_ptr[e];
  double* a = sh;
  double* rk = sh + n * n;
  double* ck = rk + n;
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
    const int i = t / n, j = t - i * n;
    const int64_t gi = (int64_t)fe[i / nfd] * nfd + i % nfd;
    const int gj = fe[j / nfd] * nfd + j % nfd;
    a[t] = csr_entry(Fptr, Fcol, Fs, Fval, gi, gj);
  }
  gj_invert(a, rk, ck, n);
  double* out = einv + einv_ptr[e];
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) out[t] = a[t];
}

// P row r = (f, beta): the edges of f in loop order, each adding its inverse's row for (f, beta).
__global__ void k_p_values(int nf, int nfd, const int* __restrict__ fptr, const int* __restrict__ face_edge,
                           const int* __restrict__ edge_ptr, const int* __restrict__ edge_face,
                           const int64_t* __restrict__ einv_ptr, const double* __restrict__ einv,
                           const int* __restrict__ Pptr, const int* __restrict__ Pcol, Slots Ps,
                           double* __restrict__ Pval) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (int64_t)nf * nfd) return;
  const int f = (int)(r / nfd), beta = (int)(r - (int64_t)f * nfd);
  const int rb = Pptr[r], rn = Pptr[r + 1] - rb;
  for (int k = 0; k < rn; ++k) Pval[Ps.at(r, k)] = 0.0;
  for (int i = fptr[f]; i < fptr[f + 1]; ++i) {
    const int e = face_edge[i];
    const int* fe = edge_face + edge_ptr[e];
    const int m = edge_ptr[e + 1] - edge_ptr[e], n = m * nfd;
    int pf = 0;
    while (fe[pf] != f) ++pf;
    const double* inv = einv + einv_ptr[e] + (int64_t)(pf * nfd + beta) * n;
    for (int j = 0; j < m; ++j) {
      const int k0 = lower_bound_i32(Pcol + rb, rn, fe[j] * nfd);
      for (int c = 0; c < nfd; ++c) Pval[Ps.at(r, k0 + c)] += inv[j * nfd + c];
    }
  }
}

// The same on face blocks: row (f, beta), block by block (face g of the row), sums over the edges of
// f in loop order the inverse entries of the edges whose patch holds g (the same terms in the same
// order as above), then writes the block row once.
template <int NFD>
__global__ void k_p_values_blk(int nf, const int* __restrict__ fptr, const int* __restrict__ face_edge,
                               const int* __restrict__ edge_ptr, const int* __restrict__ edge_face,
                               const int64_t* __restrict__ einv_ptr, const double* __restrict__ einv,
                               const int* __restrict__ bptr, const int* __restrict__ bcol,
                               double* __restrict__ Pval) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (int64_t)nf * NFD) return;
  const int f = (int)(r / NFD), beta = (int)(r - (int64_t)f * NFD);
  const int b0 = bptr[f], b1 = bptr[f + 1];
  for (int b = b0; b < b1; ++b) {
    const int g = bcol[b];
    double acc[NFD];
#pragma unroll
    for (int c = 0; c < NFD; ++c) acc[c] = 0.0;
    for (int i = fptr[f]; i < fptr[f + 1]; ++i) {
      const int e = face_edge[i];
      const int* fe = edge_face + edge_ptr[e];
      const int m = edge_ptr[e + 1] - edge_ptr[e];
      int pf = 0, pg = -1;
      for (int q = 0; q < m; ++q) {
        if (fe[q] == f) pf = q;
        if (fe[q] == g) pg = q;
      }
      if (pg < 0) continue;
      const double* inv = einv + einv_ptr[e] + (int64_t)(pf * NFD + beta) * (m * NFD) + pg * NFD;
#pragma unroll
      for (int c = 0; c < NFD; ++c) acc[c] += inv[c];
    }
    double* out = Pval + ((int64_t)b * NFD + beta) * NFD;
#pragma unroll
    for (int c = 0; c < NFD; ++c) out[c] = acc[c];
  }
}

// One block per edge on face blocks: each pair of the patch's faces copies its block of the face
// system (one search in the block row), then the inverse as in k_edge_inv.
__global__ void k_edge_inv_blk(int ne, int nfd, const int* __restrict__ edge_ptr, const int* __restrict__ edge_face,
                               const int* __restrict__ bptr, const int* __restrict__ bcol,
                               const double* __restrict__ Fval, const int64_t* __restrict__ einv_ptr,
                               double* __restrict__ einv) {
  extern __shared__ double sh[];
  const int e = blockIdx.x;
  if (e >= ne) return;
  const int m = edge_ptr[e + 1] - edge_ptr[e], n = m * nfd;
  const int* fe = edge_face + edge_ptr[e];
  double* a = sh;
  double* rk = sh + n * n;
  double* ck = rk + n;
  for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
    const int i = t / m, j = t - i * m;
    const int fi = fe[i], fj = fe[j];
    const int b0 = bptr[fi], nb = bptr[fi + 1] - b0;
    const int k = lower_bound_i32(bcol + b0, nb, fj);
    const double* blk = (k < nb && bcol[b0 + k] == fj) ? Fval + (int64_t)(b0 + k) * nfd * nfd : nullptr;
    for (int bi = 0; bi < nfd; ++bi)
      for (int c = 0; c < nfd; ++c) a[(i * nfd + bi) * n + j * nfd + c] = blk ? blk[bi * nfd + c] : 0.0;
  }
  gj_invert(a, rk, ck, n);
  double* out = einv + einv_ptr[e];
  for (int t = threadIdx.x; t < n * n; t += blockDim.x) out[t] = a[t];
}

// Face-block pattern of an order-k face-DOF matrix from its CSR pattern: every row of face f must
// list the same faces, each with all nfd columns in order (err otherwise).
__global__ void k_blk_len(int nf, int nfd, const int* __restrict__ rowptr, int* __restrict__ len,
                          int* __restrict__ err) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int64_t r0 = (int64_t)f * nfd;
  const int n = rowptr[r0 + 1] - rowptr[r0];
  bool ok = n % nfd == 0;
  for (int i = 1; i < nfd; ++i) ok = ok && rowptr[r0 + i + 1] - rowptr[r0 + i] == n;
  if (!ok) *err = 1;
  len[f] = ok ? n / nfd : 0;
}

__global__ void k_blk_cols(int nf, int nfd, const int* __restrict__ rowptr, const int* __restrict__ col,
                           const int* __restrict__ bptr, int* __restrict__ bcol, int* __restrict__ err) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int64_t r0 = (int64_t)f * nfd;
  const int nb = bptr[f + 1] - bptr[f];
  for (int j = 0; j < nb; ++j) {
    const int g = col[rowptr[r0] + j * nfd] / nfd;
    bcol[bptr[f] + j] = g;
    for (int i = 0; i < nfd; ++i)
      for (int c = 0; c < nfd; ++c)
        if (col[rowptr[r0 + i] + j * nfd + c] != g * nfd + c) *err = 1;
  }
}

// CSR values from the stored copy (export)
__global__ void k_stored_to_csr(int64_t rows, const int* __restrict__ rowptr, Slots S, const double* __restrict__ v,
                                double* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int b = rowptr[r], n = rowptr[r + 1] - b;
  for (int k = 0; k < n; ++k) out[b + k] = v[S.at(r, k)];
}

__global__ void k_round32(int64_t n, const double* __restrict__ x, float* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

// ---- inner solve: right-hand side and back-substitution --------------------------------------

// u = W_P v_i,P for every face DOF of every cell (order k): one wavefront per cell, each lane a
// face DOF, reading its row of W (contiguous) and the cell's interior part of v, so that a cell's W
// is read by one wavefront at once.
__global__ void k_schwarz_cell_u(DofLayout L, const int* __restrict__ cptr, const int* __restrict__ ldof_ptr,
                                 const double* __restrict__ W, const double* __restrict__ v, double* __restrict__ u) {
  const int P = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (P >= L.nc) return;
  const int lane = threadIdx.x & 63;
  const int Fn = (cptr[P + 1] - cptr[P]) * L.nfd;
  const int64_t fo = (int64_t)ldof_ptr[P] - (int64_t)P * L.nint;  // face-DOF incidences of the cells before P
  const double* Wp = W + fo * L.nint;
  const double* vi = v + (int64_t)L.nf * L.nfd + (int64_t)P * L.nint;
  for (int l = lane; l < Fn; l += 64) {
    const double* Wr = Wp + (int64_t)l * L.nint;
    double acc = 0.0;
    for (int a = 0; a < L.nint; ++a) acc += Wr[a] * vi[a];
    u[fo + l] = acc;
  }
}

// The same with the cell's W and v_i staged in LDS first by coalesced loads (one 64-thread block
// per cell; LDS: fn_max nint + nint doubles); the row products then run from LDS in the same order.
__global__ void __launch_bounds__(64) k_schwarz_cell_u_lds(DofLayout L, const int* __restrict__ cptr,
                                                           const int* __restrict__ ldof_ptr,
                                                           const double* __restrict__ W,
                                                           const double* __restrict__ v, double* __restrict__ u) {
  extern __shared__ double sh[];
  const int P = blockIdx.x;
  const int ni = L.nint, Fn = (cptr[P + 1] - cptr[P]) * L.nfd, n = Fn * ni;
  const int64_t fo = (int64_t)ldof_ptr[P] - (int64_t)P * ni;
  const double* Wp = W + fo * ni;
  const double* vi = v + (int64_t)L.nf * L.nfd + (int64_t)P * ni;
  double* vs = sh + n;
  for (int t = threadIdx.x; t < n; t += 64) sh[t] = Wp[t];
  for (int t = threadIdx.x; t < ni; t += 64) vs[t] = vi[t];
  __syncthreads();
  for (int l = threadIdx.x; l < Fn; l += 64) {
    double acc = 0.0;
    for (int a = 0; a < ni; ++a) acc += sh[l * ni + a] * vs[a];
    u[fo + l] = acc;
  }
}

// r0 = v_f - sum over the face's cells of sigma u (order k), or v_f (lowest order)
template <typename T>
__global__ void k_schwarz_rhs(DofLayout L, const int* __restrict__ cptr, const int8_t* __restrict__ csign,
                              const int* __restrict__ face_cell, const int* __restrict__ face_lidx,
                              const int* __restrict__ ldof_ptr, const double* __restrict__ u,
                              const double* __restrict__ v, T* __restrict__ r0) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nF = (int64_t)L.nf * L.nfd;
  if (r >= nF) return;
  double t = v[r];
  if (L.nint > 0) {
    const int f = (int)(r / L.nfd), beta = (int)(r - (int64_t)f * L.nfd);
    for (int side = 0; side < 2; ++side) {
      const int P = face_cell[2 * f + side];
      if (P < 0) continue;
      const int j = face_lidx[2 * f + side];
      const double s = (double)csign[cptr[P] + j];
      t -= s * u[(int64_t)ldof_ptr[P] - (int64_t)P * L.nint + j * L.nfd + beta];
    }
  }
  r0[r] = (T)t;
}

__global__ void k_schwarz_back(DofLayout L, const int* __restrict__ cptr, const int* __restrict__ cface,
                               const int8_t* __restrict__ csign, const int* __restrict__ ldof_ptr,
                               const double* __restrict__ Aiinv, const double* __restrict__ W,
                               const double* __restrict__ v, double* __restrict__ z) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nF = (int64_t)L.nf * L.nfd;
  if (t >= (int64_t)L.nc * L.nint) return;
  const int P = (int)(t / L.nint), a = (int)(t - (int64_t)P * L.nint);
  const double* vi = v + nF + (int64_t)P * L.nint;
  const double* Ai = Aiinv + (int64_t)P * L.nint * L.nint + (int64_t)a * L.nint;
  double acc = 0.0;
  for (int b = 0; b < L.nint; ++b) acc += Ai[b] * vi[b];
  const int s0 = cptr[P], F = cptr[P + 1] - s0;
  const double* Wc = W + ((int64_t)ldof_ptr[P] - (int64_t)P * L.nint) * L.nint + a;
  for (int j = 0; j < F; ++j) {
    const double s = (double)csign[s0 + j];
    const int64_t g0 = (int64_t)cface[s0 + j] * L.nfd;
    for (int b = 0; b < L.nfd; ++b) acc -= Wc[(int64_t)(j * L.nfd + b) * L.nint] * s * z[g0 + b];
  }
  z[nF + t] = acc;
}

// The back-substitution with the cell's W, A_ii^{-1}, v_i and signed face values staged in LDS by
// coalesced loads (one 64-thread block per cell; LDS: fn_max nint + 2 fn_max + nint^2 + nint
// doubles), summing in the same order as k_schwarz_back.
__global__ void __launch_bounds__(64) k_schwarz_back_lds(DofLayout L, const int* __restrict__ cptr,
                                                         const int* __restrict__ cface,
                                                         const int8_t* __restrict__ csign,
                                                         const int* __restrict__ ldof_ptr,
                                                         const double* __restrict__ Aiinv,
                                                         const double* __restrict__ W,
                                                         const double* __restrict__ v, double* __restrict__ z) {
  extern __shared__ double sh[];
  const int P = blockIdx.x;
  const int ni = L.nint, s0 = cptr[P], Fn = (cptr[P + 1] - s0) * L.nfd, n = Fn * ni;
  const int64_t nF = (int64_t)L.nf * L.nfd;
  const int64_t fo = (int64_t)ldof_ptr[P] - (int64_t)P * ni;
  double* Ws = sh;
  double* ss = Ws + n;
  double* zs = ss + Fn;
  double* As = zs + Fn;
  double* vs = As + ni * ni;
  const double* Wp = W + fo * ni;
  const double* Ap = Aiinv + (int64_t)P * ni * ni;
  const double* vi = v + nF + (int64_t)P * ni;
  for (int t = threadIdx.x; t < n; t += 64) Ws[t] = Wp[t];
  for (int t = threadIdx.x; t < ni * ni; t += 64) As[t] = Ap[t];
  for (int t = threadIdx.x; t < ni; t += 64) vs[t] = vi[t];
  for (int l = threadIdx.x; l < Fn; l += 64) {
    const int j = l / L.nfd, b = l - j * L.nfd;
    ss[l] = (double)csign[s0 + j];
    zs[l] = z[(int64_t)cface[s0 + j] * L.nfd + b];
  }
  __syncthreads();
  for (int a = threadIdx.x; a < ni; a += 64) {
    double acc = 0.0;
    for (int b = 0; b < ni; ++b) acc += As[a * ni + b] * vs[b];
    for (int l = 0; l < Fn; ++l) acc -= Ws[l * ni + a] * ss[l] * zs[l];
    z[nF + (int64_t)P * ni + a] = acc;
  }
}

// Face-block copy of the pattern of C (an order-k face-DOF matrix); synchronises.
void build_blocks(hipStream_t s, Scratch& tmp, const Csr& C, int nf, int nfd, FaceBlocks& B) {
  DBuf<int> len, err;
  len.alloc((size_t)nf + 1);
  err.alloc(1);
  VEM_HIP(hipMemsetAsync(err.p, 0, sizeof(int), s));
  k_blk_len<<<grid(nf), kT, 0, s>>>(nf, nfd, C.rowptr, len, err);
  VEM_HIP(hipGetLastError());
  B.nfd = nfd;
  B.nf = nf;
  B.bptr.alloc((size_t)nf + 1);
  B.nblk = scan_i32(s, tmp, len, nf, B.bptr);
  B.bcol.alloc(B.nblk);
  k_blk_cols<<<grid(nf), kT, 0, s>>>(nf, nfd, C.rowptr, C.col, B.bptr, B.bcol, err);
  VEM_HIP(hipGetLastError());
  int h_err = 0;
  VEM_HIP(hipMemcpyAsync(&h_err, err.p, sizeof(int), hipMemcpyDeviceToHost, s));
  VEM_HIP(hipStreamSynchronize(s));
  VEM_REQUIRE(h_err == 0 && B.nblk * nfd * nfd == C.nnz, VEM_EINVAL,
              "face system whose rows do not couple whole faces");
  B.val.alloc(C.nnz);
  B.val32.release();
}

}  // namespace

void schwarz_build(hipStream_t s, Scratch& tmp, const SchwarzMesh& m, const DofLayout& L, const Csr& A,
                   Schwarz& X) {
  X.built = X.ready = X.ready32 = false;
  X.blocked = false;
  // incidences of the face loops
  int64_t ninc = 0;
  {
    int h_last = 0;
    VEM_HIP(hipMemcpyAsync(&h_last, m.fptr + m.nf, sizeof(int), hipMemcpyDeviceToHost, s));
    VEM_HIP(hipStreamSynchronize(s));
    ninc = h_last;
  }
  VEM_REQUIRE(ninc > 0, VEM_EINVAL, "mesh without face loops");
  DBuf<unsigned long long> keys, keys_out;
  DBuf<int> vals, vals_out, inc_face, flag, pos;
  keys.alloc(ninc);
  keys_out.alloc(ninc);
  vals.alloc(ninc);
  vals_out.alloc(ninc);
  inc_face.alloc(ninc);
  flag.alloc(ninc + 1);
  pos.alloc(ninc + 1);
  k_inc_face<<<grid(m.nf), kT, 0, s>>>(m.nf, m.fptr, inc_face);
  k_loop_keys<<<grid(m.nf), kT, 0, s>>>(m.nf, m.nv, m.fptr, m.fvtx, keys, vals);
  VEM_HIP(hipGetLastError());
  int end_bit = 1;
  const unsigned long long kmax = (unsigned long long)m.nv * (unsigned long long)m.nv;
  while (end_bit < 64 && (1ULL << end_bit) <= kmax) ++end_bit;
  // the hipcub storage is sized for the sort and for every later scan before the sort is enqueued,
  // so that no scan reallocates it while the sort may still run
  const int64_t nF = (int64_t)L.nf * L.nfd;
  scan_reserve(tmp, std::max<int64_t>(ninc, nF));
  size_t bytes = 0;
  VEM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, keys.p, keys_out.p, vals.p, vals_out.p, (int)ninc, 0,
                                             end_bit, s));
  tmp.cub.reserve(bytes > 0 ? bytes : 1);
  VEM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.cub.p, bytes, keys.p, keys_out.p, vals.p, vals_out.p, (int)ninc, 0,
                                             end_bit, s));
  k_edge_flags<<<grid(ninc), kT, 0, s>>>(ninc, keys_out, flag);
  VEM_HIP(hipGetLastError());
  const int64_t ne = scan_i32(s, tmp, flag, ninc, pos);
  X.ne = ne;
  X.edge_ptr.alloc(ne + 1);
  X.edge_face.alloc(ninc);
  X.face_edge.alloc(ninc);
  k_edge_lists<<<grid(ninc), kT, 0, s>>>(ninc, flag, pos, vals_out, inc_face, X.edge_ptr, X.edge_face, X.face_edge,
                                          (int)ne);
  VEM_HIP(hipGetLastError());
  // largest patch
  {
    DBuf<int> mx;
    mx.alloc(2);
    VEM_HIP(hipMemsetAsync(mx.p, 0, 2 * sizeof(int), s));
    k_max_patch<<<grid(ne), kT, 0, s>>>((int)ne, X.edge_ptr, mx.p);
    VEM_HIP(hipGetLastError());
    int h_mx = 0;
    VEM_HIP(hipMemcpyAsync(&h_mx, mx.p, sizeof(int), hipMemcpyDeviceToHost, s));
    VEM_HIP(hipStreamSynchronize(s));
    X.max_patch = h_mx;
  }
  VEM_REQUIRE(X.max_patch * L.nfd <= kMaxPatchDof, VEM_EINVAL,
              "edge patch of " + std::to_string(X.max_patch) + " faces exceeds the Schwarz preconditioner's limit");
  // pattern of P on the face DOFs
  X.nF = nF;
  {
    DBuf<int> len, err;
    len.alloc(nF + 1);
    err.alloc(1);
    VEM_HIP(hipMemsetAsync(err.p, 0, sizeof(int), s));
    k_p_rowlen<<<grid(m.nf), kT, 0, s>>>(m.nf, L.nfd, m.fptr, X.face_edge, X.edge_ptr, X.edge_face, len, err);
    VEM_HIP(hipGetLastError());
    X.Pc.rows = nF;
    X.Pc.rowptr.alloc(nF + 1);
    X.Pc.nnz = scan_i32(s, tmp, len, nF, X.Pc.rowptr);
    int h_err = 0;
    VEM_HIP(hipMemcpyAsync(&h_err, err.p, sizeof(int), hipMemcpyDeviceToHost, s));
    VEM_HIP(hipStreamSynchronize(s));
    VEM_REQUIRE(h_err == 0, VEM_EINVAL, "a face shares edges with more faces than the Schwarz preconditioner holds");
    X.Pc.col.alloc(X.Pc.nnz);
    X.Pc.val.alloc(X.Pc.nnz);
    k_p_cols<<<grid(m.nf), kT, 0, s>>>(m.nf, L.nfd, m.fptr, X.face_edge, X.edge_ptr, X.edge_face, X.Pc.rowptr,
                                        X.Pc.col);
    VEM_HIP(hipGetLastError());
  }
  // the order-k face system: face-DOF part of A_gamma's pattern
  if (L.nint > 0) {
    DBuf<int> len;
    len.alloc(nF + 1);
    k_fc_rowlen<<<grid(nF), kT, 0, s>>>(nF, A.rowptr, A.col, len);
    VEM_HIP(hipGetLastError());
    X.Fc.rows = nF;
    X.Fc.rowptr.alloc(nF + 1);
    X.Fc.nnz = scan_i32(s, tmp, len, nF, X.Fc.rowptr);
    X.Fc.col.alloc(X.Fc.nnz);
    X.Fc.val.alloc(X.Fc.nnz);
    k_fc_cols<<<grid(nF), kT, 0, s>>>(nF, A.rowptr, A.col, X.Fc.rowptr, X.Fc.col);
    VEM_HIP(hipGetLastError());
    if (face_blocks_supported(L.nfd)) {
      build_blocks(s, tmp, X.Fc, m.nf, L.nfd, X.Fb);
      build_blocks(s, tmp, X.Pc, m.nf, L.nfd, X.Pb);
      X.blocked = true;
    } else {
      const Csr* csr[2] = {&X.Fc, &X.Pc};
      Sell* sell[2] = {&X.Fs, &X.Ps};
      build_sells(s, tmp, csr, sell, 2);
    }
    X.Aiinv.alloc((size_t)m.nc * L.nint * L.nint);
    // W: (sum of face DOFs over the cells) x nint
    int h_ld = 0;
    VEM_HIP(hipMemcpyAsync(&h_ld, m.ldof_ptr + m.nc, sizeof(int), hipMemcpyDeviceToHost, s));
    VEM_HIP(hipStreamSynchronize(s));
    X.W.alloc(((size_t)h_ld - (size_t)m.nc * L.nint) * L.nint);
    X.ucell.alloc((size_t)h_ld - (size_t)m.nc * L.nint);
    // condensed cell matrices, when A_if and W of the largest cell fit in 64 KiB of LDS beside A_ii
    {
      DBuf<int64_t> len;
      DBuf<int> fmax;
      len.alloc((size_t)m.nc + 1);
      fmax.alloc(1);
      VEM_HIP(hipMemsetAsync(fmax.p, 0, sizeof(int), s));
      k_cell_fn2<<<grid(m.nc), kT, 0, s>>>(m.nc, L.nfd, m.cptr, len, fmax);
      VEM_HIP(hipGetLastError());
      int h_f = 0;
      VEM_HIP(hipMemcpyAsync(&h_f, fmax.p, sizeof(int), hipMemcpyDeviceToHost, s));
      VEM_HIP(hipStreamSynchronize(s));
      X.fn_max = h_f;
      const size_t lds = ((size_t)L.nint * L.nint + 2 * L.nint + 2 * (size_t)L.nint * h_f) * sizeof(double);
      X.sp_ptr.release();
      X.Sp.release();
      if (lds <= 64 * 1024) {
        X.sp_ptr.alloc((size_t)m.nc + 1);
        const int64_t tot = scan_i64(s, tmp, len, m.nc, X.sp_ptr);
        X.Sp.alloc(tot);
      }
    }
  } else {
    const Csr* csr[1] = {&X.Pc};
    Sell* sell[1] = {&X.Ps};
    build_sells(s, tmp, csr, sell, 1);
  }
  // patch inverse offsets
  {
    DBuf<int64_t> sz;
    sz.alloc(ne + 1);
    k_patch_size<<<grid(ne), kT, 0, s>>>((int)ne, L.nfd, X.edge_ptr, sz);
    VEM_HIP(hipGetLastError());
    X.einv_ptr.alloc(ne + 1);
    const int64_t tot = scan_i64(s, tmp, sz, ne, X.einv_ptr);
    X.einv.alloc(tot);
  }
  VEM_HIP(hipStreamSynchronize(s));  // the local temporaries above are freed on return
  X.built = true;
}

void schwarz_values(hipStream_t s, const SchwarzMesh& m, const DofLayout& L, const int64_t* lmat_ptr,
                    const double* M1, const int64_t* lb_ptr, const double* Bdiv1, const double* nu,
                    double inv_gamma, const int* bnd, const Csr& A, const Sell& As, Schwarz& X) {
  VEM_REQUIRE(X.built, VEM_EINVAL, "Schwarz pattern not built");
  const Csr& F = L.nint > 0 ? X.Fc : A;
  const Sell& Fs = schwarz_face_sell(X, As, L);
  // where the face system's and P's values live
  const Slots fsl = X.blocked ? slots_of(X.Fb) : slots_of(Fs);
  double* fval = X.blocked ? X.Fb.val.p : Fs.val.p;
  const Slots psl = X.blocked ? slots_of(X.Pb) : slots_of(X.Ps);
  double* pval = X.blocked ? X.Pb.val.p : X.Ps.val.p;
  if (L.nint > 0) {
    const bool sp = X.Sp.p != nullptr;
    const size_t lds =
        ((size_t)L.nint * L.nint + 2 * L.nint + (sp ? 2 * (size_t)L.nint * X.fn_max : 0)) * sizeof(double);
    k_cell_condense<<<m.nc, 64, lds, s>>>(L, m.cptr, m.cface, lmat_ptr, M1, lb_ptr, Bdiv1, nu, inv_gamma, bnd,
                                          m.ldof_ptr, X.Aiinv, X.W, X.fn_max, X.sp_ptr, X.Sp);
    VEM_HIP(hipGetLastError());
    k_fc_values<<<grid(X.nF), kT, 0, s>>>(L, m.cptr, m.cface, m.csign, m.ldof_ptr, m.sorted_gid, m.sorted_l,
                                           m.face_cell, m.face_lidx, lmat_ptr, M1, lb_ptr, Bdiv1, nu, inv_gamma, bnd,
                                           X.W, X.sp_ptr, X.Sp, fsl, fval);
    VEM_HIP(hipGetLastError());
  }
  const int n = X.max_patch * L.nfd;
  const size_t lds = ((size_t)n * n + 2 * n) * sizeof(double);
  if (X.ne > 0 && X.blocked)
    k_edge_inv_blk<<<(int)X.ne, 64, lds, s>>>((int)X.ne, L.nfd, X.edge_ptr, X.edge_face, X.Fb.bptr, X.Fb.bcol, fval,
                                               X.einv_ptr, X.einv);
  else if (X.ne > 0)
    k_edge_inv<<<(int)X.ne, 64, lds, s>>>((int)X.ne, L.nfd, X.edge_ptr, X.edge_face, F.rowptr, F.col, fsl, fval,
                                           X.einv_ptr, X.einv);
  VEM_HIP(hipGetLastError());
  if (X.blocked) {
    const int* bp = X.Pb.bptr;
    const int* bc = X.Pb.bcol;
    switch (L.nfd) {
      case 3:
        k_p_values_blk<3><<<grid(X.nF), kT, 0, s>>>(m.nf, m.fptr, X.face_edge, X.edge_ptr, X.edge_face, X.einv_ptr,
                                                     X.einv, bp, bc, pval);
        break;
      case 6:
        k_p_values_blk<6><<<grid(X.nF), kT, 0, s>>>(m.nf, m.fptr, X.face_edge, X.edge_ptr, X.edge_face, X.einv_ptr,
                                                     X.einv, bp, bc, pval);
        break;
      case 10:
        k_p_values_blk<10><<<grid(X.nF), kT, 0, s>>>(m.nf, m.fptr, X.face_edge, X.edge_ptr, X.edge_face, X.einv_ptr,
                                                      X.einv, bp, bc, pval);
        break;
      default:
        throw Error{VEM_EINVAL, "face blocks of an unsupported size"};
    }
  } else {
    k_p_values<<<grid(X.nF), kT, 0, s>>>(m.nf, L.nfd, m.fptr, X.face_edge, X.edge_ptr, X.edge_face, X.einv_ptr,
                                          X.einv, X.Pc.rowptr, X.Pc.col, psl, pval);
  }
  VEM_HIP(hipGetLastError());
  X.ready = true;
  X.ready32 = false;
}

void schwarz_round32(hipStream_t s, const DofLayout& L, Schwarz& X) {
  if (X.blocked) {
    for (FaceBlocks* B : {&X.Fb, &X.Pb}) {
      B->val32.alloc(B->val.n);
      k_round32<<<1024, kT, 0, s>>>((int64_t)B->val.n, B->val, B->val32);
    }
    VEM_HIP(hipGetLastError());
    X.ready32 = true;
    return;
  }
  X.Ps.val32.alloc(X.Ps.nnz);
  k_round32<<<1024, kT, 0, s>>>(X.Ps.nnz, X.Ps.val, X.Ps.val32);
  if (L.nint > 0) {
    X.Fs.val32.alloc(X.Fs.nnz);
    k_round32<<<1024, kT, 0, s>>>(X.Fs.nnz, X.Fs.val, X.Fs.val32);
  }
  VEM_HIP(hipGetLastError());
  X.ready32 = true;
}

void schwarz_export(hipStream_t s, const Schwarz& X, bool face, Csr& C) {
  if (!X.blocked) {
    sell_to_csr(s, face ? X.Fs : X.Ps, C);
    return;
  }
  const FaceBlocks& B = face ? X.Fb : X.Pb;
  if (C.rows > 0)
    k_stored_to_csr<<<grid(C.rows), kT, 0, s>>>(C.rows, C.rowptr, slots_of(B), B.val, C.val);
  VEM_HIP(hipGetLastError());
}

template <typename T>
void launch_schwarz_rhs(hipStream_t s, const SchwarzMesh& m, const DofLayout& L, const Schwarz& X, const int* bnd,
                        const double* v, T* r0) {
  (void)bnd;  // W rows of prescribed DOFs are zero
  if (L.nint > 0 && L.nc > 0) {
    VEM_REQUIRE(X.ucell.p != nullptr, VEM_EINVAL, "Schwarz cell buffers not built");
    const size_t lds = ((size_t)X.fn_max * L.nint + L.nint) * sizeof(double);
    if (lds <= kCellStageLds)
      k_schwarz_cell_u_lds<<<L.nc, 64, lds, s>>>(L, m.cptr, m.ldof_ptr, X.W, v, X.ucell);
    else
      k_schwarz_cell_u<<<(L.nc + 3) / 4, 256, 0, s>>>(L, m.cptr, m.ldof_ptr, X.W, v, X.ucell);
  }
  k_schwarz_rhs<T><<<grid(X.nF), kT, 0, s>>>(L, m.cptr, m.csign, m.face_cell, m.face_lidx, m.ldof_ptr, X.ucell, v,
                                             r0);
}
template void launch_schwarz_rhs<double>(hipStream_t, const SchwarzMesh&, const DofLayout&, const Schwarz&,
                                         const int*, const double*, double*);
template void launch_schwarz_rhs<float>(hipStream_t, const SchwarzMesh&, const DofLayout&, const Schwarz&,
                                        const int*, const double*, float*);

void launch_schwarz_back(hipStream_t s, const SchwarzMesh& m, const DofLayout& L, const Schwarz& X,
                         const double* v, double* z) {
  const int64_t n = (int64_t)L.nc * L.nint;
  if (n == 0) return;
  const size_t lds = ((size_t)X.fn_max * L.nint + 2 * (size_t)X.fn_max + (size_t)L.nint * L.nint + L.nint) *
                     sizeof(double);
  if (lds <= kCellStageLds)
    k_schwarz_back_lds<<<L.nc, 64, lds, s>>>(L, m.cptr, m.cface, m.csign, m.ldof_ptr, X.Aiinv, X.W, v, z);
  else
    k_schwarz_back<<<grid(n), kT, 0, s>>>(L, m.cptr, m.cface, m.csign, m.ldof_ptr, X.Aiinv, X.W, v, z);
}

}  // namespace vem
