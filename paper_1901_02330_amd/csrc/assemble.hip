// Global assembly by gathering (no floating-point atomics, so every run gives
// the same bits): the saddle matrix K = [M B^T; B 0], the regularised flux
// block A_gamma = M + B^T B / gamma (Block-Reg, eq. block_diag) and the
// approximate Schur complement S = B diag(M)^{-1} B^T (Block-Schur,
// eq. block_schur, taken with the sign that makes it SPD).
//
// DOF layout: flux unknown d < nf*nfd is moment b of face f = d / nfd with
// respect to the face's global normal; d >= nf*nfd are interior moments,
// nint per cell.  Pressure unknowns are npd moments per cell.  A local DOF
// l of cell P is a face DOF (face l / nfd of the cell, sign sigma of that
// face) or an interior DOF (sign +1).  Local matrices are stored densely per
// cell: M1 (ndof x ndof, nu = 1) at lmat_ptr[P], B_div (npd x ndof) at
// lb_ptr[P].  Each row of K is built by merging the sorted DOF lists of the
// (at most two) cells that hold the row's DOF.
#include "vem_internal.h"

#include <climits>

namespace vem {
namespace {

constexpr int kThreads = 256;
inline int nblocks(int64_t n) { return (int)((n + kThreads - 1) / kThreads); }

__device__ inline int ndof_of(const DofLayout& L, const int* cptr, int P) {
  return (cptr[P + 1] - cptr[P]) * L.nfd + L.nint;
}

__device__ inline void ldof_gid_sign(const DofLayout& L, const int* cptr, const int* cface, const int8_t* csign,
                                     int P, int l, int& gid, double& sg) {
  int s = cptr[P], F = cptr[P + 1] - s;
  if (l < F * L.nfd) {
    int j = l / L.nfd, b = l - j * L.nfd;
    gid = cface[s + j] * L.nfd + b;
    sg = (double)csign[s + j];
  } else {
    gid = L.nf * L.nfd + P * L.nint + (l - F * L.nfd);
    sg = 1.0;
  }
}

__device__ inline double ldof_sign(const DofLayout& L, const int* cptr, const int8_t* csign, int P, int l) {
  int s = cptr[P], F = cptr[P + 1] - s;
  return l < F * L.nfd ? (double)csign[s + l / L.nfd] : 1.0;
}

// With flux boundary data (bnd != nullptr: bnd[f] = 1 on boundary faces) the DOFs of the
// boundary faces are prescribed.
__device__ inline bool fixed_dof(const DofLayout& L, const int* bnd, int64_t gid) {
  return bnd && gid < (int64_t)L.nf * L.nfd && bnd[gid / L.nfd];
}

// Cells holding flux DOF d (ascending cell id) and the DOF's local index in each.
__device__ inline int dof_cells(const DofLayout& L, int64_t d, const int* cptr, const int* face_cell,
                                const int* face_lidx, int P[2], int l[2]) {
  int64_t nff = (int64_t)L.nf * L.nfd;
  if (d < nff) {
    int f = (int)(d / L.nfd), b = (int)(d - (int64_t)f * L.nfd);
    int n = 0;
    for (int side = 0; side < 2; ++side) {
      int c = face_cell[2 * f + side];
      if (c >= 0) {
        P[n] = c;
        l[n] = face_lidx[2 * f + side] * L.nfd + b;
        ++n;
      }
    }
    if (n == 2 && P[0] > P[1]) {
      int t = P[0];
      P[0] = P[1];
      P[1] = t;
      t = l[0];
      l[0] = l[1];
      l[1] = t;
    }
    return n;
  }
  int64_t r = d - nff;
  int c = (int)(r / L.nint);
  P[0] = c;
  l[0] = (cptr[c + 1] - cptr[c]) * L.nfd + (int)(r - (int64_t)c * L.nint);
  return 1;
}

// Per cell: local DOFs sorted by global id (face DOFs by face id, interior last).
__global__ void k_ldof_sort(DofLayout L, const int* __restrict__ cptr, const int* __restrict__ cface,
                            const int* __restrict__ ldof_ptr, int* sorted_gid, int* sorted_l) {
  int P = blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= L.nc) return;
  int s = cptr[P], F = cptr[P + 1] - s;
  int o = ldof_ptr[P];
  // insertion sort of the faces (F <= kMaxCellFaces)
  int order[kMaxCellFaces];
  for (int j = 0; j < F; ++j) {
    int f = cface[s + j];
    int k = j;
    while (k > 0 && cface[s + order[k - 1]] > f) {
      order[k] = order[k - 1];
      --k;
    }
    order[k] = j;
  }
  int q = 0;
  for (int k = 0; k < F; ++k) {
    int j = order[k];
    int f = cface[s + j];
    for (int b = 0; b < L.nfd; ++b, ++q) {
      sorted_gid[o + q] = f * L.nfd + b;
      sorted_l[o + q] = j * L.nfd + b;
    }
  }
  for (int b = 0; b < L.nint; ++b, ++q) {
    sorted_gid[o + q] = L.nf * L.nfd + P * L.nint + b;
    sorted_l[o + q] = F * L.nfd + b;
  }
}

// Neighbour cells of P through its faces, sorted and unique, P included.
__device__ inline int cell_neighbours(const int* cptr, const int* cface, const int* face_cell, int P,
                                      int* nb /* >= kMaxCellFaces + 1 */) {
  int s = cptr[P], F = cptr[P + 1] - s;
  int n = 0;
  auto insert = [&](int c) {
    for (int q = 0; q < n; ++q)
      if (nb[q] == c) return;
    int k = n;
    while (k > 0 && nb[k - 1] > c) {
      nb[k] = nb[k - 1];
      --k;
    }
    nb[k] = c;
    ++n;
  };
  insert(P);
  for (int j = 0; j < F; ++j) {
    int f = cface[s + j];
    int c0 = face_cell[2 * f], c1 = face_cell[2 * f + 1];
    int o = (c0 == P) ? c1 : c0;
    if (o >= 0) insert(o);
  }
  return n;
}

__global__ void k_rowlen(DofLayout L, const int* __restrict__ cptr, const int* __restrict__ ldof_ptr,
                         const int* __restrict__ sorted_gid, const int* __restrict__ face_cell,
                         const int* __restrict__ face_lidx, const int* __restrict__ cface, int* lenK, int* lenA,
                         int* lenS) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < L.Nu) {
    int P[2], l[2];
    int nc = dof_cells(L, r, cptr, face_cell, face_lidx, P, l);
    int cnt;
    if (nc == 1) {
      cnt = ldof_ptr[P[0] + 1] - ldof_ptr[P[0]];
    } else {
      const int* A = sorted_gid + ldof_ptr[P[0]];
      const int* B = sorted_gid + ldof_ptr[P[1]];
      int na = ldof_ptr[P[0] + 1] - ldof_ptr[P[0]], nb = ldof_ptr[P[1] + 1] - ldof_ptr[P[1]];
      int ia = 0, ib = 0;
      cnt = 0;
      while (ia < na || ib < nb) {
        int ga = ia < na ? A[ia] : INT_MAX, gb = ib < nb ? B[ib] : INT_MAX;
        int g = ga < gb ? ga : gb;
        if (ga == g) ++ia;
        if (gb == g) ++ib;
        ++cnt;
      }
    }
    lenA[r] = cnt;
    lenK[r] = cnt + nc * L.npd;
  } else if (r < L.Nu + L.Np) {
    int64_t q = r - L.Nu;
    int P = (int)(q / L.npd);
    lenK[r] = ldof_ptr[P + 1] - ldof_ptr[P];
    int nb[kMaxCellFaces + 1];
    lenS[q] = cell_neighbours(cptr, cface, face_cell, P, nb) * L.npd;
  }
}

__global__ void k_fill_patterns(DofLayout L, const int* __restrict__ cptr, const int* __restrict__ ldof_ptr,
                                const int* __restrict__ sorted_gid, const int* __restrict__ face_cell,
                                const int* __restrict__ face_lidx, const int* __restrict__ cface,
                                const int* __restrict__ Kptr, int* Kcol, int* Kdiag, const int* __restrict__ Aptr,
                                int* Acol, int* Adiag, const int* __restrict__ Sptr, int* Scol, int* Sdiag) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < L.Nu) {
    int P[2], l[2];
    int nc = dof_cells(L, r, cptr, face_cell, face_lidx, P, l);
    int k = Kptr[r], a = Aptr[r];
    const int* A = sorted_gid + ldof_ptr[P[0]];
    int na = ldof_ptr[P[0] + 1] - ldof_ptr[P[0]];
    const int* B = nc == 2 ? sorted_gid + ldof_ptr[P[1]] : A;
    int nb = nc == 2 ? ldof_ptr[P[1] + 1] - ldof_ptr[P[1]] : 0;
    int ia = 0, ib = 0;
    while (ia < na || ib < nb) {
      int ga = ia < na ? A[ia] : INT_MAX, gb = ib < nb ? B[ib] : INT_MAX;
      int g = ga < gb ? ga : gb;
      if (ga == g) ++ia;
      if (gb == g) ++ib;
      if (g == r) {
        Kdiag[r] = k;
        Adiag[r] = a;
      }
      Kcol[k++] = g;
      Acol[a++] = g;
    }
    for (int s = 0; s < nc; ++s)
      for (int q = 0; q < L.npd; ++q) Kcol[k++] = (int)(L.Nu + (int64_t)P[s] * L.npd + q);
  } else if (r < L.Nu + L.Np) {
    int64_t q = r - L.Nu;
    int P = (int)(q / L.npd), g = (int)(q - (int64_t)P * L.npd);
    int k = Kptr[r];
    for (int i = ldof_ptr[P]; i < ldof_ptr[P + 1]; ++i) Kcol[k++] = sorted_gid[i];
    int nb[kMaxCellFaces + 1];
    int n = cell_neighbours(cptr, cface, face_cell, P, nb);
    int o = Sptr[q];
    for (int i = 0; i < n; ++i)
      for (int dd = 0; dd < L.npd; ++dd) {
        int c = nb[i] * L.npd + dd;
        if (nb[i] == P && dd == g) Sdiag[q] = o;
        Scol[o++] = c;
      }
  }
}

__global__ void k_values(DofLayout L, const int* __restrict__ cptr, const int* __restrict__ cface,
                         const int8_t* __restrict__ csign, const int* __restrict__ ldof_ptr,
                         const int* __restrict__ sorted_gid, const int* __restrict__ sorted_l,
                         const int* __restrict__ face_cell, const int* __restrict__ face_lidx,
                         const int64_t* __restrict__ lmat_ptr, const double* __restrict__ M1,
                         const int64_t* __restrict__ lb_ptr, const double* __restrict__ Bdiv1,
                         const double* __restrict__ nu, double inv_gamma, const int* __restrict__ bnd,
                         const int* __restrict__ Kslice, double* Kval, const int* __restrict__ Aslice, double* Aval) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // entry k of row r sits at slot slice_ptr[r/64] + r%64 + 64k of the SELL arrays: the
  // stores of a wave's 64 rows are contiguous for each k.  Aval null: K only.
  // prescribed flux DOFs: identity rows and columns in K and A_gamma
  const bool fixed_row = r < L.Nu && fixed_dof(L, bnd, r);
  if (r < L.Nu) {
    int P[2], l[2];
    int nc = dof_cells(L, r, cptr, face_cell, face_lidx, P, l);
    int nd[2];
    double sr[2];
    const double* Mrow[2];
    const double* Bp[2];
    for (int s = 0; s < nc; ++s) {
      nd[s] = ndof_of(L, cptr, P[s]);
      sr[s] = ldof_sign(L, cptr, csign, P[s], l[s]);
      Mrow[s] = M1 + lmat_ptr[P[s]] + (int64_t)l[s] * nd[s];
      Bp[s] = Bdiv1 + lb_ptr[P[s]];
    }
    const int64_t kb = (int64_t)Kslice[r >> 6] + (r & 63);
    const int64_t ab = Aval ? (int64_t)Aslice[r >> 6] + (r & 63) : 0;
    int k = 0, a = 0;
    const int* A = sorted_gid + ldof_ptr[P[0]];
    const int* Al = sorted_l + ldof_ptr[P[0]];
    int na = ldof_ptr[P[0] + 1] - ldof_ptr[P[0]];
    const int* B = nc == 2 ? sorted_gid + ldof_ptr[P[1]] : A;
    const int* Bl = nc == 2 ? sorted_l + ldof_ptr[P[1]] : Al;
    int nb = nc == 2 ? ldof_ptr[P[1] + 1] - ldof_ptr[P[1]] : 0;
    int ia = 0, ib = 0;
    while (ia < na || ib < nb) {
      int ga = ia < na ? A[ia] : INT_MAX, gb = ib < nb ? B[ib] : INT_MAX;
      int g = ga < gb ? ga : gb;
      double mv = 0.0, bb = 0.0;
      if (ga == g) {
        int lg = Al[ia];
        double ss = sr[0] * ldof_sign(L, cptr, csign, P[0], lg);
        mv += nu[P[0]] * ss * Mrow[0][lg];
        if (Aval) {
          double t = 0.0;
          for (int q = 0; q < L.npd; ++q) t += Bp[0][q * nd[0] + l[0]] * Bp[0][q * nd[0] + lg];
          bb += ss * t;
        }
        ++ia;
      }
      if (gb == g) {
        int lg = Bl[ib];
        double ss = sr[1] * ldof_sign(L, cptr, csign, P[1], lg);
        mv += nu[P[1]] * ss * Mrow[1][lg];
        if (Aval) {
          double t = 0.0;
          for (int q = 0; q < L.npd; ++q) t += Bp[1][q * nd[1] + l[1]] * Bp[1][q * nd[1] + lg];
          bb += ss * t;
        }
        ++ib;
      }
      if (fixed_row || fixed_dof(L, bnd, g)) {
        mv = g == r ? 1.0 : 0.0;
        bb = 0.0;
      }
      Kval[kb + 64 * (int64_t)(k++)] = mv;
      if (Aval) Aval[ab + 64 * (int64_t)(a++)] = mv + inv_gamma * bb;
    }
    for (int s = 0; s < nc; ++s)
      for (int q = 0; q < L.npd; ++q)
        Kval[kb + 64 * (int64_t)(k++)] = fixed_row ? 0.0 : -sr[s] * Bp[s][q * nd[s] + l[s]];
  } else if (r < L.Nu + L.Np) {
    int64_t q = r - L.Nu;
    int P = (int)(q / L.npd), g = (int)(q - (int64_t)P * L.npd);
    int nd = ndof_of(L, cptr, P);
    const double* Bp = Bdiv1 + lb_ptr[P] + (int64_t)g * nd;
    const int64_t kb = (int64_t)Kslice[r >> 6] + (r & 63);
    int k = 0;
    for (int i = ldof_ptr[P]; i < ldof_ptr[P + 1]; ++i) {
      int lg = sorted_l[i];
      Kval[kb + 64 * (int64_t)(k++)] =
          fixed_dof(L, bnd, sorted_gid[i]) ? 0.0 : -ldof_sign(L, cptr, csign, P, lg) * Bp[lg];
    }
  }
}

__global__ void k_diag_inv(int64_t n, const int* __restrict__ pos, const double* __restrict__ val, double* d,
                           double* dinv) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = val[pos[i]];
  if (d) d[i] = v;
  dinv[i] = 1.0 / v;
}

// S[(P,g),(Q,e)] = sum_d B[(P,g),d] B[(Q,e),d] / diag(M)_d over flux DOFs d shared by P and Q.
__global__ void k_schur_values(DofLayout L, const int* __restrict__ cptr, const int* __restrict__ cface,
                               const int8_t* __restrict__ csign, const int* __restrict__ ldof_ptr,
                               const int* __restrict__ face_cell, const int* __restrict__ face_lidx,
                               const int64_t* __restrict__ lb_ptr, const double* __restrict__ Bdiv1,
                               const double* __restrict__ dM, const int* __restrict__ bnd,
                               const int* __restrict__ Sptr, const int* __restrict__ Scol,
                               const int* __restrict__ Sslice, double* Sval) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.Np) return;
  int P = (int)(q / L.npd), g = (int)(q - (int64_t)P * L.npd);
  int s = cptr[P], F = cptr[P + 1] - s;
  int ndP = F * L.nfd + L.nint;
  const double* BP = Bdiv1 + lb_ptr[P];
  // CSR entry k of this row goes to SELL slot sb + 64k
  const int64_t sb = (int64_t)Sslice[q >> 6] + (q & 63) - 64 * (int64_t)Sptr[q];
  for (int k = Sptr[q]; k < Sptr[q + 1]; ++k) {
    int c = Scol[k];
    int Q = c / L.npd, e = c - Q * L.npd;
    double v = 0.0;
    if (Q == P) {
      for (int l = 0; l < ndP; ++l) {
        int gid;
        double sg;
        ldof_gid_sign(L, cptr, cface, csign, P, l, gid, sg);
        if (fixed_dof(L, bnd, gid)) continue;  // B has no column for a prescribed flux
        v += BP[g * ndP + l] * BP[e * ndP + l] / dM[gid];  // the two signs cancel
      }
    } else {
      int ndQ = ndof_of(L, cptr, Q);
      const double* BQ = Bdiv1 + lb_ptr[Q];
      for (int j = 0; j < F; ++j) {
        int f = cface[s + j];
        int side = face_cell[2 * f] == Q ? 0 : (face_cell[2 * f + 1] == Q ? 1 : -1);
        if (side < 0) continue;
        int jq = face_lidx[2 * f + side];
        double sp = (double)csign[s + j], sq = (double)csign[cptr[Q] + jq];
        for (int b = 0; b < L.nfd; ++b) {
          int lp = j * L.nfd + b, lq = jq * L.nfd + b;
          v += sp * BP[g * ndP + lp] * sq * BQ[e * ndQ + lq] / dM[f * L.nfd + b];
        }
      }
    }
    Sval[sb + 64 * (int64_t)k] = v;
  }
}

// Right-hand side with flux boundary data: out = b - K xB on the free rows and out = xB on the
// prescribed ones, with xB the prescribed fluxes (zero elsewhere).  K xB is formed from the
// coefficient-free local matrices (only prescribed columns contribute), so it does not depend on the
// identity rows K holds in this mode.  One thread per row, the row's cells in a fixed order.
__global__ void k_flux_rhs(DofLayout L, const int* __restrict__ cptr, const int* __restrict__ cface,
                           const int8_t* __restrict__ csign, const int* __restrict__ face_cell,
                           const int* __restrict__ face_lidx, const int64_t* __restrict__ lmat_ptr,
                           const double* __restrict__ M1, const int64_t* __restrict__ lb_ptr,
                           const double* __restrict__ Bdiv1, const double* __restrict__ nu,
                           const int* __restrict__ bnd, const double* __restrict__ xB,
                           const double* __restrict__ b, double* __restrict__ out) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= L.Nu + L.Np) return;
  double acc = 0.0;
  if (r < L.Nu) {
    if (fixed_dof(L, bnd, r)) {
      out[r] = xB[r];
      return;
    }
    int P[2], l[2];
    int nc = dof_cells(L, r, cptr, face_cell, face_lidx, P, l);
    for (int c = 0; c < nc; ++c) {
      const int nd = ndof_of(L, cptr, P[c]);
      const double sr = ldof_sign(L, cptr, csign, P[c], l[c]);
      const double* Mrow = M1 + lmat_ptr[P[c]] + (int64_t)l[c] * nd;
      const int F = cptr[P[c] + 1] - cptr[P[c]];
      for (int j = 0; j < F * L.nfd; ++j) {
        int gid;
        double sg;
        ldof_gid_sign(L, cptr, cface, csign, P[c], j, gid, sg);
        if (fixed_dof(L, bnd, gid)) acc += nu[P[c]] * sr * sg * Mrow[j] * xB[gid];
      }
    }
  } else {
    const int64_t q = r - L.Nu;
    const int P = (int)(q / L.npd), g = (int)(q - (int64_t)P * L.npd);
    const int nd = ndof_of(L, cptr, P);
    const double* Bp = Bdiv1 + lb_ptr[P] + (int64_t)g * nd;
    const int F = cptr[P + 1] - cptr[P];
    for (int j = 0; j < F * L.nfd; ++j) {
      int gid;
      double sg;
      ldof_gid_sign(L, cptr, cface, csign, P, j, gid, sg);
      if (fixed_dof(L, bnd, gid)) acc += -sg * Bp[j] * xB[gid];
    }
  }
  out[r] = b[r] - acc;
}

// The discrete constant pressure n_p (the moment DOFs of p = 1: (1/|P|) int_P m_a, from the
// cell monomial moments when given, else 1) and the mean weights w (w . p = int_Omega p_h:
// |P| on the moment of the constant, 0 on the others).
__global__ void k_pressure_constants(DofLayout L, int nsm, const double* __restrict__ cmom,
                                     const double* __restrict__ cvol, double* __restrict__ np,
                                     double* __restrict__ w) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.Np) return;
  const int P = (int)(q / L.npd), a = (int)(q - (int64_t)P * L.npd);
  np[q] = cmom ? cmom[(int64_t)P * nsm + a] / cvol[P] : 1.0;
  w[q] = a == 0 ? cvol[P] : 0.0;
}

// g[P] = nu_P lambda_P^T M1_P u_P over the cell's oriented local flux DOFs (one wavefront per cell)
__global__ void __launch_bounds__(64) k_coef_grad(DofLayout L, const int* __restrict__ cptr,
                                                  const int* __restrict__ cface, const int8_t* __restrict__ csign,
                                                  const int64_t* __restrict__ lmat_ptr,
                                                  const double* __restrict__ M1, const double* __restrict__ nu,
                                                  const double* __restrict__ u, const double* __restrict__ lam,
                                                  double* __restrict__ g) {
  const int P = blockIdx.x;
  if (P >= L.nc) return;
  const int nd = ndof_of(L, cptr, P);
  const double* M = M1 + lmat_ptr[P];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nd; i += 64) {
    int gi;
    double si;
    ldof_gid_sign(L, cptr, cface, csign, P, i, gi, si);
    double t = 0.0;
    for (int j = 0; j < nd; ++j) {
      int gj;
      double sj;
      ldof_gid_sign(L, cptr, cface, csign, P, j, gj, sj);
      t += M[(int64_t)i * nd + j] * sj * u[gj];
    }
    acc += si * lam[gi] * t;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if (threadIdx.x == 0) g[P] = nu[P] * acc;
}

__global__ void k_cell_sizes(DofLayout L, const int* __restrict__ cptr, int64_t* ndof, int64_t* nmat,
                             int64_t* nb) {
  int P = blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= L.nc) return;
  int64_t n = (int64_t)(cptr[P + 1] - cptr[P]) * L.nfd + L.nint;
  ndof[P] = n;
  nmat[P] = n * n;
  nb[P] = n * L.npd;
}

}  // namespace

void launch_coef_grad(hipStream_t s, DofLayout L, const int* cptr, const int* cface, const int8_t* csign,
                      const int64_t* lmat_ptr, const double* M1, const double* nu, const double* u,
                      const double* lam, double* g) {
  if (L.nc > 0) k_coef_grad<<<L.nc, 64, 0, s>>>(L, cptr, cface, csign, lmat_ptr, M1, nu, u, lam, g);
}

void launch_cell_sizes(hipStream_t s, DofLayout L, const int* cptr, int64_t* ndof, int64_t* nmat, int64_t* nb) {
  k_cell_sizes<<<nblocks(L.nc), kThreads, 0, s>>>(L, cptr, ndof, nmat, nb);
}

void launch_ldof_sort(hipStream_t s, DofLayout L, const int* cptr, const int* cface, const int* ldof_ptr,
                      int* sorted_gid, int* sorted_l) {
  k_ldof_sort<<<nblocks(L.nc), kThreads, 0, s>>>(L, cptr, cface, ldof_ptr, sorted_gid, sorted_l);
}
void launch_rowlen(hipStream_t s, DofLayout L, const int* cptr, const int* ldof_ptr, const int* sorted_gid,
                   const int* face_cell, const int* face_lidx, const int* cface, int* lenK, int* lenA, int* lenS) {
  k_rowlen<<<nblocks(L.Nu + L.Np), kThreads, 0, s>>>(L, cptr, ldof_ptr, sorted_gid, face_cell, face_lidx, cface,
                                                     lenK, lenA, lenS);
}
void launch_fill_patterns(hipStream_t s, DofLayout L, const int* cptr, const int* ldof_ptr, const int* sorted_gid,
                          const int* face_cell, const int* face_lidx, const int* cface, const int* Kptr, int* Kcol,
                          int* Kdiag, const int* Aptr, int* Acol, int* Adiag, const int* Sptr, int* Scol,
                          int* Sdiag) {
  k_fill_patterns<<<nblocks(L.Nu + L.Np), kThreads, 0, s>>>(L, cptr, ldof_ptr, sorted_gid, face_cell, face_lidx,
                                                            cface, Kptr, Kcol, Kdiag, Aptr, Acol, Adiag, Sptr, Scol,
                                                            Sdiag);
}
void launch_values(hipStream_t s, DofLayout L, const int* cptr, const int* cface, const int8_t* csign,
                   const int* ldof_ptr, const int* sorted_gid, const int* sorted_l, const int* face_cell,
                   const int* face_lidx, const int64_t* lmat_ptr, const double* M1, const int64_t* lb_ptr,
                   const double* Bdiv1, const double* nu, double inv_gamma, const int* bnd, const int* Kslice,
                   double* Kval, const int* Aslice, double* Aval) {
  k_values<<<nblocks(L.Nu + L.Np), kThreads, 0, s>>>(L, cptr, cface, csign, ldof_ptr, sorted_gid, sorted_l,
                                                     face_cell, face_lidx, lmat_ptr, M1, lb_ptr, Bdiv1, nu,
                                                     inv_gamma, bnd, Kslice, Kval, Aslice, Aval);
}
void launch_flux_rhs(hipStream_t s, DofLayout L, const int* cptr, const int* cface, const int8_t* csign,
                     const int* face_cell, const int* face_lidx, const int64_t* lmat_ptr, const double* M1,
                     const int64_t* lb_ptr, const double* Bdiv1, const double* nu, const int* bnd, const double* xB,
                     const double* b, double* out) {
  k_flux_rhs<<<nblocks(L.Nu + L.Np), kThreads, 0, s>>>(L, cptr, cface, csign, face_cell, face_lidx, lmat_ptr, M1,
                                                       lb_ptr, Bdiv1, nu, bnd, xB, b, out);
}
void launch_pressure_constants(hipStream_t s, DofLayout L, int nsm, const double* cmom, const double* cvol,
                               double* np, double* w) {
  if (L.Np > 0) k_pressure_constants<<<nblocks(L.Np), kThreads, 0, s>>>(L, nsm, cmom, cvol, np, w);
}
void launch_diag_inv(hipStream_t s, int64_t n, const int* diagpos, const double* val, double* d, double* dinv) {
  if (n > 0) k_diag_inv<<<nblocks(n), kThreads, 0, s>>>(n, diagpos, val, d, dinv);
}
void launch_schur_values(hipStream_t s, DofLayout L, const int* cptr, const int* cface, const int8_t* csign,
                         const int* ldof_ptr, const int* face_cell, const int* face_lidx, const int64_t* lb_ptr,
                         const double* Bdiv1, const double* dM, const int* bnd, const int* Sptr, const int* Scol,
                         const int* Sslice, double* Sval) {
  k_schur_values<<<nblocks(L.Np), kThreads, 0, s>>>(L, cptr, cface, csign, ldof_ptr, face_cell, face_lidx, lb_ptr,
                                                    Bdiv1, dM, bnd, Sptr, Scol, Sslice, Sval);
}

}  // namespace vem
