// Local matrices of the paper's order-k mixed virtual element (Sections 2
// and 4), k = 1, 2, 3, for general polyhedra.
//
// Degrees of freedom (eqs. facePoly, gradMom, crossMom): per face the moments
// of v.n_f against the face scaled monomials of degree <= k (face frame
// e1, e2, origin x_f, scale h_f); per cell the gradient moments
// (h_P/|P|) int v . grad m_a, 1 <= |a| <= k-1, and the cross moments
// (1/|P|) int v . (m_I x m) over M^{G,+}_{k-1} = {(m,0,0): m has no x} u
// {(0,m,0)} u {(0,0,m)} (m of degree <= k-1; the constant counts as having
// no x).  Pressure: P_{k-1} with moment DOFs (eq. presMom).
//
// Integration.  Every integral is of a polynomial and is computed exactly:
//  * face integrals by the conical-product rule on the fan triangles of the
//    face, k+1 points per direction (exact to degree 2k+1);
//  * cell integrals of the scaled monomials m_g (homogeneous of degree |g|
//    about x_P) from face integrals through the divergence theorem applied
//    to (x - x_P) m_g:  int_P m_g = (1/(3+|g|)) sum_f ((x_f - x_P).n_f) int_f m_g.
//
// Construction per cell, in the order of Section 4.1 and 4.3:
//  D[i, (c,a)] = dof_i(e_c m_a);  face function phi_i.n_f = sum_d T_f[d, b] m^f_d
//  with T_f = |f| H_f^{-1};  div phi_i = H_{k-1}^{-1} R[:, i] with R[g, i] =
//  -int phi_i . grad m_g + sum_f int_f (phi_i.n_f) m_g (integration by parts);
//  B_proj[(c,a), i] = int phi_i . e_c m_a through Props. xDec/yDec/zDec and
//  inTermsOfGPerpBasis (gradient part: a gradient moment when 1 <= degree <=
//  k-1, integration by parts otherwise; cross part: cross moments);
//  Pi* = (I_3 (x) H_k)^{-1} B_proj;  with W = G + |P| D^T D,
//  M1 = Pi*^T W Pi* - |P| (D Pi* + (D Pi*)^T) + |P| I  (= Pi*^T G Pi* +
//  |P| (I - D Pi*)^T (I - D Pi*), the stabilised form with nu = 1);
//  B_div,P = |P| H_{k-1}^{-1} R (pressure basis dual to the moments).
// The products are small dense FP64 contractions (ndof x 3 dim P_k x ndof);
// FP64 matrix cores have no advantage over the FP64 vector units here.
#include "vem_internal.h"

namespace vem {
namespace {

__host__ __device__ constexpr int dimP3(int k) { return k < 0 ? 0 : (k + 1) * (k + 2) * (k + 3) / 6; }
__host__ __device__ constexpr int dimP2(int k) { return k < 0 ? 0 : (k + 1) * (k + 2) / 2; }
__host__ __device__ constexpr int dimGp(int k) { return (2 * k * k * k + 9 * k * k + 7 * k) / 6; }

// graded index of a 3D multi-index (degree, then x power descending, then y power descending)
__device__ inline int idx3(int a1, int a2, int a3) {
  int d = a1 + a2 + a3, s = d - a1;
  return d * (d + 1) * (d + 2) / 6 + s * (s + 1) / 2 + (s - a2);
}
__device__ inline int idx2(int b1, int b2) {
  int d = b1 + b2;
  return d * (d + 1) / 2 + (d - b1);
}
// exponents of the i-th 3D multi-index
__device__ inline void exp3(int i, int& a1, int& a2, int& a3) {
  int d = 0;
  while (dimP3(d) <= i) ++d;
  int r = i - dimP3(d - 1);
  // within degree d: a1 = d, d-1, ..., blocks of size d - a1 + 1
  int a = d;
  while (r >= d - a + 1) {
    r -= d - a + 1;
    --a;
  }
  a1 = a;
  a2 = (d - a) - r;
  a3 = d - a1 - a2;
}
__device__ inline void exp2(int i, int& b1, int& b2) {
  int d = 0;
  while (dimP2(d) <= i) ++d;
  int r = i - dimP2(d - 1);
  b1 = d - r;
  b2 = r;
}

__device__ inline double ipow(double x, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= x;
  return r;
}

template <int K>
struct PK {
  static constexpr int NS = dimP3(K);        // dim P_k(P)
  static constexpr int NS1 = dimP3(K - 1);   // dim P_{k-1}(P): pressure DOFs
  static constexpr int NS2 = dimP3(K + 1);   // cell monomials used on faces
  static constexpr int NSM = dimP3(2 * K);   // cell moments
  static constexpr int NFD = dimP2(K);       // face DOFs per face
  static constexpr int NF2 = dimP2(2 * K);   // face moments for the face Gram matrix
  static constexpr int NG = NS1 - 1;         // gradient moments
  static constexpr int NCX = dimGp(K);       // cross moments
  static constexpr int NINT = NG + NCX;
  static constexpr int N3 = 3 * NS;          // vector monomials
  static constexpr int NQ = K + 1;           // face rule points per direction
  static constexpr int NPT = NQ * NQ;        // points per triangle
};

// cross-DOF set member x -> (component d, multi-index mu); x-part: monomials without x
template <int K>
__device__ inline void cross_member(int x, int& d, int& m1, int& m2, int& m3) {
  constexpr int NS1 = PK<K>::NS1;
  constexpr int NX = dimP2(K - 1);  // monomials of degree <= k-1 in (y, z)
  if (x < NX) {
    d = 0;
    int b1, b2;
    exp2(x, b1, b2);
    m1 = 0;
    m2 = b1;
    m3 = b2;
  } else {
    x -= NX;
    d = x < NS1 ? 1 : 2;
    exp3(x < NS1 ? x : x - NS1, m1, m2, m3);
  }
}
// position of (d, mu) in the cross set (mu of the set)
template <int K>
__device__ inline int cross_pos(int d, int m1, int m2, int m3) {
  constexpr int NX = dimP2(K - 1);
  if (d == 0) return idx2(m2, m3);
  return NX + (d - 1) * PK<K>::NS1 + idx3(m1, m2, m3);
}

// ---- per incidence: FP[g] = int_f m_g (|g| <= 2k), FM[d][g] = int_f m^f_d m_g (|g| <= k+1) ----
// One 64-thread block (one wavefront) per cell-face incidence: the points of a
// fan triangle are staged in LDS, then every lane integrates its outputs.
template <int K>
__global__ void __launch_bounds__(64) k_pk_face_moments(int64_t ninc, const int* __restrict__ inc_cell,
                                                        const int* __restrict__ cface,
                                                        const double* __restrict__ xyz,
                                                        const int* __restrict__ fptr, const int* __restrict__ fvtx,
                                                        const double* __restrict__ fcen,
                                                        const double* __restrict__ fdiam,
                                                        const double* __restrict__ fe1,
                                                        const double* __restrict__ fe2,
                                                        const double* __restrict__ ccen,
                                                        const double* __restrict__ cdiam,
                                                        const double* __restrict__ tri_ref, double* FP, double* FM) {
  using C = PK<K>;
  constexpr int NOUT = C::NSM + C::NFD * C::NS2;
  constexpr int NQO = (NOUT + 63) / 64;
  __shared__ double pts[C::NPT][4];
  const int lane = threadIdx.x;
  const int64_t j = blockIdx.x;
  if (j >= ninc) return;  // uniform for the whole block
  const int f = cface[j], P = inc_cell[j];
  const int fs = fptr[f], nv = fptr[f + 1] - fs;
  const double px = ccen[3 * P], py = ccen[3 * P + 1], pz = ccen[3 * P + 2], ih = 1.0 / cdiam[P];
  const double fx = fcen[3 * f], fy = fcen[3 * f + 1], fz = fcen[3 * f + 2], ihf = 1.0 / fdiam[f];
  const double e1x = fe1[3 * f], e1y = fe1[3 * f + 1], e1z = fe1[3 * f + 2];
  const double e2x = fe2[3 * f], e2y = fe2[3 * f + 1], e2z = fe2[3 * f + 2];
  int og[NQO], od[NQO];
#pragma unroll
  for (int q = 0; q < NQO; ++q) {
    const int o = lane + 64 * q;
    od[q] = -1;
    og[q] = -1;
    if (o < C::NSM) {
      og[q] = o;
    } else if (o < NOUT) {
      od[q] = (o - C::NSM) / C::NS2;
      og[q] = (o - C::NSM) - od[q] * C::NS2;
    }
  }
  double acc[NQO];
#pragma unroll
  for (int q = 0; q < NQO; ++q) acc[q] = 0.0;
  const int v0 = fvtx[fs];
  const double Ax = xyz[3 * v0], Ay = xyz[3 * v0 + 1], Az = xyz[3 * v0 + 2];
  for (int a = 1; a + 1 < nv; ++a) {
    if (lane < C::NPT) {
      const int va = fvtx[fs + a], vb = fvtx[fs + a + 1];
      const double Bx = xyz[3 * va] - Ax, By = xyz[3 * va + 1] - Ay, Bz = xyz[3 * va + 2] - Az;
      const double Cx = xyz[3 * vb] - Ax, Cy = xyz[3 * vb + 1] - Ay, Cz = xyz[3 * vb + 2] - Az;
      const double nx = By * Cz - Bz * Cy, ny = Bz * Cx - Bx * Cz, nz = Bx * Cy - By * Cx;
      const double a2 = sqrt(nx * nx + ny * ny + nz * nz);
      const double xi = tri_ref[3 * lane], eta = tri_ref[3 * lane + 1], w = tri_ref[3 * lane + 2];
      pts[lane][0] = Ax + xi * Bx + eta * Cx;
      pts[lane][1] = Ay + xi * By + eta * Cy;
      pts[lane][2] = Az + xi * Bz + eta * Cz;
      pts[lane][3] = a2 * w;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQO; ++q) {
      if (og[q] < 0) continue;
      int g1, g2, g3, d1 = 0, d2 = 0;
      exp3(og[q], g1, g2, g3);
      if (od[q] >= 0) exp2(od[q], d1, d2);
      double s = 0.0;
      for (int r = 0; r < C::NPT; ++r) {
        const double X = pts[r][0], Y = pts[r][1], Z = pts[r][2];
        double v = pts[r][3] * ipow((X - px) * ih, g1) * ipow((Y - py) * ih, g2) * ipow((Z - pz) * ih, g3);
        if (od[q] >= 0) {
          const double dx = X - fx, dy = Y - fy, dz = Z - fz;
          v *= ipow((dx * e1x + dy * e1y + dz * e1z) * ihf, d1) * ipow((dx * e2x + dy * e2y + dz * e2z) * ihf, d2);
        }
        s += v;
      }
      acc[q] += s;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NQO; ++q) {
    if (og[q] < 0) continue;
    if (od[q] < 0)
      FP[j * C::NSM + og[q]] = acc[q];
    else
      FM[j * (C::NFD * C::NS2) + od[q] * C::NS2 + og[q]] = acc[q];
  }
}

// small dense SPD solve helpers (column-major free, row-major arrays)
template <int N>
__device__ inline void cholesky(double* A) {  // in place, lower factor in A
  for (int j = 0; j < N; ++j) {
    double s = A[j * N + j];
    for (int k = 0; k < j; ++k) s -= A[j * N + k] * A[j * N + k];
    s = sqrt(s);
    A[j * N + j] = s;
    for (int i = j + 1; i < N; ++i) {
      double t = A[i * N + j];
      for (int k = 0; k < j; ++k) t -= A[i * N + k] * A[j * N + k];
      A[i * N + j] = t / s;
    }
  }
}
template <int N>
__device__ inline void chol_solve(const double* L, double* b) {  // b <- A^{-1} b
  for (int i = 0; i < N; ++i) {
    double t = b[i];
    for (int k = 0; k < i; ++k) t -= L[i * N + k] * b[k];
    b[i] = t / L[i * N + i];
  }
  for (int i = N - 1; i >= 0; --i) {
    double t = b[i];
    for (int k = i + 1; k < N; ++k) t -= L[k * N + i] * b[k];
    b[i] = t / L[i * N + i];
  }
}

// ---- per face: T_f = |f| H_f^{-1}, H_f[a][b] = int_f m^f_a m^f_b ----------------------------
template <int K>
__global__ void k_pk_face_gram(int nf, const double* __restrict__ xyz, const int* __restrict__ fptr,
                               const int* __restrict__ fvtx, const double* __restrict__ farea,
                               const double* __restrict__ fcen, const double* __restrict__ fdiam,
                               const double* __restrict__ fe1, const double* __restrict__ fe2,
                               const double* __restrict__ tri_ref, double* Tf) {
  using C = PK<K>;
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  double mom[C::NF2];
  for (int i = 0; i < C::NF2; ++i) mom[i] = 0.0;
  const int fs = fptr[f], nv = fptr[f + 1] - fs;
  const double fx = fcen[3 * f], fy = fcen[3 * f + 1], fz = fcen[3 * f + 2], ihf = 1.0 / fdiam[f];
  const double e1x = fe1[3 * f], e1y = fe1[3 * f + 1], e1z = fe1[3 * f + 2];
  const double e2x = fe2[3 * f], e2y = fe2[3 * f + 1], e2z = fe2[3 * f + 2];
  const int v0 = fvtx[fs];
  const double Ax = xyz[3 * v0], Ay = xyz[3 * v0 + 1], Az = xyz[3 * v0 + 2];
  for (int a = 1; a + 1 < nv; ++a) {
    const int va = fvtx[fs + a], vb = fvtx[fs + a + 1];
    const double Bx = xyz[3 * va] - Ax, By = xyz[3 * va + 1] - Ay, Bz = xyz[3 * va + 2] - Az;
    const double Cx = xyz[3 * vb] - Ax, Cy = xyz[3 * vb + 1] - Ay, Cz = xyz[3 * vb + 2] - Az;
    const double nx = By * Cz - Bz * Cy, ny = Bz * Cx - Bx * Cz, nz = Bx * Cy - By * Cx;
    const double a2 = sqrt(nx * nx + ny * ny + nz * nz);
    for (int r = 0; r < C::NPT; ++r) {
      const double xi = tri_ref[3 * r], eta = tri_ref[3 * r + 1], w = a2 * tri_ref[3 * r + 2];
      const double dx = Ax + xi * Bx + eta * Cx - fx, dy = Ay + xi * By + eta * Cy - fy,
                   dz = Az + xi * Bz + eta * Cz - fz;
      const double s = (dx * e1x + dy * e1y + dz * e1z) * ihf, t = (dx * e2x + dy * e2y + dz * e2z) * ihf;
      for (int i = 0; i < C::NF2; ++i) {
        int b1, b2;
        exp2(i, b1, b2);
        mom[i] += w * ipow(s, b1) * ipow(t, b2);
      }
    }
  }
  double H[C::NFD * C::NFD];
  for (int a = 0; a < C::NFD; ++a)
    for (int b = 0; b < C::NFD; ++b) {
      int a1, a2, b1, b2;
      exp2(a, a1, a2);
      exp2(b, b1, b2);
      H[a * C::NFD + b] = mom[idx2(a1 + b1, a2 + b2)];
    }
  cholesky<C::NFD>(H);
  const double A = farea[f];
  for (int b = 0; b < C::NFD; ++b) {
    double e[C::NFD];
    for (int i = 0; i < C::NFD; ++i) e[i] = i == b ? A : 0.0;
    chol_solve<C::NFD>(H, e);
    for (int d = 0; d < C::NFD; ++d) Tf[(int64_t)f * C::NFD * C::NFD + d * C::NFD + b] = e[d];
  }
}

// ---- per cell (one 256-thread block): D, divergence, B_proj, Pi*, M1, B_div --------------------
template <int K>
__global__ void __launch_bounds__(256) k_pk_cell(int nc, const int* __restrict__ cptr, const int* __restrict__ cface,
                                                 const int8_t* __restrict__ csign, const double* __restrict__ farea,
                                                 const double* __restrict__ fnormal, const double* __restrict__ fcen,
                                                 const double* __restrict__ cvol, const double* __restrict__ ccen,
                                                 const double* __restrict__ cdiam, const double* __restrict__ FP,
                                                 const double* __restrict__ FM, const double* __restrict__ Tf,
                                                 const int* __restrict__ ldof_ptr, double* Dg, double* Pg, double* Xg,
                                                 double* Cg, const int64_t* __restrict__ lmat_ptr, double* M1,
                                                 const int64_t* __restrict__ lb_ptr, double* Bdiv1, double* cmom) {
  using C = PK<K>;
  constexpr int NS = C::NS, NS1 = C::NS1, N3 = C::N3, NFD = C::NFD, NS2 = C::NS2;
  const int P = blockIdx.x;
  if (P >= nc) return;
  const int t = threadIdx.x, nt = blockDim.x;
  const int s0 = cptr[P], F = cptr[P + 1] - s0;
  const int ndof = F * NFD + C::NINT;
  const int og = F * NFD, ox = F * NFD + C::NG;
  const double vol = cvol[P], hP = cdiam[P];
  const double px = ccen[3 * P], py = ccen[3 * P + 1], pz = ccen[3 * P + 2];
  __shared__ double I[C::NSM];
  __shared__ double LK[NS * NS];
  __shared__ double LK1[NS1 * NS1];
  __shared__ double W[N3 * N3];
  // scratch of this cell: D (ndof x N3), Pi* / B_proj (N3 x ndof), X = W Pi* (N3 x ndof), cdiv (NS1 x ndof)
  const int64_t lo = ldof_ptr[P];
  double* D = Dg + lo * N3;
  double* Pi = Pg + lo * N3;
  double* X = Xg + lo * N3;
  double* Cd = Cg + lo * NS1;

  // cell moments from the face integrals (divergence theorem on (x - x_P) m_g)
  for (int g = t; g < C::NSM; g += nt) {
    int g1, g2, g3;
    exp3(g, g1, g2, g3);
    double s = 0.0;
    for (int j = 0; j < F; ++j) {
      const int f = cface[s0 + j];
      const double sg = (double)csign[s0 + j];
      const double dist = sg * ((fcen[3 * f] - px) * fnormal[3 * f] + (fcen[3 * f + 1] - py) * fnormal[3 * f + 1] +
                                (fcen[3 * f + 2] - pz) * fnormal[3 * f + 2]);
      s += dist * FP[(int64_t)(s0 + j) * C::NSM + g];
    }
    I[g] = s / (3.0 + g1 + g2 + g3);
    cmom[(int64_t)P * C::NSM + g] = I[g];
  }
  __syncthreads();
  for (int e = t; e < NS * NS; e += nt) {
    int a1, a2, a3, b1, b2, b3;
    exp3(e / NS, a1, a2, a3);
    exp3(e % NS, b1, b2, b3);
    LK[e] = I[idx3(a1 + b1, a2 + b2, a3 + b3)];
    if (e / NS < NS1 && e % NS < NS1) LK1[(e / NS) * NS1 + e % NS] = LK[e];
  }
  __syncthreads();
  if (t == 0) cholesky<NS>(LK);
  if (t == 1) cholesky<NS1>(LK1);
  __syncthreads();

  // D[i, (c,a)]: DOFs of the vector monomials
  for (int e = t; e < ndof * N3; e += nt) {
    const int i = e / N3, col = e % N3, c = col / NS;
    int a1, a2, a3;
    exp3(col % NS, a1, a2, a3);
    double v = 0.0;
    if (i < og) {
      const int j = i / NFD, b = i % NFD;
      const int f = cface[s0 + j];
      const double nout = (double)csign[s0 + j] * fnormal[3 * f + c];
      v = nout * FM[(int64_t)(s0 + j) * NFD * NS2 + b * NS2 + idx3(a1, a2, a3)] / farea[f];
    } else if (i < ox) {
      int g1, g2, g3;
      exp3(i - og + 1, g1, g2, g3);
      const int gc = c == 0 ? g1 : (c == 1 ? g2 : g3);
      if (gc > 0)
        v = gc * I[idx3(a1 + g1 - (c == 0), a2 + g2 - (c == 1), a3 + g3 - (c == 2))] / vol;
    } else {
      int d, m1, m2, m3;
      cross_member<K>(i - ox, d, m1, m2, m3);
      // (m_I x e_d)_c = eps_{c a d} m_{e_a}
      const int a = 3 - c - d;  // the only index with eps != 0 when c != d
      if (c != d) {
        const double eps = ((c + 1) % 3 == a) ? 1.0 : -1.0;  // eps_{c a d} for a cyclic triple
        v = eps * I[idx3(a1 + m1 + (a == 0), a2 + m2 + (a == 1), a3 + m3 + (a == 2))] / vol;
      }
    }
    D[(int64_t)i * N3 + col] = v;
  }
  // R and div phi_i = H_{k-1}^{-1} R[:, i]  (one thread per DOF i)
  for (int i = t; i < ndof; i += nt) {
    double r[NS1];
    for (int g = 0; g < NS1; ++g) r[g] = 0.0;
    if (i < og) {
      const int j = i / NFD, b0 = i % NFD;
      const int f = cface[s0 + j];
      const double* T = Tf + (int64_t)f * NFD * NFD;
      const double* fm = FM + (int64_t)(s0 + j) * NFD * NS2;
      for (int g = 0; g < NS1; ++g) {
        double s = 0.0;
        for (int d = 0; d < NFD; ++d) s += T[d * NFD + b0] * fm[d * NS2 + g];
        r[g] = s;
      }
    } else if (i < ox) {
      r[i - og + 1] = -vol / hP;
    }
    chol_solve<NS1>(LK1, r);
    for (int g = 0; g < NS1; ++g) {
      Cd[(int64_t)g * ndof + i] = r[g];
      Bdiv1[lb_ptr[P] + (int64_t)g * ndof + i] = vol * r[g];
    }
  }
  __syncthreads();
  // B_proj (stored in Pi), one thread per (c, a, i)
  for (int e = t; e < N3 * ndof; e += nt) {
    const int row = e / ndof, i = e % ndof, c = row / NS;
    int a1, a2, a3;
    exp3(row % NS, a1, a2, a3);
    const double s = a1 + a2 + a3 + 1.0;
    const double gco = hP / s;
    const int b1 = a1 + (c == 0), b2 = a2 + (c == 1), b3 = a3 + (c == 2);
    const int bd = b1 + b2 + b3;
    double v = 0.0;
    if (bd <= K - 1) {
      if (i == og + idx3(b1, b2, b3) - 1) v = gco * vol / hP;
    } else {
      double t1 = 0.0;
      for (int g = 0; g < NS1; ++g) {
        int g1, g2, g3;
        exp3(g, g1, g2, g3);
        t1 += Cd[(int64_t)g * ndof + i] * I[idx3(g1 + b1, g2 + b2, g3 + b3)];
      }
      v = -gco * t1;
      if (i < og) {
        const int j = i / NFD, b0 = i % NFD;
        const int f = cface[s0 + j];
        const double* T = Tf + (int64_t)f * NFD * NFD;
        const double* fm = FM + (int64_t)(s0 + j) * NFD * NS2;
        const int bi = idx3(b1, b2, b3);
        double t2 = 0.0;
        for (int d = 0; d < NFD; ++d) t2 += T[d * NFD + b0] * fm[d * NS2 + bi];
        v += gco * t2;
      }
    }
    if (i >= ox) {
      // cross part of e_c m_a (Props. xDec, yDec, zDec; x terms with an x power by inTermsOfGPerpBasis)
      double cf[2];
      int cd[2], cm[2][3];
      if (c == 0) {
        cf[0] = -a3 / s; cd[0] = 1; cm[0][0] = a1; cm[0][1] = a2; cm[0][2] = a3 - 1;
        cf[1] = a2 / s;  cd[1] = 2; cm[1][0] = a1; cm[1][1] = a2 - 1; cm[1][2] = a3;
      } else if (c == 1) {
        cf[0] = a3 / s;  cd[0] = 0; cm[0][0] = a1; cm[0][1] = a2; cm[0][2] = a3 - 1;
        cf[1] = -a1 / s; cd[1] = 2; cm[1][0] = a1 - 1; cm[1][1] = a2; cm[1][2] = a3;
      } else {
        cf[0] = a1 / s;  cd[0] = 1; cm[0][0] = a1 - 1; cm[0][1] = a2; cm[0][2] = a3;
        cf[1] = -a2 / s; cd[1] = 0; cm[1][0] = a1; cm[1][1] = a2 - 1; cm[1][2] = a3;
      }
      for (int q = 0; q < 2; ++q) {
        if (cf[q] == 0.0) continue;
        const int m1 = cm[q][0], m2 = cm[q][1], m3 = cm[q][2];
        if (cd[q] == 0 && m1 >= 1) {
          // m_I x (m,0,0) = -m_I x (0, m x^-1 y, 0) - m_I x (0, 0, m x^-1 z)
          if (i - ox == cross_pos<K>(1, m1 - 1, m2 + 1, m3)) v -= cf[q] * vol;
          if (i - ox == cross_pos<K>(2, m1 - 1, m2, m3 + 1)) v -= cf[q] * vol;
        } else if (i - ox == cross_pos<K>(cd[q], m1, m2, m3)) {
          v += cf[q] * vol;
        }
      }
    }
    Pi[(int64_t)row * ndof + i] = v;
  }
  __syncthreads();
  // Pi* = (I_3 (x) H_k)^{-1} B_proj: one thread per (component, DOF)
  for (int e = t; e < 3 * ndof; e += nt) {
    const int c = e / ndof, i = e % ndof;
    double b[NS];
    for (int a = 0; a < NS; ++a) b[a] = Pi[(int64_t)(c * NS + a) * ndof + i];
    chol_solve<NS>(LK, b);
    for (int a = 0; a < NS; ++a) Pi[(int64_t)(c * NS + a) * ndof + i] = b[a];
  }
  // W = G + |P| D^T D
  for (int e = t; e < N3 * N3; e += nt) {
    const int a = e / N3, b = e % N3;
    double s = 0.0;
    for (int i = 0; i < ndof; ++i) s += D[(int64_t)i * N3 + a] * D[(int64_t)i * N3 + b];
    double g = 0.0;
    if (a / NS == b / NS) {
      int a1, a2, a3, b1, b2, b3;
      exp3(a % NS, a1, a2, a3);
      exp3(b % NS, b1, b2, b3);
      g = I[idx3(a1 + b1, a2 + b2, a3 + b3)];
    }
    W[e] = g + vol * s;
  }
  __syncthreads();
  // X = W Pi*
  for (int e = t; e < N3 * ndof; e += nt) {
    const int a = e / ndof, i = e % ndof;
    double s = 0.0;
    for (int b = 0; b < N3; ++b) s += W[a * N3 + b] * Pi[(int64_t)b * ndof + i];
    X[(int64_t)a * ndof + i] = s;
  }
  __syncthreads();
  // M1 = Pi*^T X - |P| (D Pi* + (D Pi*)^T) + |P| I
  double* Mo = M1 + lmat_ptr[P];
  for (int e = t; e < ndof * ndof; e += nt) {
    const int i = e / ndof, j = e % ndof;
    double s = 0.0, q = 0.0;
    for (int a = 0; a < N3; ++a) {
      s += Pi[(int64_t)a * ndof + i] * X[(int64_t)a * ndof + j];
      q += D[(int64_t)i * N3 + a] * Pi[(int64_t)a * ndof + j] + D[(int64_t)j * N3 + a] * Pi[(int64_t)a * ndof + i];
    }
    Mo[e] = s - vol * q + (i == j ? vol : 0.0);
  }
}

// ---- loads: F_P[g] = |P| (H_{k-1}^{-1} int_P f m)_g; boundary g = -sigma T_f^T int_f p_D m^f --------
template <int K>
__global__ void k_pk_load_tets(int64_t ntet, int npts, const double* __restrict__ ref, const double* __restrict__ refw,
                               const int* __restrict__ tet_inc, const int* __restrict__ tet_a,
                               const int* __restrict__ inc_cell, const double* __restrict__ xyz,
                               const int* __restrict__ fptr, const int* __restrict__ fvtx,
                               const int* __restrict__ cface, const int8_t* __restrict__ csign,
                               const double* __restrict__ xref, const double* __restrict__ ccen,
                               const double* __restrict__ cdiam, const double* __restrict__ fq, double* tet_sum) {
  constexpr int NS1 = PK<K>::NS1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntet) return;
  const int j = tet_inc[t], a = tet_a[t];
  const int P = inc_cell[j];
  const int f = cface[j];
  const int fs = fptr[f];
  const double Ox = xref[3 * P], Oy = xref[3 * P + 1], Oz = xref[3 * P + 2];
  const int v0 = fvtx[fs], va = fvtx[fs + a], vb = fvtx[fs + a + 1];
  const double Ax = xyz[3 * v0] - Ox, Ay = xyz[3 * v0 + 1] - Oy, Az = xyz[3 * v0 + 2] - Oz;
  const double Bx = xyz[3 * va] - Ox, By = xyz[3 * va + 1] - Oy, Bz = xyz[3 * va + 2] - Oz;
  const double Cx = xyz[3 * vb] - Ox, Cy = xyz[3 * vb + 1] - Oy, Cz = xyz[3 * vb + 2] - Oz;
  const double det = (Ax * (By * Cz - Bz * Cy) - Ay * (Bx * Cz - Bz * Cx) + Az * (Bx * Cy - By * Cx)) * (double)csign[j];
  const double px = ccen[3 * P], py = ccen[3 * P + 1], pz = ccen[3 * P + 2], ih = 1.0 / cdiam[P];
  double acc[NS1];
  for (int g = 0; g < NS1; ++g) acc[g] = 0.0;
  const double* fv = fq + t * npts;
  for (int r = 0; r < npts; ++r) {
    const double xi = ref[3 * r], eta = ref[3 * r + 1], ze = ref[3 * r + 2];
    const double X = Ox + xi * Ax + eta * Bx + ze * Cx, Y = Oy + xi * Ay + eta * By + ze * Cy,
                 Z = Oz + xi * Az + eta * Bz + ze * Cz;
    const double w = refw[r] * fv[r];
    for (int g = 0; g < NS1; ++g) {
      int g1, g2, g3;
      exp3(g, g1, g2, g3);
      acc[g] += w * ipow((X - px) * ih, g1) * ipow((Y - py) * ih, g2) * ipow((Z - pz) * ih, g3);
    }
  }
  for (int g = 0; g < NS1; ++g) tet_sum[t * NS1 + g] = det * acc[g];
}

template <int K>
__global__ void k_pk_load_cells(int nc, const int* __restrict__ ctp, const double* __restrict__ tet_sum,
                                const double* __restrict__ cmom, const double* __restrict__ cvol, double* rhs_p) {
  constexpr int NS1 = PK<K>::NS1, NSM = PK<K>::NSM;
  const int P = blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= nc) return;
  double m[NS1];
  for (int g = 0; g < NS1; ++g) m[g] = 0.0;
  for (int t = ctp[P]; t < ctp[P + 1]; ++t)
    for (int g = 0; g < NS1; ++g) m[g] += tet_sum[(int64_t)t * NS1 + g];
  double H[NS1 * NS1];
  for (int a = 0; a < NS1; ++a)
    for (int b = 0; b < NS1; ++b) {
      int a1, a2, a3, b1, b2, b3;
      exp3(a, a1, a2, a3);
      exp3(b, b1, b2, b3);
      H[a * NS1 + b] = cmom[(int64_t)P * NSM + idx3(a1 + b1, a2 + b2, a3 + b3)];
    }
  cholesky<NS1>(H);
  chol_solve<NS1>(H, m);
  const double v = cvol[P];
  for (int g = 0; g < NS1; ++g) rhs_p[(int64_t)P * NS1 + g] = -v * m[g];
}

template <int K>
__global__ void k_pk_bnd_rhs(int nb, int npts, const double* __restrict__ ref, const double* __restrict__ refw,
                             const int* __restrict__ bface, const int* __restrict__ btp,
                             const double* __restrict__ xyz, const int* __restrict__ fptr,
                             const int* __restrict__ fvtx, const int* __restrict__ face_cell,
                             const double* __restrict__ fcen, const double* __restrict__ fdiam,
                             const double* __restrict__ fe1, const double* __restrict__ fe2,
                             const double* __restrict__ Tf, const double* __restrict__ pq, double* rhs_u) {
  constexpr int NFD = PK<K>::NFD;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const int f = bface[i];
  const int fs = fptr[f], nv = fptr[f + 1] - fs;
  const double fx = fcen[3 * f], fy = fcen[3 * f + 1], fz = fcen[3 * f + 2], ihf = 1.0 / fdiam[f];
  const double e1x = fe1[3 * f], e1y = fe1[3 * f + 1], e1z = fe1[3 * f + 2];
  const double e2x = fe2[3 * f], e2y = fe2[3 * f + 1], e2z = fe2[3 * f + 2];
  double acc[NFD];
  for (int d = 0; d < NFD; ++d) acc[d] = 0.0;
  int64_t q = (int64_t)btp[i] * npts;
  const int v0 = fvtx[fs];
  const double Ax = xyz[3 * v0], Ay = xyz[3 * v0 + 1], Az = xyz[3 * v0 + 2];
  for (int a = 1; a + 1 < nv; ++a) {
    const int va = fvtx[fs + a], vb = fvtx[fs + a + 1];
    const double Bx = xyz[3 * va] - Ax, By = xyz[3 * va + 1] - Ay, Bz = xyz[3 * va + 2] - Az;
    const double Cx = xyz[3 * vb] - Ax, Cy = xyz[3 * vb + 1] - Ay, Cz = xyz[3 * vb + 2] - Az;
    const double nx = By * Cz - Bz * Cy, ny = Bz * Cx - Bx * Cz, nz = Bx * Cy - By * Cx;
    const double a2 = sqrt(nx * nx + ny * ny + nz * nz);
    for (int r = 0; r < npts; ++r, ++q) {
      const double xi = ref[2 * r], eta = ref[2 * r + 1];
      const double dx = Ax + xi * Bx + eta * Cx - fx, dy = Ay + xi * By + eta * Cy - fy,
                   dz = Az + xi * Bz + eta * Cz - fz;
      const double s = (dx * e1x + dy * e1y + dz * e1z) * ihf, t = (dx * e2x + dy * e2y + dz * e2z) * ihf;
      const double w = a2 * refw[r] * pq[q];
      for (int d = 0; d < NFD; ++d) {
        int d1, d2;
        exp2(d, d1, d2);
        acc[d] += w * ipow(s, d1) * ipow(t, d2);
      }
    }
  }
  const double sg = face_cell[2 * f] >= 0 ? 1.0 : -1.0;
  const double* T = Tf + (int64_t)f * NFD * NFD;
  for (int b = 0; b < NFD; ++b) {
    double s = 0.0;
    for (int d = 0; d < NFD; ++d) s += T[d * NFD + b] * acc[d];
    rhs_u[(int64_t)f * NFD + b] = -sg * s;
  }
}

inline int g256(int64_t n) { return (int)((n + 255) / 256); }

template <int K>
void run_local(const PaperLocalArgs& a) {
  using C = PK<K>;
  hipStream_t s = a.s;
  k_pk_face_moments<K><<<(int)a.ninc, 64, 0, s>>>(a.ninc, a.inc_cell, a.cface, a.xyz, a.fptr, a.fvtx,
                                                              a.fcen, a.fdiam, a.fe1, a.fe2, a.ccen, a.cdiam,
                                                              a.tri_ref, a.FP, a.FM);
  k_pk_face_gram<K><<<g256(a.nf), 256, 0, s>>>(a.nf, a.xyz, a.fptr, a.fvtx, a.farea, a.fcen, a.fdiam, a.fe1, a.fe2,
                                               a.tri_ref, a.Tf);
  k_pk_cell<K><<<a.nc, 256, 0, s>>>(a.nc, a.cptr, a.cface, a.csign, a.farea, a.fnormal, a.fcen, a.cvol, a.ccen,
                                    a.cdiam, a.FP, a.FM, a.Tf, a.ldof_ptr, a.Dg, a.Pg, a.Xg, a.Cg, a.lmat_ptr, a.M1,
                                    a.lb_ptr, a.Bdiv1, a.cmom);
  (void)sizeof(C);
}

// Prescribed boundary fluxes (flux boundary data): the face moments (1/|f|) int_f (u.n_f) m^f_b
// (eq. facePoly) of a boundary face, from u at the face points (structure of arrays).
template <int K>
__global__ void k_pk_bnd_flux(int nb, int npts, int64_t total, const double* __restrict__ ref,
                              const double* __restrict__ refw, const int* __restrict__ bface,
                              const int* __restrict__ btp, const double* __restrict__ xyz,
                              const int* __restrict__ fptr, const int* __restrict__ fvtx,
                              const double* __restrict__ fcen, const double* __restrict__ fdiam,
                              const double* __restrict__ fe1, const double* __restrict__ fe2,
                              const double* __restrict__ fnormal, const double* __restrict__ farea,
                              const double* __restrict__ uq, double* xB) {
  constexpr int NFD = PK<K>::NFD;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const int f = bface[i];
  const int fs = fptr[f], nv = fptr[f + 1] - fs;
  const double fx = fcen[3 * f], fy = fcen[3 * f + 1], fz = fcen[3 * f + 2], ihf = 1.0 / fdiam[f];
  const double e1x = fe1[3 * f], e1y = fe1[3 * f + 1], e1z = fe1[3 * f + 2];
  const double e2x = fe2[3 * f], e2y = fe2[3 * f + 1], e2z = fe2[3 * f + 2];
  const double nx0 = fnormal[3 * f], ny0 = fnormal[3 * f + 1], nz0 = fnormal[3 * f + 2];
  double acc[NFD];
  for (int d = 0; d < NFD; ++d) acc[d] = 0.0;
  int64_t q = (int64_t)btp[i] * npts;
  const int v0 = fvtx[fs];
  const double Ax = xyz[3 * v0], Ay = xyz[3 * v0 + 1], Az = xyz[3 * v0 + 2];
  for (int a = 1; a + 1 < nv; ++a) {
    const int va = fvtx[fs + a], vb = fvtx[fs + a + 1];
    const double Bx = xyz[3 * va] - Ax, By = xyz[3 * va + 1] - Ay, Bz = xyz[3 * va + 2] - Az;
    const double Cx = xyz[3 * vb] - Ax, Cy = xyz[3 * vb + 1] - Ay, Cz = xyz[3 * vb + 2] - Az;
    const double nx = By * Cz - Bz * Cy, ny = Bz * Cx - Bx * Cz, nz = Bx * Cy - By * Cx;
    const double a2 = sqrt(nx * nx + ny * ny + nz * nz);
    for (int r = 0; r < npts; ++r, ++q) {
      const double xi = ref[2 * r], eta = ref[2 * r + 1];
      const double dx = Ax + xi * Bx + eta * Cx - fx, dy = Ay + xi * By + eta * Cy - fy,
                   dz = Az + xi * Bz + eta * Cz - fz;
      const double s = (dx * e1x + dy * e1y + dz * e1z) * ihf, t = (dx * e2x + dy * e2y + dz * e2z) * ihf;
      const double un = uq[q] * nx0 + uq[total + q] * ny0 + uq[2 * total + q] * nz0;
      const double w = a2 * refw[r] * un;
      for (int d = 0; d < NFD; ++d) {
        int d1, d2;
        exp2(d, d1, d2);
        acc[d] += w * ipow(s, d1) * ipow(t, d2);
      }
    }
  }
  for (int b = 0; b < NFD; ++b) xB[(int64_t)f * NFD + b] = acc[b] / farea[f];
}

template <int K>
void run_loads(const PaperLoadArgs& a) {
  hipStream_t s = a.s;
  if (a.ntet > 0)
    k_pk_load_tets<K><<<g256(a.ntet), 256, 0, s>>>(a.ntet, a.npts_cell, a.ref_cell, a.w_cell, a.tet_inc, a.tet_a,
                                                   a.inc_cell, a.xyz, a.fptr, a.fvtx, a.cface, a.csign, a.xref,
                                                   a.ccen, a.cdiam, a.fq, a.tet_sum);
  k_pk_load_cells<K><<<g256(a.nc), 256, 0, s>>>(a.nc, a.cell_tet_ptr, a.tet_sum, a.cmom, a.cvol, a.rhs_p);
  if (a.pq && a.nb > 0)
    k_pk_bnd_rhs<K><<<g256(a.nb), 256, 0, s>>>(a.nb, a.npts_face, a.ref_face, a.w_face, a.bface, a.btri_ptr, a.xyz,
                                               a.fptr, a.fvtx, a.face_cell, a.fcen, a.fdiam, a.fe1, a.fe2, a.Tf,
                                               a.pq, a.rhs_u);
  if (a.uq && a.nb > 0)
    k_pk_bnd_flux<K><<<g256(a.nb), 256, 0, s>>>(a.nb, a.npts_face, a.nq_face_total, a.ref_face, a.w_face, a.bface,
                                                a.btri_ptr, a.xyz, a.fptr, a.fvtx, a.fcen, a.fdiam, a.fe1, a.fe2,
                                                a.fnormal, a.farea, a.uq, a.xB);
}

}  // namespace

PaperSizes paper_sizes(int k) {
  PaperSizes z{};
  z.nfd = dimP2(k);
  z.npd = dimP3(k - 1);
  z.nint = dimP3(k - 1) - 1 + dimGp(k);
  z.n3 = 3 * dimP3(k);
  z.nsm = dimP3(2 * k);
  z.nfm = dimP2(k) * dimP3(k + 1);
  z.nq = k + 1;
  return z;
}

void launch_paper_local(int k, const PaperLocalArgs& a) {
  switch (k) {
    case 1: run_local<1>(a); break;
    case 2: run_local<2>(a); break;
    case 3: run_local<3>(a); break;
    default: throw Error{VEM_EINVAL, "the paper's element is built for k = 1, 2, 3"};
  }
}

void launch_paper_loads(int k, const PaperLoadArgs& a) {
  switch (k) {
    case 1: run_loads<1>(a); break;
    case 2: run_loads<2>(a); break;
    case 3: run_loads<3>(a); break;
    default: throw Error{VEM_EINVAL, "the paper's element is built for k = 1, 2, 3"};
  }
}

}  // namespace vem
