// Mesh validation, face/cell geometry, tetrahedral splitting and quadrature
// kernels.  Geometry follows the definitions of Section 2 of the paper
// (barycentres and diameters of faces and cells); the splitting of cells
// into tetrahedra and faces into triangles carries the load quadrature
// (Remark of Section 4.3: the load term depends only on the rule used).
#include "vem_internal.h"

namespace vem {
namespace {

constexpr int kThreads = 256;

inline int nblocks(int64_t n, int t = kThreads) { return (int)((n + t - 1) / t); }

struct V3 {
  double x, y, z;
};
__device__ inline V3 ld3(const double* p, int64_t i) { return {p[3 * i], p[3 * i + 1], p[3 * i + 2]}; }
__device__ inline void st3(double* p, int64_t i, V3 v) {
  p[3 * i] = v.x;
  p[3 * i + 1] = v.y;
  p[3 * i + 2] = v.z;
}
// structure of arrays: x[0..n), y[n..2n), z[2n..3n)
__device__ inline void st3_soa(double* p, int64_t n, int64_t i, V3 v) {
  p[i] = v.x;
  p[n + i] = v.y;
  p[2 * n + i] = v.z;
}
__device__ inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
__device__ inline double norm(V3 a) { return sqrt(dot(a, a)); }

// --- validation and face -> cell incidence -------------------------------------------------
// Offset arrays of a mesh handed over in device memory: both start at 0 and never decrease.
// out[0] collects error bits (1: face_ptr decreases, 2: cell_ptr decreases, 4: a first entry
// is not 0), out[1] the largest number of faces of a cell; one atomic per block.
__global__ void __launch_bounds__(kThreads) k_check_offsets(int64_t nf, const int* __restrict__ fptr, int64_t nc,
                                                            const int* __restrict__ cptr, int* out) {
  __shared__ int sh[kThreads / 64][2];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int err = 0, m = 0;
  if (i < nf && fptr[i + 1] < fptr[i]) err |= 1;
  if (i < nc) {
    const int d = cptr[i + 1] - cptr[i];
    if (d < 0) err |= 2;
    m = d;
  }
  if (i == 0 && (fptr[0] != 0 || cptr[0] != 0)) err |= 4;
  for (int o = 32; o > 0; o >>= 1) {
    err |= __shfl_xor(err, o, 64);
    const int mo = __shfl_xor(m, o, 64);
    m = mo > m ? mo : m;
  }
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x >> 6][0] = err;
    sh[threadIdx.x >> 6][1] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / 64; ++w) {
      err |= sh[w][0];
      m = sh[w][1] > m ? sh[w][1] : m;
    }
    if (err) atomicOr(out, err);
    if (m > 0) atomicMax(out + 1, m);
  }
}

__global__ void k_check_mesh(int nv, int nf, int nc, const int* __restrict__ fptr, const int* __restrict__ fvtx,
                             const int* __restrict__ cptr, const int* __restrict__ cface,
                             const int8_t* __restrict__ csign, int* face_cnt, int* face_cell, int* face_lidx,
                             int* inc_cell, int* err) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nf) {
    int s = fptr[t], e = fptr[t + 1];
    if (e - s < 3) atomicOr(err, 8);
    for (int j = s; j < e; ++j) {
      int v = fvtx[j];
      if (v < 0 || v >= nv) atomicOr(err, 16);
    }
  }
  if (t < nc) {
    int s = cptr[t], e = cptr[t + 1];
    if (e - s < 4 || e - s > kMaxCellFaces) atomicOr(err, 1);
    for (int j = s; j < e; ++j) {
      inc_cell[j] = t;
      int f = cface[j];
      int sg = csign[j];
      if (f < 0 || f >= nf) {
        atomicOr(err, 2);
        continue;
      }
      if (sg != 1 && sg != -1) {
        atomicOr(err, 4);
        continue;
      }
      int slot = 2 * f + (sg > 0 ? 0 : 1);
      int old = atomicAdd(&face_cnt[slot], 1);
      if (old == 0) {
        face_cell[slot] = t;
        face_lidx[slot] = j - s;
      }
    }
  }
}

__global__ void k_check_faces(int nf, const int* __restrict__ cnt, const double* __restrict__ area, int* is_bnd,
                              int* err) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int c0 = cnt[2 * f], c1 = cnt[2 * f + 1];
  if (c0 > 1 || c1 > 1 || c0 + c1 == 0) atomicOr(err, 32);
  is_bnd[f] = (c0 + c1 == 1) ? 1 : 0;
  double a = area[f];
  if (!(a > 0.0) || !isfinite(a)) atomicOr(err, 64);
}

__global__ void k_check_cells(int nc, const double* __restrict__ vol, int* err) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  double v = vol[c];
  if (!(v > 0.0) || !isfinite(v)) atomicOr(err, 128);
}

// --- geometry -------------------------------------------------------------------------------
// Face: area vector from the fan (v0, v_a, v_{a+1}); unit normal; area centroid;
// diameter (largest vertex distance); frame e1 = longest loop edge, e2 = n x e1.
__global__ void k_face_geometry(int nf, const double* __restrict__ xyz, const int* __restrict__ fptr,
                                const int* __restrict__ fvtx, double* area, double* normal, double* cen,
                                double* diam, double* e1, double* e2) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int s = fptr[f], n = fptr[f + 1] - s;
  V3 A = ld3(xyz, fvtx[s]);
  V3 av = {0, 0, 0};
  for (int a = 1; a + 1 < n; ++a) {
    V3 B = ld3(xyz, fvtx[s + a]), C = ld3(xyz, fvtx[s + a + 1]);
    av = av + 0.5 * cross(B - A, C - A);
  }
  double ar = norm(av);
  V3 nr = (1.0 / ar) * av;
  V3 cs = {0, 0, 0};
  for (int a = 1; a + 1 < n; ++a) {
    V3 B = ld3(xyz, fvtx[s + a]), C = ld3(xyz, fvtx[s + a + 1]);
    double ta = dot(0.5 * cross(B - A, C - A), nr);
    cs = cs + (ta / 3.0) * (A + B + C);
  }
  double dmax = 0.0, lmax = -1.0;
  V3 emax = {0, 0, 0};
  for (int i = 0; i < n; ++i) {
    V3 P = ld3(xyz, fvtx[s + i]);
    V3 Q = ld3(xyz, fvtx[s + (i + 1) % n]);
    V3 E = Q - P;
    double l = norm(E);
    if (l > lmax) {
      lmax = l;
      emax = E;
    }
    for (int j = i + 1; j < n; ++j) dmax = fmax(dmax, norm(ld3(xyz, fvtx[s + j]) - P));
  }
  V3 u1 = (1.0 / lmax) * emax;
  area[f] = ar;
  st3(normal, f, nr);
  st3(cen, f, (1.0 / ar) * cs);
  diam[f] = dmax;
  st3(e1, f, u1);
  st3(e2, f, cross(nr, u1));
}

// Cell: x_ref = mean over face-vertex incidences; volume and centroid summed over the
// tetrahedra (x_ref, v0, v_a, v_{a+1}) signed by sigma; diameter over vertex pairs.
__global__ void k_cell_geometry(int nc, const double* __restrict__ xyz, const int* __restrict__ fptr,
                                const int* __restrict__ fvtx, const int* __restrict__ cptr,
                                const int* __restrict__ cface, const int8_t* __restrict__ csign, double* vol,
                                double* cen, double* diam, double* xref) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  int s = cptr[c], e = cptr[c + 1];
  V3 O = {0, 0, 0};
  int cnt = 0;
  for (int j = s; j < e; ++j) {
    int f = cface[j];
    int fs = fptr[f], fe = fptr[f + 1];
    V3 fsum = {0, 0, 0};
    for (int q = fs; q < fe; ++q) fsum = fsum + ld3(xyz, fvtx[q]);
    O = O + fsum;
    cnt += fe - fs;
  }
  O = (1.0 / cnt) * O;
  double v = 0.0;
  V3 m = {0, 0, 0};
  for (int j = s; j < e; ++j) {
    int f = cface[j];
    double sg = (double)csign[j];
    int fs = fptr[f], n = fptr[f + 1] - fs;
    V3 A = ld3(xyz, fvtx[fs]);
    for (int a = 1; a + 1 < n; ++a) {
      V3 B = ld3(xyz, fvtx[fs + a]), C = ld3(xyz, fvtx[fs + a + 1]);
      double t = dot(A - O, cross(B - O, C - O)) * sg / 6.0;
      v += t;
      m = m + (t / 4.0) * (O + A + B + C);
    }
  }
  // largest vertex-vertex distance; squared distances are compared and one root taken
  // (the root is monotone and correctly rounded, so this is the same number).  Every vertex of
  // face j is compared with every vertex of the faces j2 >= j: a face of at most kFaceV vertices
  // is held in registers (its padding slots repeat its first vertex, which leaves the maximum
  // unchanged), so each vertex of the later faces is loaded once per face j rather than once per
  // vertex of face j.  A wavefront per cell with the incidences staged in LDS was measured slower:
  // the chain of dependent index loads dominates, and a thread per cell overlaps 64 of them per
  // wave.
  constexpr int kFaceV = 8;
  double dmax2 = 0.0;
  for (int j = s; j < e; ++j) {
    const int f = cface[j];
    const int fs = fptr[f], nj = fptr[f + 1] - fs;
    if (nj <= kFaceV) {
      V3 P[kFaceV];
#pragma unroll
      for (int u = 0; u < kFaceV; ++u) P[u] = ld3(xyz, fvtx[fs + (u < nj ? u : 0)]);
      for (int j2 = j; j2 < e; ++j2) {
        const int f2 = cface[j2];
        for (int q2 = fptr[f2]; q2 < fptr[f2 + 1]; ++q2) {
          const V3 Q = ld3(xyz, fvtx[q2]);
#pragma unroll
          for (int u = 0; u < kFaceV; ++u) {
            const V3 d = Q - P[u];
            dmax2 = fmax(dmax2, dot(d, d));
          }
        }
      }
    } else {
      for (int q = fs; q < fs + nj; ++q) {
        const V3 P = ld3(xyz, fvtx[q]);
        for (int j2 = j; j2 < e; ++j2) {
          const int f2 = cface[j2];
          for (int q2 = fptr[f2]; q2 < fptr[f2 + 1]; ++q2) {
            const V3 d = ld3(xyz, fvtx[q2]) - P;
            dmax2 = fmax(dmax2, dot(d, d));
          }
        }
      }
    }
  }
  vol[c] = v;
  st3(cen, c, (1.0 / v) * m);
  diam[c] = sqrt(dmax2);
  st3(xref, c, O);
}

// --- tetrahedra and quadrature --------------------------------------------------------------
__global__ void k_tet_counts(int nc, const int* __restrict__ fptr, const int* __restrict__ cptr,
                             const int* __restrict__ cface, int* cnt) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  int t = 0;
  for (int j = cptr[c]; j < cptr[c + 1]; ++j) {
    int f = cface[j];
    t += fptr[f + 1] - fptr[f] - 2;
  }
  cnt[c] = t;
}

__global__ void k_tets(int nc, const int* __restrict__ fptr, const int* __restrict__ cptr,
                       const int* __restrict__ cface, const int* __restrict__ ctp, int* tet_inc, int* tet_a) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  int t = ctp[c];
  for (int j = cptr[c]; j < cptr[c + 1]; ++j) {
    int f = cface[j];
    int n = fptr[f + 1] - fptr[f];
    for (int a = 1; a + 1 < n; ++a) {
      tet_inc[t] = j;
      tet_a[t] = a;
      ++t;
    }
  }
}

__global__ void k_bnd_tri_counts(int nb, const int* __restrict__ bface, const int* __restrict__ fptr, int* cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  int f = bface[i];
  cnt[i] = fptr[f + 1] - fptr[f] - 2;
}

// Points x = O + xi (v0 - O) + eta (v_a - O) + zeta (v_{a+1} - O).  A block takes a run of
// whole tetrahedra (about 4096 points, at most kQpTets tetrahedra): their corners are fetched
// once into LDS by one thread each, then the block's threads write the run's points in
// order, so that consecutive threads store consecutive entries of each coordinate array.  The
// reference points are staged in LDS too, so the write loop reads no global memory.  LDS is
// sized to the run (about 15 KB at 27 points per tetrahedron), which leaves room for eight
// blocks per CU to overlap their corner fetches (chains of dependent index loads).
constexpr int kQpTets = 256;
constexpr int kQpRefMax = 216;  // reference points per tetrahedron: 6 per direction at most
inline int qp_tets_per_block(int npts) {
  const int t = 8192 / (npts > 0 ? npts : 1);
  return t < 1 ? 1 : (t > kQpTets ? kQpTets : t);
}
inline size_t qp_lds_bytes(int npts) {
  return sizeof(double) * (12 * (size_t)qp_tets_per_block(npts) + 3 * (size_t)npts);
}

__global__ void __launch_bounds__(kThreads) k_qp_cell(int64_t ntet, int npts, int tets_per_block,
                                                      const double* __restrict__ ref,
                                                      const int* __restrict__ tet_inc, const int* __restrict__ tet_a,
                                                      const int* __restrict__ inc_cell, const double* __restrict__ xyz,
                                                      const int* __restrict__ fptr, const int* __restrict__ fvtx,
                                                      const int* __restrict__ cface, const double* __restrict__ xref,
                                                      double* qp) {
  extern __shared__ double qp_lds[];
  double* corner = qp_lds;                        // [tets_per_block][12]: O, v0, v_a, v_{a+1}
  double* sref = qp_lds + 12 * tets_per_block;  // [3 npts]
  const int64_t t0 = (int64_t)blockIdx.x * tets_per_block;
  const int nt = (int)(ntet - t0 < tets_per_block ? ntet - t0 : tets_per_block);
  {
    constexpr int kPer = (3 * kQpRefMax + kThreads - 1) / kThreads;
    const int nr = 3 * npts;
    double rv[kPer];  // slots past the table reload its last entry (no branch around a load)
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int q = threadIdx.x + u * kThreads;
      rv[u] = ref[q < nr ? q : nr - 1];
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int q = threadIdx.x + u * kThreads;
      if (q < nr) sref[q] = rv[u];
    }
  }
  for (int i = threadIdx.x; i < nt; i += kThreads) {
    const int64_t t = t0 + i;
    const int j = tet_inc[t], a = tet_a[t];
    const int fs = fptr[cface[j]];
    const V3 v[4] = {ld3(xref, inc_cell[j]), ld3(xyz, fvtx[fs]), ld3(xyz, fvtx[fs + a]), ld3(xyz, fvtx[fs + a + 1])};
    for (int c = 0; c < 4; ++c) {
      corner[12 * i + 3 * c] = v[c].x;
      corner[12 * i + 3 * c + 1] = v[c].y;
      corner[12 * i + 3 * c + 2] = v[c].z;
    }
  }
  __syncthreads();
  const int64_t total = ntet * npts, q0 = t0 * npts;
  const int np = nt * npts;
  for (int q = threadIdx.x; q < np; q += kThreads) {
    const int i = q / npts, r = q - i * npts;
    const double* c = corner + 12 * i;
    const V3 O{c[0], c[1], c[2]}, A{c[3], c[4], c[5]}, B{c[6], c[7], c[8]}, C{c[9], c[10], c[11]};
    const double xi = sref[3 * r], eta = sref[3 * r + 1], zeta = sref[3 * r + 2];
    st3_soa(qp, total, q0 + q, O + xi * (A - O) + eta * (B - O) + zeta * (C - O));
  }
}

// Boundary-face points: triangles (v0, v_a, v_{a+1}), x = v0 + xi (v_a - v0) + eta (v_{a+1} - v0).
__global__ void k_qp_face(int nb, int npts, int64_t total, const double* __restrict__ ref,
                          const int* __restrict__ bface, const int* __restrict__ btp, const double* __restrict__ xyz,
                          const int* __restrict__ fptr, const int* __restrict__ fvtx, double* qp) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  int f = bface[i];
  int fs = fptr[f], n = fptr[f + 1] - fs;
  int64_t q = (int64_t)btp[i] * npts;
  V3 A = ld3(xyz, fvtx[fs]);
  for (int a = 1; a + 1 < n; ++a) {
    V3 B = ld3(xyz, fvtx[fs + a]), C = ld3(xyz, fvtx[fs + a + 1]);
    for (int r = 0; r < npts; ++r, ++q) st3_soa(qp, total, q, A + ref[2 * r] * (B - A) + ref[2 * r + 1] * (C - A));
  }
}

// Per tetrahedron: sigma det * sum_r w_r f(x_r).  A block takes a run of whole tetrahedra
// (at most kThreads of them, at most kLoadPts points): their point values are contiguous,
// are read into LDS with coalesced loads all in flight at once (a fixed count per thread, so
// that no load waits for the previous one's store), and each thread then sums its own
// tetrahedron's points in order.
constexpr int kLoadPts = 4096;
constexpr int kLoadPerThread = kLoadPts / kThreads;
inline int load_tets_per_block(int npts) {
  const int t = kLoadPts / (npts > 0 ? npts : 1);
  return t < 1 ? 1 : (t > kThreads ? kThreads : t);
}

__global__ void __launch_bounds__(kThreads) k_load_tets(int64_t ntet, int npts, int tets_per_block,
                                                        const double* __restrict__ refw,
                                                        const int* __restrict__ tet_inc, const int* __restrict__ tet_a,
                                                        const int* __restrict__ inc_cell,
                                                        const double* __restrict__ xyz, const int* __restrict__ fptr,
                                                        const int* __restrict__ fvtx, const int* __restrict__ cface,
                                                        const int8_t* __restrict__ csign,
                                                        const double* __restrict__ xref, const double* __restrict__ fq,
                                                        double* tet_sum) {
  __shared__ double vals[kLoadPts];
  const int64_t t0 = (int64_t)blockIdx.x * tets_per_block;
  const int nt = (int)(ntet - t0 < tets_per_block ? ntet - t0 : tets_per_block);
  const int np = nt * npts;
  const int64_t q0 = t0 * npts;
  // The determinant's chain of dependent index loads runs on every thread (threads past the run
  // repeat its last tetrahedron and discard the result), without a branch, so that it proceeds while
  // the point-value loads are in flight.
  double v[kLoadPerThread];  // slots past the run reload its last value (no branch around a load)
#pragma unroll
  for (int u = 0; u < kLoadPerThread; ++u) {
    const int q = threadIdx.x + u * kThreads;
    v[u] = fq[q0 + (q < np ? q : np - 1)];
  }
  const int i = threadIdx.x;
  const int64_t t = t0 + (i < nt ? i : nt - 1);
  const int j = tet_inc[t], a = tet_a[t];
  const int fs = fptr[cface[j]];
  const V3 O = ld3(xref, inc_cell[j]);
  const V3 A = ld3(xyz, fvtx[fs]), B = ld3(xyz, fvtx[fs + a]), C = ld3(xyz, fvtx[fs + a + 1]);
  const double det = dot(A - O, cross(B - O, C - O)) * (double)csign[j];
#pragma unroll
  for (int u = 0; u < kLoadPerThread; ++u) {
    const int q = threadIdx.x + u * kThreads;
    if (q < np) vals[q] = v[u];
  }
  __syncthreads();
  if (i >= nt) return;
  double acc = 0.0;
  for (int r = 0; r < npts; ++r) acc += refw[r] * vals[i * npts + r];
  tet_sum[t0 + i] = det * acc;
}

__global__ void k_load_cells(int nc, const int* __restrict__ ctp, const double* __restrict__ tet_sum,
                             double* rhs_p) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  double acc = 0.0;
  for (int t = ctp[c]; t < ctp[c + 1]; ++t) acc += tet_sum[t];
  rhs_p[c] = -acc;  // pressure rows of b = [g; -F]
}

// g_f = -sigma int_f p_D for the boundary faces (sigma of the single adjacent cell).
__global__ void k_bnd_rhs(int nb, int npts, const double* __restrict__ refw, const int* __restrict__ bface,
                          const int* __restrict__ btp, const double* __restrict__ xyz, const int* __restrict__ fptr,
                          const int* __restrict__ fvtx, const int* __restrict__ face_cell,
                          const double* __restrict__ pq, double* rhs_u) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  int f = bface[i];
  int fs = fptr[f], n = fptr[f + 1] - fs;
  int64_t q = (int64_t)btp[i] * npts;
  V3 A = ld3(xyz, fvtx[fs]);
  double acc = 0.0;
  for (int a = 1; a + 1 < n; ++a) {
    V3 B = ld3(xyz, fvtx[fs + a]), C = ld3(xyz, fvtx[fs + a + 1]);
    double a2 = norm(cross(B - A, C - A));
    double s = 0.0;
    for (int r = 0; r < npts; ++r, ++q) s += refw[r] * pq[q];
    acc += a2 * s;
  }
  double sg = face_cell[2 * f] >= 0 ? 1.0 : -1.0;
  rhs_u[f] = -sg * acc;
}

// Prescribed boundary fluxes (flux boundary data): the DOF of boundary face f is
// (1/|f|) int_f u.n_f, from u at the face points (structure of arrays, `total` points).
__global__ void k_bnd_flux(int nb, int npts, int64_t total, const double* __restrict__ refw,
                           const int* __restrict__ bface, const int* __restrict__ btp, const double* __restrict__ xyz,
                           const int* __restrict__ fptr, const int* __restrict__ fvtx,
                           const double* __restrict__ fnormal, const double* __restrict__ farea,
                           const double* __restrict__ uq, double* xB) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  int f = bface[i];
  int fs = fptr[f], n = fptr[f + 1] - fs;
  int64_t q = (int64_t)btp[i] * npts;
  const V3 nf = ld3(fnormal, f);
  V3 A = ld3(xyz, fvtx[fs]);
  double acc = 0.0;
  for (int a = 1; a + 1 < n; ++a) {
    V3 B = ld3(xyz, fvtx[fs + a]), C = ld3(xyz, fvtx[fs + a + 1]);
    double a2 = norm(cross(B - A, C - A));
    double s = 0.0;
    for (int r = 0; r < npts; ++r, ++q)
      s += refw[r] * (uq[q] * nf.x + uq[total + q] * nf.y + uq[2 * total + q] * nf.z);
    acc += a2 * s;
  }
  xB[f] = acc / farea[f];
}

}  // namespace

void launch_bnd_flux(hipStream_t s, int nb, int npts, int64_t total, const double* refw, const int* bface,
                     const int* btri_ptr, const double* xyz, const int* fptr, const int* fvtx, const double* fnormal,
                     const double* farea, const double* uq, double* xB) {
  if (nb > 0)
    k_bnd_flux<<<nblocks(nb), kThreads, 0, s>>>(nb, npts, total, refw, bface, btri_ptr, xyz, fptr, fvtx, fnormal,
                                                farea, uq, xB);
}

void launch_check_mesh(hipStream_t s, int nv, int nf, int nc, const int* fptr, const int* fvtx, const int* cptr,
                       const int* cface, const int8_t* csign, int* face_cnt, int* face_cell, int* face_lidx,
                       int* inc_cell, int* err) {
  int n = nf > nc ? nf : nc;
  k_check_mesh<<<nblocks(n), kThreads, 0, s>>>(nv, nf, nc, fptr, fvtx, cptr, cface, csign, face_cnt, face_cell,
                                               face_lidx, inc_cell, err);
}
void launch_check_offsets(hipStream_t s, int64_t nf, const int* fptr, int64_t nc, const int* cptr, int* out) {
  const int64_t n = nf > nc ? nf : nc;
  if (n > 0) k_check_offsets<<<(int)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(nf, fptr, nc, cptr, out);
}
void launch_check_faces(hipStream_t s, int nf, const int* face_cnt, const double* area, int* is_bnd, int* err) {
  k_check_faces<<<nblocks(nf), kThreads, 0, s>>>(nf, face_cnt, area, is_bnd, err);
}
void launch_check_cells(hipStream_t s, int nc, const double* vol, int* err) {
  k_check_cells<<<nblocks(nc), kThreads, 0, s>>>(nc, vol, err);
}
void launch_face_geometry(hipStream_t s, int nf, const double* xyz, const int* fptr, const int* fvtx, double* area,
                          double* normal, double* cen, double* diam, double* e1, double* e2) {
  k_face_geometry<<<nblocks(nf), kThreads, 0, s>>>(nf, xyz, fptr, fvtx, area, normal, cen, diam, e1, e2);
}
void launch_cell_geometry(hipStream_t s, int nc, const double* xyz, const int* fptr, const int* fvtx,
                          const int* cptr, const int* cface, const int8_t* csign, double* vol, double* cen,
                          double* diam, double* xref) {
  k_cell_geometry<<<nblocks(nc), kThreads, 0, s>>>(nc, xyz, fptr, fvtx, cptr, cface, csign, vol, cen, diam, xref);
}
void launch_tet_counts(hipStream_t s, int nc, const int* fptr, const int* cptr, const int* cface, int* cnt) {
  k_tet_counts<<<nblocks(nc), kThreads, 0, s>>>(nc, fptr, cptr, cface, cnt);
}
void launch_tets(hipStream_t s, int nc, const int* fptr, const int* cptr, const int* cface, const int* cell_tet_ptr,
                 int* tet_inc, int* tet_a) {
  k_tets<<<nblocks(nc), kThreads, 0, s>>>(nc, fptr, cptr, cface, cell_tet_ptr, tet_inc, tet_a);
}
void launch_bnd_tri_counts(hipStream_t s, int nb, const int* bface, const int* fptr, int* cnt) {
  if (nb > 0) k_bnd_tri_counts<<<nblocks(nb), kThreads, 0, s>>>(nb, bface, fptr, cnt);
}
void launch_qp_cell(hipStream_t s, int64_t ntet, int npts, const double* ref, const int* tet_inc, const int* tet_a,
                    const int* inc_cell, const double* xyz, const int* fptr, const int* fvtx, const int* cface,
                    const double* xref, double* qp) {
  VEM_REQUIRE(npts <= kQpRefMax, VEM_EINVAL, "more cell quadrature points per tetrahedron than staged");
  if (ntet > 0 && npts > 0) {
    const int tpb = qp_tets_per_block(npts);
    k_qp_cell<<<(int)((ntet + tpb - 1) / tpb), kThreads, qp_lds_bytes(npts), s>>>(ntet, npts, tpb, ref, tet_inc,
                                                                                  tet_a, inc_cell, xyz, fptr, fvtx,
                                                                                  cface, xref, qp);
  }
}
void launch_qp_face(hipStream_t s, int nb, int npts, int64_t total, const double* ref, const int* bface,
                    const int* btri_ptr, const double* xyz, const int* fptr, const int* fvtx, double* qp) {
  if (nb > 0)
    k_qp_face<<<nblocks(nb), kThreads, 0, s>>>(nb, npts, total, ref, bface, btri_ptr, xyz, fptr, fvtx, qp);
}
void launch_load_tets(hipStream_t s, int64_t ntet, int npts, const double* refw, const int* tet_inc,
                      const int* tet_a, const int* inc_cell, const double* xyz, const int* fptr, const int* fvtx,
                      const int* cface, const int8_t* csign, const double* xref, const double* fq,
                      double* tet_sum) {
  if (ntet > 0 && npts > 0) {
    const int tpb = load_tets_per_block(npts);
    k_load_tets<<<(int)((ntet + tpb - 1) / tpb), kThreads, 0, s>>>(ntet, npts, tpb, refw, tet_inc, tet_a, inc_cell,
                                                                     xyz, fptr, fvtx, cface, csign, xref, fq, tet_sum);
  }
}
void launch_load_cells(hipStream_t s, int nc, const int* cell_tet_ptr, const double* tet_sum, double* rhs_p) {
  k_load_cells<<<nblocks(nc), kThreads, 0, s>>>(nc, cell_tet_ptr, tet_sum, rhs_p);
}
void launch_bnd_rhs(hipStream_t s, int nb, int npts, const double* refw, const int* bface, const int* btri_ptr,
                    const double* xyz, const int* fptr, const int* fvtx, const int* face_cell, const double* pq,
                    double* rhs_u) {
  if (nb > 0)
    k_bnd_rhs<<<nblocks(nb), kThreads, 0, s>>>(nb, npts, refw, bface, btri_ptr, xyz, fptr, fvtx, face_cell, pq,
                                               rhs_u);
}

}  // namespace vem
