// Local matrices of the lowest-order mixed virtual element (face space P_0,
// divergence and pressure P_0), one thread per local row.
//
// With c_i = |f_i| (x_{f_i} - x_P) and n_i the outward unit normal of face i,
// the paper's construction (Section 4.1: DOFs of eq. facePoly, divergence and
// L2 projector through integration by parts; Section 4.3: stabilised form)
// gives for the lowest order
//   D[i, c] = n_i[c]          (DOFs of the constant fields e_c),
//   Pi*     = C^T / |P|        (int_P phi_i . e_c = c_i[c], G = |P| I),
//   div phi_i = |f_i| / |P|,
// hence, expanding M_P = nu [Pi*^T G Pi* + |P| (I - D Pi*)^T (I - D Pi*)],
//   M1[i][j] = (c_i.c_j + c_i^T (N^T N) c_j) / |P| + |P| delta_ij - n_i.c_j - n_j.c_i
// with N^T N = sum_k n_k n_k^T, and B_div,P[i] = int_P div phi_i = |f_i|.
// M1 is the coefficient-free (nu = 1) matrix; the global flux block scales it
// by nu_P cell by cell.
#include "vem_internal.h"

namespace vem {
namespace {

__global__ void k_lo_local(int64_t ninc, const int* __restrict__ inc_cell, const int* __restrict__ cptr,
                           const int* __restrict__ cface, const int8_t* __restrict__ csign,
                           const double* __restrict__ farea, const double* __restrict__ fnormal,
                           const double* __restrict__ fcen, const double* __restrict__ cvol,
                           const double* __restrict__ ccen, const int64_t* __restrict__ lmat_ptr, double* M1,
                           const int64_t* __restrict__ lb_ptr, double* Bdiv1) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ninc) return;
  int P = inc_cell[t];
  int s = cptr[P], F = cptr[P + 1] - s;
  int i = (int)(t - s);
  double vol = cvol[P];
  double px = ccen[3 * P], py = ccen[3 * P + 1], pz = ccen[3 * P + 2];
  // N^T N (symmetric 3x3); the sign of n_k cancels
  double nxx = 0, nxy = 0, nxz = 0, nyy = 0, nyz = 0, nzz = 0;
  for (int k = 0; k < F; ++k) {
    int f = cface[s + k];
    double a = fnormal[3 * f], b = fnormal[3 * f + 1], c = fnormal[3 * f + 2];
    nxx += a * a;
    nxy += a * b;
    nxz += a * c;
    nyy += b * b;
    nyz += b * c;
    nzz += c * c;
  }
  int fi = cface[s + i];
  double si = (double)csign[s + i];
  double ai = farea[fi];
  double cix = ai * (fcen[3 * fi] - px), ciy = ai * (fcen[3 * fi + 1] - py), ciz = ai * (fcen[3 * fi + 2] - pz);
  double nix = si * fnormal[3 * fi], niy = si * fnormal[3 * fi + 1], niz = si * fnormal[3 * fi + 2];
  // (N^T N) c_i
  double tx = nxx * cix + nxy * ciy + nxz * ciz;
  double ty = nxy * cix + nyy * ciy + nyz * ciz;
  double tz = nxz * cix + nyz * ciy + nzz * ciz;
  double* row = M1 + lmat_ptr[P] + (int64_t)i * F;
  for (int j = 0; j < F; ++j) {
    int fj = cface[s + j];
    double sj = (double)csign[s + j];
    double aj = farea[fj];
    double cjx = aj * (fcen[3 * fj] - px), cjy = aj * (fcen[3 * fj + 1] - py), cjz = aj * (fcen[3 * fj + 2] - pz);
    double njx = sj * fnormal[3 * fj], njy = sj * fnormal[3 * fj + 1], njz = sj * fnormal[3 * fj + 2];
    double v = (cix * cjx + ciy * cjy + ciz * cjz + tx * cjx + ty * cjy + tz * cjz) / vol;
    v -= nix * cjx + niy * cjy + niz * cjz;
    v -= njx * cix + njy * ciy + njz * ciz;
    if (j == i) v += vol;
    row[j] = v;
  }
  Bdiv1[lb_ptr[P] + i] = ai;
}

}  // namespace

void launch_lo_local(hipStream_t s, int64_t ninc, const int* inc_cell, const int* cptr, const int* cface,
                     const int8_t* csign, const double* farea, const double* fnormal, const double* fcen,
                     const double* cvol, const double* ccen, const int64_t* lmat_ptr, double* M1,
                     const int64_t* lb_ptr, double* Bdiv1) {
  if (ninc <= 0) return;
  k_lo_local<<<(int)((ninc + 255) / 256), 256, 0, s>>>(ninc, inc_cell, cptr, cface, csign, farea, fnormal, fcen,
                                                       cvol, ccen, lmat_ptr, M1, lb_ptr, Bdiv1);
}

}  // namespace vem
