// Internal declarations of the mixed-VEM HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "vem.h"

namespace vem {

struct Error {
  int code;
  std::string msg;
};

#define VEM_HIP(call)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      throw ::vem::Error{VEM_EHIP, std::string(#call) + " failed: " + hipGetErrorString(e_)}; \
  } while (0)

#define VEM_REQUIRE(cond, code, text)                   \
  do {                                                  \
    if (!(cond)) throw ::vem::Error{(code), (text)};    \
  } while (0)

// Owned device buffer.
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    if (count == n && p) return;
    release();
    if (count) {
      hipError_t e = hipMalloc(&p, count * sizeof(T));
      if (e != hipSuccess) {
        p = nullptr;
        throw Error{VEM_ENOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed"};
      }
    }
    n = count;
  }
  // grow-only: keeps the allocation when it is already large enough
  void reserve(size_t count) {
    if (count <= n && p) return;
    alloc(count);
  }
  operator T*() const { return p; }
};

// Pinned host buffer.
template <class T>
struct HBuf {
  T* p = nullptr;
  size_t n = 0;
  HBuf() = default;
  HBuf(const HBuf&) = delete;
  HBuf& operator=(const HBuf&) = delete;
  ~HBuf() {
    if (p) (void)hipHostFree(p);
  }
  void alloc(size_t count, unsigned flags = hipHostMallocDefault) {
    if (count <= n && p) return;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    VEM_HIP(hipHostMalloc((void**)&p, count * sizeof(T), flags));
    n = count;
  }
  T& operator[](size_t i) { return p[i]; }
};

// Grow-only device scratch owned by a handle, for the temporaries of the set-up calls:
// a hipMalloc/hipFree pair per call synchronises the device and costs 0.1-0.5 ms.
// Slots are handed out by the caller; no two live temporaries share a slot.
struct Scratch {
  DBuf<unsigned char> cub;  // hipcub temporary storage
  DBuf<int64_t> i64[8];
  DBuf<int> i32[4];
  DBuf<double> f64[8];
  HBuf<int64_t> tot;        // pinned landing slots for the totals of asynchronous scans
  HBuf<int> ti;             // pinned landing slots for small integer results
};

// Reduction scratch: per-block partial sums.
constexpr int kRedBlocks = 1024;   // grid of the reduction kernels
constexpr int kRedThreads = 256;
constexpr int kMaxDots = 34;       // largest number of simultaneous dot products
constexpr int kMaxRestart = 32;
constexpr int kMaxCellFaces = 64;
// Inner-CG grids: at most 256 CUs x 2048 resident threads, so that the whole grid is
// resident in one round (larger systems loop over rows; a second round of blocks would
// pay the partial-sum prologue again: 10% slower on the 64^3 A_gamma iteration).  The
// FP64 pipelined iteration takes 1024-thread blocks when every row has a thread, and
// 256-thread blocks when threads loop over rows (measured on 64^3: S 10.8 us with 1024
// against 11.7 us with 256; A_gamma 31.5 us with 256 against 33.5 us with 1024).
constexpr int kPcgMaxThreads = 256 * 2048;
constexpr int kPcgBlocks = kPcgMaxThreads / 256;  // most blocks of any inner-CG grid
constexpr int kPcgThreads = 1024;  // block size of the FP32 inner-CG kernels

// Device-resident state of one inner (pipelined) Jacobi-CG solve.  `count` is
// reset by every init kernel; `total` sums the iterations of all inner solves
// since the host last cleared it (once per outer solve).
struct PcgState {
  double gamma[2], alpha[2], gamma0, tol2;
  int count, maxit, done, total;
};

// Vectors of one inner CG solve (x is the solution), FP64 or FP32.
template <typename T>
struct PcgWorkT {
  T *x, *r, *z, *s, *p, *w0, *w1;
  const T* dinv;
};
using PcgWork = PcgWorkT<double>;
using PcgWork32 = PcgWorkT<float>;

// Compressed sparse row matrix on the device.
struct Csr {
  int64_t rows = 0, nnz = 0;
  DBuf<int> rowptr, col;
  DBuf<double> val;
};

// SELL-64 copy of a CSR matrix (64-row slices, column-major inside a slice).
struct Sell {
  int64_t rows = 0, nslices = 0, nnz = 0;
  int max_len = 0;       // longest slice (entries per row after padding)
  int fixed_len = 0;     // every slice padded to max_len (short rows only), else 0
  DBuf<int> slice_ptr, slice_len, col, src;
  DBuf<double> val;
  DBuf<double> val_cs;   // column-scaled copy A D^{-1} (inner CG matrices only)
  DBuf<float> val32;     // FP32 rounding of val (mixed-precision inner solves)
  DBuf<float> val32_cs;  // FP32 rounding of val_cs (mixed-precision pipelined inner solves)
};
// SELL copies of `count` (<= 3) CSR matrices, with one host synchronisation for all of
// their padded sizes (uses tmp.i64[2m], tmp.i64[2m+1] for matrix m and slots 0..count-1).
void build_sells(hipStream_t s, Scratch& tmp, const Csr* const* A, Sell* const* S, int count);
// A.val from the SELL values (A shares S's pattern)
void sell_to_csr(hipStream_t s, const Sell& S, Csr& A);
// diag[r] (the CSR position of row r's diagonal) becomes its SELL slot, for the first ndiag rows
// (the rows that have a diagonal entry: K's flux rows; every row of A_gamma and S)
void sell_diag_slots(hipStream_t s, int64_t ndiag, const Csr& A, const Sell& S, int* diag);

// ---- launchers (one translation unit each; all take the handle's stream) ----

// mesh / geometry
void launch_face_geometry(hipStream_t s, int nf, const double* xyz, const int* fptr, const int* fvtx, double* area,
                          double* normal, double* cen, double* diam, double* e1, double* e2);
void launch_cell_geometry(hipStream_t s, int nc, const double* xyz, const int* fptr, const int* fvtx,
                          const int* cptr, const int* cface, const int8_t* csign, double* vol, double* cen,
                          double* diam, double* xref);
void launch_check_mesh(hipStream_t s, int nv, int nf, int nc, const int* fptr, const int* fvtx, const int* cptr,
                       const int* cface, const int8_t* csign, int* face_cnt, int* face_cell, int* face_lidx,
                       int* inc_cell, int* err);
// out[0] = error bits of the two offset arrays, out[1] = max faces per cell (out zeroed first)
void launch_check_offsets(hipStream_t s, int64_t nf, const int* fptr, int64_t nc, const int* cptr, int* out);
void launch_check_faces(hipStream_t s, int nf, const int* face_cnt, const double* area, int* is_bnd, int* err);
void launch_check_cells(hipStream_t s, int nc, const double* vol, int* err);
void launch_tets(hipStream_t s, int nc, const int* fptr, const int* cptr, const int* cface, const int* cell_tet_ptr,
                 int* tet_inc, int* tet_a);
void launch_tet_counts(hipStream_t s, int nc, const int* fptr, const int* cptr, const int* cface, int* cnt);
void launch_bnd_tri_counts(hipStream_t s, int nb, const int* bface, const int* fptr, int* cnt);
void launch_qp_cell(hipStream_t s, int64_t ntet, int npts, const double* ref, const int* tet_inc, const int* tet_a,
                    const int* inc_cell, const double* xyz, const int* fptr, const int* fvtx, const int* cface,
                    const double* xref, double* qp);
void launch_qp_face(hipStream_t s, int nb, int npts, int64_t total, const double* ref, const int* bface,
                    const int* btri_ptr, const double* xyz, const int* fptr, const int* fvtx, double* qp);
// prescribed boundary fluxes (1/|f|) int_f u.n_f of the lowest-order element, into xB[f]
void launch_bnd_flux(hipStream_t s, int nb, int npts, int64_t total, const double* refw, const int* bface,
                     const int* btri_ptr, const double* xyz, const int* fptr, const int* fvtx, const double* fnormal,
                     const double* farea, const double* uq, double* xB);
void launch_load_tets(hipStream_t s, int64_t ntet, int npts, const double* refw, const int* tet_inc,
                      const int* tet_a, const int* inc_cell, const double* xyz, const int* fptr, const int* fvtx,
                      const int* cface, const int8_t* csign, const double* xref, const double* fq,
                      double* tet_sum);
void launch_load_cells(hipStream_t s, int nc, const int* cell_tet_ptr, const double* tet_sum, double* rhs_p);
void launch_bnd_rhs(hipStream_t s, int nb, int npts, const double* refw, const int* bface, const int* btri_ptr,
                    const double* xyz, const int* fptr, const int* fvtx, const int* face_cell, const double* pq,
                    double* rhs_u);

// lowest-order local matrices
void launch_lo_local(hipStream_t s, int64_t ninc, const int* inc_cell, const int* cptr, const int* cface,
                     const int8_t* csign, const double* farea, const double* fnormal, const double* fcen,
                     const double* cvol, const double* ccen, const int64_t* lmat_ptr, double* M1,
                     const int64_t* lb_ptr, double* Bdiv1);

// the paper's order-k element (k = 1, 2, 3)
struct PaperSizes {
  int nfd, npd, nint, n3, nsm, nfm, nq;  // face DOFs, pressure DOFs, interior DOFs, 3 dim P_k,
                                         // cell moments, face integrals per incidence, face rule points
};
PaperSizes paper_sizes(int k);
struct PaperLocalArgs {
  hipStream_t s;
  int nf, nc;
  int64_t ninc;
  const int *inc_cell, *cptr, *cface, *fptr, *fvtx, *ldof_ptr;
  const int8_t* csign;
  const double *xyz, *farea, *fnormal, *fcen, *fdiam, *fe1, *fe2, *cvol, *ccen, *cdiam;
  const double* tri_ref;  // (xi, eta, w) per point of the face rule with k+1 points per direction
  double *FP, *FM, *Tf, *cmom;
  double *Dg, *Pg, *Xg, *Cg;  // per-cell scratch (sum of ndof) x {3 dim P_k, 3 dim P_k, 3 dim P_k, npd}
  const int64_t *lmat_ptr, *lb_ptr;
  double *M1, *Bdiv1;
};
void launch_paper_local(int k, const PaperLocalArgs& a);
struct PaperLoadArgs {
  hipStream_t s;
  int nc, nb, npts_cell, npts_face;
  int64_t ntet;
  const double *ref_cell, *w_cell, *ref_face, *w_face;
  const int *tet_inc, *tet_a, *inc_cell, *fptr, *fvtx, *cface, *cell_tet_ptr, *bface, *btri_ptr, *face_cell;
  const int8_t* csign;
  const double *xyz, *xref, *ccen, *cdiam, *cvol, *cmom, *fcen, *fdiam, *fe1, *fe2, *Tf;
  const double *fq, *pq;
  double *tet_sum, *rhs_p, *rhs_u;
  // flux boundary data: u at the boundary-face points (structure of arrays, nq_face_total points)
  // gives the prescribed face moments xB (indexed by global flux DOF); uq == nullptr skips them
  const double *uq, *fnormal, *farea;
  int64_t nq_face_total;
  double* xB;
};
void launch_paper_loads(int k, const PaperLoadArgs& a);

// generic assembly (element described by nfd face DOFs per face, nint interior and npd pressure DOFs per cell)
struct DofLayout {
  int nf, nc, nfd, nint, npd;
  int64_t Nu, Np;
};
void launch_ldof_sort(hipStream_t s, DofLayout L, const int* cptr, const int* cface, const int* ldof_ptr,
                      int* sorted_gid, int* sorted_l);
void launch_rowlen(hipStream_t s, DofLayout L, const int* cptr, const int* ldof_ptr, const int* sorted_gid,
                   const int* face_cell, const int* face_lidx, const int* cface, int* lenK, int* lenA, int* lenS);
void launch_fill_patterns(hipStream_t s, DofLayout L, const int* cptr, const int* ldof_ptr, const int* sorted_gid,
                          const int* face_cell, const int* face_lidx, const int* cface, const int* Kptr, int* Kcol,
                          int* Kdiag, const int* Aptr, int* Acol, int* Adiag, const int* Sptr, int* Scol,
                          int* Sdiag);
void launch_cell_sizes(hipStream_t s, DofLayout L, const int* cptr, int64_t* ndof, int64_t* nmat, int64_t* nb);
void launch_coef_grad(hipStream_t s, DofLayout L, const int* cptr, const int* cface, const int8_t* csign,
                      const int64_t* lmat_ptr, const double* M1, const double* nu, const double* u,
                      const double* lam, double* g);
void launch_values(hipStream_t s, DofLayout L, const int* cptr, const int* cface, const int8_t* csign,
                   const int* ldof_ptr, const int* sorted_gid, const int* sorted_l, const int* face_cell,
                   const int* face_lidx, const int64_t* lmat_ptr, const double* M1, const int64_t* lb_ptr,
                   const double* Bdiv1, const double* nu, double inv_gamma, const int* bnd, const int* Kslice,
                   double* Kval, const int* Aslice, double* Aval);
// flux boundary data: out = b - K xB on the free rows, xB on the prescribed ones
void launch_flux_rhs(hipStream_t s, DofLayout L, const int* cptr, const int* cface, const int8_t* csign,
                     const int* face_cell, const int* face_lidx, const int64_t* lmat_ptr, const double* M1,
                     const int64_t* lb_ptr, const double* Bdiv1, const double* nu, const int* bnd, const double* xB,
                     const double* b, double* out);
// the discrete constant pressure and the mean weights (cmom == nullptr: one pressure DOF per cell)
void launch_pressure_constants(hipStream_t s, DofLayout L, int nsm, const double* cmom, const double* cvol,
                               double* np, double* w);
// out = x - v (dot * inv_vv), dot a device scalar (out may be x)
void launch_project(hipStream_t s, int64_t n, const double* x, const double* v, const double* dot, double inv_vv,
                    double* out);
void launch_diag_inv(hipStream_t s, int64_t n, const int* diagpos, const double* val, double* d, double* dinv);
void launch_schur_values(hipStream_t s, DofLayout L, const int* cptr, const int* cface, const int8_t* csign,
                         const int* ldof_ptr, const int* face_cell, const int* face_lidx, const int64_t* lb_ptr,
                         const double* Bdiv1, const double* dM, const int* bnd, const int* Sptr, const int* Scol,
                         const int* Sslice, double* Sval);
void launch_rhs_from_moments(hipStream_t s, int64_t Nu, int64_t Np, double* rhs);

// sparse/Krylov
void launch_spmv(hipStream_t s, const Sell& A, const double* x, double* y);
void launch_residual(hipStream_t s, const Sell& A, const double* x, const double* b, double* r, double* partials,
                     double* out);
// The reductions below write their results to out (device) and, when hout is given (the device
// address of pinned host memory), a copy there for the host.
void launch_dots(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* w, double* partials,
                 double* out, double* hout = nullptr);
void launch_update_dots(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* h, double* w,
                        double* partials, double* out, double* hout = nullptr);
// First Gram-Schmidt pass with the previous step's second pass folded in: V[k-1] = (V[k-1] -
// V[0..k-1) hp) / sqrt(hp[k-1] - |hp[0..k-1)|^2) in place, then out[0..k) = V^T w (k >= 2)
void launch_dots_fix(hipStream_t s, int64_t n, int k, double* V, int64_t ldv, const double* hp, const double* w,
                     double* partials, double* out, double* hout = nullptr);
void launch_scale_to(hipStream_t s, int64_t n, const double* w, const double* norm2, double* dst);
void launch_scale_by(hipStream_t s, int64_t n, const double* x, const double* d, double c, double* y);
void launch_combine(hipStream_t s, int64_t n, int k, const double* Z, int64_t ldz, const double* y, double* x);
void launch_copy(hipStream_t s, int64_t n, const double* x, double* y);
void launch_fill(hipStream_t s, int64_t n, double v, double* y);
void launch_sum(hipStream_t s, int64_t n, const double* x, double* partials, double* out);
// inner CG: part needs 4 * kPcgBlocks doubles; launch_col_scale fills A.val_cs = A D^{-1}
void launch_col_scale(hipStream_t s, Sell& A, const double* dinv);
void launch_pcg_init(hipStream_t s, const Sell& A, const PcgWork& w, const double* b, PcgState* st, double tol,
                     int maxit, double* part);
void launch_pcg_iter(hipStream_t s, int i, const Sell& A, const PcgWork& w, PcgState* st, double* part);
// FP32 inner CG: classical Jacobi-PCG on FP32 copies of the matrix values and of D^{-1}, FP32 vectors,
// dot products accumulated in FP64 (launch_col_scale32 makes the FP32 copies)
void launch_col_scale32(hipStream_t s, Sell& A, const double* dinv, float* dinv32);
void launch_pcg_init32(hipStream_t s, const Sell& A, const PcgWork32& w, const double* b, PcgState* st, double tol,
                       int maxit, double* part);
void launch_pcg_iter32(hipStream_t s, int i, const Sell& A, const PcgWork32& w, PcgState* st, double* part);
// the classical iteration in FP64 (unscaled values; two kernels per iteration)
void launch_pcg_init64c(hipStream_t s, const Sell& A, const PcgWork& w, const double* b, PcgState* st, double tol,
                        double* part);
void launch_pcg_iter64c(hipStream_t s, int i, const Sell& A, const PcgWork& w, PcgState* st, double* part);
// the pipelined iteration in FP32 (vectors and column-scaled values; dot products in FP64)
void launch_pcg_init32p(hipStream_t s, const Sell& A, const PcgWork32& w, const double* b, PcgState* st, double tol,
                        int maxit, double* part);
void launch_pcg_iter32p(hipStream_t s, int i, const Sell& A, const PcgWork32& w, PcgState* st, double* part);
void launch_to_f64(hipStream_t s, int64_t n, const float* x, double* y);
// A diagonal scaling y = d x of n FP64 entries that a launch performs beside its own work.
struct ScaleJob {
  int64_t n = 0;
  const double* x = nullptr;
  const double* d = nullptr;
  double* y = nullptr;
};
// Chebyshev-Jacobi inner solve: m products, interval [c hi, hi] with 1/hi at inv_hi (device), on the
// column-scaled values (val_cs, FP32: val32_cs) and w.dinv; x (FP64: w.x; FP32: w.x rounded); the
// iterates alternate in w.p and w.s, and FP32 keeps b rounded in w.r; adds m to st->total.  The
// first product also performs `side` (Block-Schur's diag(M)^{-1} on the flux part), saving a launch.
template <typename T>
void launch_cheb(hipStream_t s, const Sell& A, const PcgWorkT<T>& w, const double* b, const double* inv_hi,
                 double c, int m, PcgState* st, const ScaleJob& side = ScaleJob{});
// mean kernel time (ms) of reps middle-form Chebyshev products, each timed by its own start and stop
// events (after a degree-2 solve that sets up the iterates; synchronises)
template <typename T>
double time_cheb_products(hipStream_t s, const Sell& A, const PcgWorkT<T>& w, const double* b,
                          const double* inv_hi, double c, int reps, PcgState* st);
// inv_hi[0] = 1 / (Gershgorin bound of D^{-1}A); part holds up to 1024 doubles
void launch_gershgorin(hipStream_t s, const Sell& A, const double* dinv, double* part, double* inv_hi);

// ---- edge-patch additive Schwarz for the regularised block (Block-Reg) ----
// Face system: the lowest order uses A_gamma itself; the order-k element condenses the interior
// DOFs of each cell (A_gamma is a sum of cell matrices and an interior DOF belongs to one cell),
// leaving F = A_ff - A_fi A_ii^{-1} A_if on the face DOFs.  The preconditioner of the CG on F is
// P = sum_e R_e^T F_e^{-1} R_e over the mesh edges e, R_e restricting to the DOFs of the faces
// that contain e (the patches that hold the local divergence-free fields).
// Order-k face systems couple whole faces: the entries between two faces form a dense nfd x nfd
// block (nfd face DOFs each).  Block rows by face, one column index per block:
//   bcol[bptr[f] + j] = face of block j of face f (ascending),
//   val[((bptr[f] + j) nfd + i) nfd + c] = entry (f nfd + i, bcol nfd + c),
// so a DOF row reads its nfd entries of a block contiguously, with no padding and one 4-byte index
// per nfd^2 entries (against one per entry, and padded slices, in SELL-64).
struct FaceBlocks {
  int nfd = 0;
  int64_t nf = 0, nblk = 0;
  DBuf<int> bptr, bcol;
  DBuf<double> val;
  DBuf<float> val32;
};
// the face-DOF counts with a block kernel (the paper's k = 1, 2, 3)
inline bool face_blocks_supported(int nfd) { return nfd == 3 || nfd == 6 || nfd == 10; }

struct Schwarz {
  bool built = false;  // pattern of the current discretisation
  bool blocked = false;  // order k: F and P held as face blocks (Fb, Pb) instead of SELL (Fs, Ps)
  bool ready = false;  // values for the current coefficient, gamma and boundary data
  bool ready32 = false;
  double gamma = 0.0;
  int64_t ne = 0, nF = 0;
  int max_patch = 0;                 // largest number of faces around an edge
  DBuf<int> edge_ptr, edge_face;     // faces of each edge, ascending
  DBuf<int> face_edge;               // edge of each face-loop incidence (face_ptr order)
  DBuf<int64_t> einv_ptr;            // offsets of the patch inverses
  DBuf<double> einv;
  Csr Fc;                            // face system (order k only; the lowest order uses A)
  Sell Fs;
  Csr Pc;                            // the Schwarz operator on the face DOFs
  Sell Ps;
  FaceBlocks Fb, Pb;                 // F and P as face blocks (blocked)
  DBuf<int64_t> w_ptr;               // order k: per cell W = A_fi A_ii^{-1} (face DOFs x nint)
  DBuf<double> W, Aiinv;             // and A_ii^{-1} (nint x nint)
  DBuf<double> ucell;                // order k: W v_i per cell face DOF (inner-solve right-hand side)
  int fn_max = 0;                    // order k: most face DOFs of a cell
  DBuf<int64_t> sp_ptr;              // order k: per cell the condensed matrix A_ff - W A_if
  DBuf<double> Sp;                   // (face DOFs^2, row-major), when its set-up fits in LDS
};
struct SchwarzMesh {
  int nv, nf, nc;
  const int *fptr, *fvtx, *cptr, *cface, *face_cell, *face_lidx, *ldof_ptr, *sorted_gid, *sorted_l;
  const int8_t* csign;
};
// edges and patterns (coefficient-free; synchronises)
void schwarz_build(hipStream_t s, Scratch& tmp, const SchwarzMesh& m, const DofLayout& L, const Csr& A,
                   Schwarz& X);
// values for nu and gamma (A / As: the assembled A_gamma, used directly at the lowest order)
void schwarz_values(hipStream_t s, const SchwarzMesh& m, const DofLayout& L, const int64_t* lmat_ptr,
                    const double* M1, const int64_t* lb_ptr, const double* Bdiv1, const double* nu,
                    double inv_gamma, const int* bnd, const Csr& A, const Sell& As, Schwarz& X);
// FP32 roundings of P and (order k) of the face system, for mixed-precision inner solves
void schwarz_round32(hipStream_t s, const DofLayout& L, Schwarz& X);
// CSR values of the face system (face) or of P into C.val (C: X.Fc or X.Pc) from whichever copy
// the solver holds (SELL or face blocks); the lowest order's face system is A_gamma itself
void schwarz_export(hipStream_t s, const Schwarz& X, bool face, Csr& C);
// the face system's SELL (As at the lowest order) and CSR pattern
inline const Sell& schwarz_face_sell(const Schwarz& X, const Sell& As, const DofLayout& L) {
  return L.nint > 0 ? X.Fs : As;
}
// r0 = v_f - sum_P sigma W_P v_{i,P} (order k) or v_f (lowest order), in T
template <typename T>
void launch_schwarz_rhs(hipStream_t s, const SchwarzMesh& m, const DofLayout& L, const Schwarz& X, const int* bnd,
                        const double* v, T* r0);
// z_i = A_ii^{-1} v_i - W^T sigma x_f on the interior DOFs (order k only)
void launch_schwarz_back(hipStream_t s, const SchwarzMesh& m, const DofLayout& L, const Schwarz& X,
                         const double* v, double* z);
// CG on the face system F with the Schwarz operator P, two kernels per iteration (the products
// F p and P r carried by recurrences, one gathered vector per kernel):
//   [product] beta, stop test; p = z + beta p; q = F z + beta q; partials p.q
//   [update]  alpha; x += alpha p; r -= alpha q; z -= alpha P q; partials r.z
// Work layout: x, r, z, p, w0 = q.  T = double, or float with FP64 dot products.
// F: the face system's SELL (schwarz_face_sell), used unless X.blocked.  early_exit: each kernel reads
// the stop flag before anything else and returns at once when it is set (for iterations enqueued in
// chunks between polls, where launches past convergence would otherwise load their first rows).
template <typename T>
void launch_scg_init(hipStream_t s, const Schwarz& X, const PcgWorkT<T>& w, PcgState* st, double tol, double* part);
template <typename T>
void launch_scg_iter(hipStream_t s, int i, const Sell& F, const Schwarz& X, const PcgWorkT<T>& w, PcgState* st,
                     double* part, bool early_exit = false);

// host utilities
void gauss_jacobi01(int n, int alpha, double* t, double* w);  // int_0^1 (1-t)^alpha g(t) dt
void tet_reference_rule(int n, std::vector<double>& pts, std::vector<double>& w);
void tri_reference_rule(int n, std::vector<double>& pts, std::vector<double>& w);
// Exclusive prefix sums with the total appended (ptr has n+1 entries).
//  - scan_*_async enqueue the scan and a copy of the total into the pinned slot
//    tmp.tot[slot] (0 <= slot < 8) without waiting: several scans then share one host
//    synchronisation.  Call scan_reserve(tmp, n) first with the largest n of the group,
//    so that no scan of the group reallocates the shared hipcub storage.
//  - scan_i32_async goes through the 64-bit buffer p64 (n + 1 entries); a total beyond
//    2^31 - 1 is the caller's to reject once it has synchronised.
//  - scan_i32 / scan_i64 synchronise and return the total (scan_i32 uses tmp.i64[3]).
void scan_reserve(Scratch& tmp, int64_t n);
void scan_i64_async(hipStream_t s, Scratch& tmp, const int64_t* len, int64_t n, int64_t* ptr, int slot);
void scan_i32_async(hipStream_t s, Scratch& tmp, const int* len, int64_t n, int* ptr, DBuf<int64_t>& p64, int slot);
int64_t scan_i32(hipStream_t s, Scratch& tmp, const int* len, int64_t n, int* ptr);
int64_t scan_i64(hipStream_t s, Scratch& tmp, const int64_t* len, int64_t n, int64_t* ptr);
void launch_compact_flags(hipStream_t s, int64_t n, const int* flag, const int* pos, int* out);

}  // namespace vem
