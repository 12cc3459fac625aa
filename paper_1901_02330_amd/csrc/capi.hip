// C ABI entry points, set-up orchestration and the flexible GMRES driver.
//
// Everything numerical runs in the kernels of mesh.hip, element_lo.hip,
// assemble.hip and krylov.hip; this file owns device memory, enqueues those
// kernels on the handle's stream and runs the host side of FGMRES (Givens
// rotations on the (m+1) x m Hessenberg matrix, one 8-byte-class read-back per
// Arnoldi step).
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <new>

#include "vem_internal.h"

using namespace vem;

// A captured run of kGraphIters inner-CG iterations (parities fixed by position), replayed on the
// handle's stream; `key` records the buffers it references so that it is re-captured when they move.
constexpr int kGraphIters = 8;
// inner solves capped at this many iterations run without host polling
constexpr int kBlindInner = 64;
// doubles per Arnoldi step read back by the host: h, its correction and ||w||^2
constexpr int kColSlot = 2 * kMaxDots + 1;
struct InnerGraph {
  hipGraphExec_t exec = nullptr;
  const void* key[8] = {};
  InnerGraph() = default;
  InnerGraph(const InnerGraph&) = delete;
  InnerGraph& operator=(const InnerGraph&) = delete;
  ~InnerGraph() { reset(); }
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
  }
};

// Device memory behind vem_set_rhs_noalloc, for callers that cannot allocate: the per-tetrahedron
// load sums of one right-hand side build (ntet doubles at the lowest order, ntet * dim P_{k-1} for
// the order-k element).  Each device holds its own copy until the process ends; host code never
// passes this name to a kernel (on the host it is only a stand-in for the symbol), it uses the
// address that hipGetSymbolAddress returned on that device (noalloc_scratch below).
constexpr int64_t kNoAllocDoubles = int64_t(4) << 20;  // 32 MiB
static __device__ __align__(256) double scratch[kNoAllocDoubles];

struct vem_ctx {
  ~vem_ctx() {
    for (InnerGraph* g : {&gS, &gA, &gS32, &gA32}) g->reset();
    if (cap) (void)hipStreamDestroy(cap);
    for (hipEvent_t& e : step_done)
      if (e) (void)hipEventDestroy(e);
  }
  InnerGraph gS, gA, gS32, gA32;
  hipStream_t cap = nullptr;  // private stream used only to capture graphs
  hipStream_t stream = nullptr;
  int device = 0;
  double* noalloc = nullptr;  // this device's copy of `scratch` (vem_set_rhs_noalloc)
  std::string last_error;

  // mesh (device copies) and host copies of the offsets
  bool has_mesh = false;
  int nv = 0, nf = 0, nc = 0;
  int64_t nfv = 0, ncf = 0;
  std::vector<int> h_fptr, h_cptr;
  int max_cell_faces = 0;
  DBuf<double> xyz;
  DBuf<int> fptr, fvtx, cptr, cface, inc_cell;
  DBuf<int8_t> csign;
  DBuf<int> face_cnt, face_cell, face_lidx, is_bnd;

  // geometry
  DBuf<double> f_area, f_normal, f_cen, f_diam, f_e1, f_e2;
  DBuf<double> c_vol, c_cen, c_diam, c_xref;
  double h = 0.0, gamma_default = 0.0;

  // quadrature
  int load_n = 3;
  int64_t ntet = 0, nbf = 0, nbtri = 0;
  DBuf<int> cell_tet_ptr, tet_inc, tet_a, bface, btri_ptr;
  DBuf<double> qref_cell, qw_cell, qref_face, qw_face;
  int qrule_n = 0;   // the n whose reference rules are on the device (0: none)
  DBuf<double> pk_trip;  // triangle rule (points, weight) of the order-k face integrals
  int pk_trip_nq = 0;
  int npts_cell = 0, npts_face = 0;

  // discretisation
  bool has_disc = false;
  int family = VEM_LO, korder = 0;
  DofLayout L{};
  DBuf<int> ldof_ptr, sorted_gid, sorted_l;
  DBuf<int64_t> lmat_ptr, lb_ptr;
  DBuf<double> M1, Bdiv1;
  DBuf<double> nu, rhs;
  // paper's element: face transfer matrices T_f = |f| H_f^{-1}, cell moments of the scaled monomials
  DBuf<double> pk_Tf, pk_cmom;

  // matrices
  Csr K, A, S;
  Sell Ks, As, Ss;
  Schwarz sz;  // Block-Reg's edge-patch Schwarz preconditioner (built on first use)
  DBuf<int> Kdiag, Adiag, Sdiag;
  DBuf<double> dM, dMinv, dAinv, dSinv;
  DBuf<double> cheb;  // 1 / Gershgorin bound of D^{-1}S [0] and of D^{-1}A_gamma [1] (Chebyshev inner form)
  DBuf<float> dAinv32, dSinv32;
  double gamma_A = 0.0;
  // the coefficient-dependent values are built on first use after vem_discretize /
  // vem_set_coefficient / vem_set_boundary, and only those a call needs: K and diag(M) (k_ready),
  // S (s_ready, Block-Schur), A_gamma at gamma_A (a_ready, Block-Reg), FP32 shadows (s32, a32)
  bool k_ready = false, s_ready = false, a_ready = false, s32_ready = false, a32_ready = false;
  int expect_S = 0, expect_A = 0;  // last inner-CG iteration counts (chunk sizing)

  // solver workspace
  int64_t ws_N = 0;
  int ws_m = 0;
  DBuf<double> Vb, Zb, xw;
  DBuf<double> pr, pz, ps, pp, pw0, pw1, pxw;
  DBuf<float> px32;
  DBuf<double> partials, pcgpart, scal;
  DBuf<PcgState> pcg;
  HBuf<double> hbuf;
  // Arnoldi scalars of every step of a restart cycle, one slot per step (pinned), and
  // the events that mark each step's copy (steps alternate between the two)
  HBuf<double> hcol;
  double* hcol_dev = nullptr;  // the device address of hcol (pinned host memory the kernels write)
  Scratch tmp;  // temporaries of the set-up calls
  // boundary data: VEM_BC_PRESSURE (natural, in g) or VEM_BC_FLUX (prescribed boundary fluxes xB and
  // a zero-mean pressure; n_p is the discrete constant pressure, pw the mean weights)
  int bc = VEM_BC_PRESSURE;
  DBuf<double> xB, rhs_flux, n_p, pw, ptmp;
  double np_nn = 1.0, np_wn = 1.0;
  hipEvent_t step_done[2] = {nullptr, nullptr};
  HBuf<PcgState> hpcg;
  // multi-field batch: nb_nu coefficient fields (nu, cell-major per field) and nb_rhs right-hand sides
  int64_t nb_nu = 0, nb_rhs = 0;
  DBuf<double> nu_batch, rhs_batch;
};

namespace {

// ---------------------------------------------------------------------------------------
// host utilities: Gauss-Jacobi rules (bracketing + bisection on the three-term recurrence)
void jacobi_eval(int n, double a, double b, double x, double& p) {
  if (n == 0) {
    p = 1.0;
    return;
  }
  double p0 = 1.0, p1 = 0.5 * (a - b + (a + b + 2.0) * x);
  for (int k = 2; k <= n; ++k) {
    double c = 2.0 * k + a + b;
    double a1 = 2.0 * k * (k + a + b) * (c - 2.0);
    double a2 = (c - 1.0) * (a * a - b * b);
    double a3 = (c - 2.0) * (c - 1.0) * c;
    double a4 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * c;
    double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
}

}  // namespace

namespace vem {

namespace {
// Nodes and weights of int_0^1 (1 - t)^alpha g(t) dt, exact for degree 2n - 1.
void gauss_jacobi01_compute(int n, int alpha, double* t, double* w);
}  // namespace

// The rules depend on (n, alpha) only; each is computed once per process (the root search
// costs a few hundred microseconds) and copied out of a table afterwards.
void gauss_jacobi01(int n, int alpha, double* t, double* w) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, std::vector<double>> memo;  // n nodes, then n weights
  std::vector<double> tw;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = memo.find({n, alpha});
    if (it != memo.end()) tw = it->second;
  }
  if (tw.empty()) {
    tw.resize(2 * (size_t)n);
    gauss_jacobi01_compute(n, alpha, tw.data(), tw.data() + n);
    std::lock_guard<std::mutex> lock(mu);
    memo.emplace(std::make_pair(n, alpha), tw);
  }
  std::copy(tw.begin(), tw.begin() + n, t);
  std::copy(tw.begin() + n, tw.end(), w);
}

namespace {
void gauss_jacobi01_compute(int n, int alpha, double* t, double* w) {
  const double a = alpha, b = 0.0;
  std::vector<double> roots;
  const int grid = 20000;
  double xl = -1.0, pl;
  jacobi_eval(n, a, b, xl, pl);
  for (int i = 1; i <= grid && (int)roots.size() < n; ++i) {
    double xr = -1.0 + 2.0 * i / grid, pr;
    jacobi_eval(n, a, b, xr, pr);
    if (pl == 0.0) {
      roots.push_back(xl);
    } else if ((pl < 0) != (pr < 0) && pr != 0.0) {
      double lo = xl, hi = xr, plo = pl;
      for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi), pm;
        if (mid == lo || mid == hi) break;
        jacobi_eval(n, a, b, mid, pm);
        if ((pm < 0) == (plo < 0)) {
          lo = mid;
          plo = pm;
        } else {
          hi = mid;
        }
      }
      roots.push_back(0.5 * (lo + hi));
    }
    xl = xr;
    pl = pr;
  }
  VEM_REQUIRE((int)roots.size() == n, VEM_EINVAL, "Gauss-Jacobi root search failed");
  // w_i = 2^{a+b+1} G(n+a+1) G(n+b+1) / (G(n+a+b+1) n!) / ((1-x^2) P_n'(x)^2),
  // P_n^{(a,b)}' = (n+a+b+1)/2 P_{n-1}^{(a+1,b+1)}
  double lc = (a + b + 1.0) * std::log(2.0) + std::lgamma(n + a + 1.0) + std::lgamma(n + b + 1.0) -
              std::lgamma(n + a + b + 1.0) - std::lgamma(n + 1.0);
  for (int i = 0; i < n; ++i) {
    double x = roots[i], q;
    jacobi_eval(n - 1, a + 1.0, b + 1.0, x, q);
    double dp = 0.5 * (n + a + b + 1.0) * q;
    double wi = std::exp(lc) / ((1.0 - x * x) * dp * dp);
    t[i] = 0.5 * (1.0 + x);
    w[i] = wi / std::pow(2.0, a + 1.0);
  }
}
}  // namespace

void tet_reference_rule(int n, std::vector<double>& pts, std::vector<double>& w) {
  std::vector<double> a(n), wa(n), b(n), wb(n), c(n), wc(n);
  gauss_jacobi01(n, 2, a.data(), wa.data());
  gauss_jacobi01(n, 1, b.data(), wb.data());
  gauss_jacobi01(n, 0, c.data(), wc.data());
  pts.clear();
  w.clear();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        pts.push_back(a[i]);
        pts.push_back(b[j] * (1.0 - a[i]));
        pts.push_back(c[k] * (1.0 - a[i]) * (1.0 - b[j]));
        w.push_back(wa[i] * wb[j] * wc[k]);
      }
}

void tri_reference_rule(int n, std::vector<double>& pts, std::vector<double>& w) {
  std::vector<double> a(n), wa(n), b(n), wb(n);
  gauss_jacobi01(n, 1, a.data(), wa.data());
  gauss_jacobi01(n, 0, b.data(), wb.data());
  pts.clear();
  w.clear();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      pts.push_back(a[i]);
      pts.push_back(b[j] * (1.0 - a[i]));
      w.push_back(wa[i] * wb[j]);
    }
}

}  // namespace vem

// ---------------------------------------------------------------------------------------
// scans and small helper kernels
namespace {

struct ToI64 {
  __host__ __device__ int64_t operator()(int v) const { return (int64_t)v; }
};

__global__ void k_narrow(int64_t n, const int64_t* __restrict__ in, int* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (int)in[i];
}

// ptr[n] = ptr[n-1] + len[n-1] (0 when n = 0): the total after an exclusive scan of n entries
template <typename It>
__global__ void k_scan_tail(int64_t n, It len, int64_t* __restrict__ ptr) {
  ptr[n] = n > 0 ? ptr[n - 1] + (int64_t)len[n - 1] : 0;
}

__global__ void k_set_last_zero_i32(int* p) { *p = 0; }
__global__ void k_set_last_zero_i64(int64_t* p) { *p = 0; }

__global__ void k_compact(int64_t n, const int* __restrict__ flag, const int* __restrict__ pos, int* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) out[pos[i]] = (int)i;
}

__global__ void k_fill_i32(int64_t n, int v, int* p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline int grid_of(int64_t n) { return (int)((n + 255) / 256); }

void fill_i32(hipStream_t s, int64_t n, int v, int* p) {
  if (n > 0) k_fill_i32<<<grid_of(n), 256, 0, s>>>(n, v, p);
}

}  // namespace

namespace vem {

void scan_reserve(Scratch& tmp, int64_t n) {
  size_t b64 = 0, b32 = 0;
  const int64_t* l64 = nullptr;
  int64_t* p64 = nullptr;
  hipcub::TransformInputIterator<int64_t, ToI64, const int*> it(nullptr, ToI64());
  VEM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, b64, l64, p64, (int)n, (hipStream_t)0));
  VEM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, b32, it, p64, (int)n, (hipStream_t)0));
  const size_t bytes = b64 > b32 ? b64 : b32;
  tmp.cub.reserve(bytes > 0 ? bytes : 1);
  tmp.tot.alloc(8);
}

void scan_i64_async(hipStream_t s, Scratch& tmp, const int64_t* len, int64_t n, int64_t* ptr, int slot) {
  size_t bytes = 0;
  VEM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, len, ptr, (int)n, s));
  VEM_REQUIRE(bytes <= tmp.cub.n && tmp.tot.p && slot >= 0 && slot < 8, VEM_EINVAL, "scan scratch not reserved");
  VEM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.cub.p, bytes, len, ptr, (int)n, s));
  k_scan_tail<<<1, 1, 0, s>>>(n, len, ptr);  // ptr[n] = ptr[n-1] + len[n-1]
  VEM_HIP(hipGetLastError());
  VEM_HIP(hipMemcpyAsync(tmp.tot.p + slot, ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
}

void scan_i32_async(hipStream_t s, Scratch& tmp, const int* len, int64_t n, int* ptr, DBuf<int64_t>& p64,
                    int slot) {
  p64.reserve(n + 1);
  hipcub::TransformInputIterator<int64_t, ToI64, const int*> it(len, ToI64());
  size_t bytes = 0;
  VEM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, it, p64.p, (int)n, s));
  VEM_REQUIRE(bytes <= tmp.cub.n && tmp.tot.p && slot >= 0 && slot < 8, VEM_EINVAL, "scan scratch not reserved");
  VEM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.cub.p, bytes, it, p64.p, (int)n, s));
  k_scan_tail<<<1, 1, 0, s>>>(n, it, p64.p);
  VEM_HIP(hipGetLastError());
  VEM_HIP(hipMemcpyAsync(tmp.tot.p + slot, p64.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  k_narrow<<<grid_of(n + 1), 256, 0, s>>>(n + 1, p64.p, ptr);  // a total past 2^31-1 is rejected by the caller
  VEM_HIP(hipGetLastError());
}

int64_t scan_i64(hipStream_t s, Scratch& tmp, const int64_t* len, int64_t n, int64_t* ptr) {
  scan_reserve(tmp, n);
  scan_i64_async(s, tmp, len, n, ptr, 0);
  VEM_HIP(hipStreamSynchronize(s));
  return tmp.tot.p[0];
}

int64_t scan_i32(hipStream_t s, Scratch& tmp, const int* len, int64_t n, int* ptr) {
  scan_reserve(tmp, n);
  scan_i32_async(s, tmp, len, n, ptr, tmp.i64[3], 0);
  VEM_HIP(hipStreamSynchronize(s));
  const int64_t total = tmp.tot.p[0];
  VEM_REQUIRE(total <= INT_MAX, VEM_ENOMEM, "more than 2^31-1 entries in a sparse pattern");
  return total;
}

void launch_compact_flags(hipStream_t s, int64_t n, const int* flag, const int* pos, int* out) {
  if (n > 0) k_compact<<<grid_of(n), 256, 0, s>>>(n, flag, pos, out);
}

}  // namespace vem

// ---------------------------------------------------------------------------------------
namespace {

template <class F>
vem_status guarded(vem_handle h, F&& body) {
  try {
    body();
    return VEM_OK;
  } catch (const Error& e) {
    if (h) h->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    if (h) h->last_error = "host allocation failed";
    return VEM_ENOMEM;
  } catch (const std::exception& e) {
    if (h) h->last_error = e.what();
    return VEM_EINVAL;
  }
}

void sync(vem_handle h) { VEM_HIP(hipStreamSynchronize(h->stream)); }

void check_launch() { VEM_HIP(hipGetLastError()); }

int read_err(vem_handle h, const int* derr) {
  int e = 0;
  VEM_HIP(hipMemcpyAsync(&e, derr, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  sync(h);
  return e;
}

std::string mesh_err_text(int e) {
  std::string t;
  if (e & 1) t += " cell with fewer than 4 or more than 64 faces;";
  if (e & 2) t += " face index out of range;";
  if (e & 4) t += " sign not +-1;";
  if (e & 8) t += " face with fewer than 3 vertices;";
  if (e & 16) t += " vertex index out of range;";
  if (e & 32) t += " face not shared by one cell or by two cells of opposite sign;";
  if (e & 64) t += " face of zero or non-finite area;";
  if (e & 128) t += " cell of non-positive or non-finite volume;";
  return "bad mesh:" + t;
}

// The device address of `scratch` on the current device, looked up once per device (the symbol
// has one copy per device, at a different address on each).
double* noalloc_scratch(int device) {
  static std::mutex mu;
  static std::map<int, double*> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it != addr.end()) return it->second;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    throw Error{VEM_EHIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e)};
  addr[device] = (double*)p;
  return (double*)p;
}

void ensure_scratch(vem_handle h) {
  if (!h->partials.p) {
    h->partials.alloc((size_t)kRedBlocks * kMaxDots);
    h->pcgpart.alloc(4 * (size_t)kPcgBlocks);
    h->scal.alloc(4 * kMaxDots + 16);
    h->pcg.alloc(1);
    h->hbuf.alloc(4 * kMaxDots + 16);
    // coherent: the kernels' stores reach host memory without passing through the GPU's caches
    h->hcol.alloc((size_t)(kMaxRestart + 1) * kColSlot, hipHostMallocMapped | hipHostMallocCoherent);
    VEM_HIP(hipHostGetDevicePointer((void**)&h->hcol_dev, h->hcol.p, 0));
    h->hpcg.alloc(1);
    for (hipEvent_t& e : h->step_done) VEM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    sync(h);
  }
}

// total of a device double array (synchronises)
// ----- coefficient-dependent values (K, diagonals, S, A_gamma), built lazily -----
void invalidate_values(vem_handle h) {
  h->k_ready = h->s_ready = h->a_ready = h->s32_ready = h->a32_ready = false;
  h->sz.ready = h->sz.ready32 = false;
}

// Builds the coefficient-dependent values a call needs and that are not current: K and diag(M)
// always, S when needS, A_gamma at gamma when needA, their FP32 shadows when f32.  The value
// kernels write the SELL copies directly; the CSR arrays are filled only for an export.
void ensure_values(vem_handle h, bool needS, bool needA, bool f32, double gamma) {
  hipStream_t s = h->stream;
  const DofLayout L = h->L;
  const int* bnd = h->bc == VEM_BC_FLUX ? h->is_bnd.p : nullptr;
  const bool redoA = needA && (!h->a_ready || gamma != h->gamma_A);
  if (!h->k_ready || redoA) {
    launch_values(s, L, h->cptr, h->cface, h->csign, h->ldof_ptr, h->sorted_gid, h->sorted_l, h->face_cell,
                  h->face_lidx, h->lmat_ptr, h->M1, h->lb_ptr, h->Bdiv1, h->nu, redoA ? 1.0 / gamma : 0.0, bnd,
                  h->Ks.slice_ptr, h->Ks.val, h->As.slice_ptr, redoA ? h->As.val.p : nullptr);
    launch_diag_inv(s, L.Nu, h->Kdiag, h->Ks.val, h->dM, h->dMinv);
    h->k_ready = true;
    if (redoA) {
      launch_diag_inv(s, L.Nu, h->Adiag, h->As.val, nullptr, h->dAinv);
      launch_col_scale(s, h->As, h->dAinv);
      launch_gershgorin(s, h->As, h->dAinv, h->partials, h->cheb.p + 1);
      h->gamma_A = gamma;
      h->a_ready = true;
      h->a32_ready = false;
    }
  }
  if (needS && !h->s_ready) {
    launch_schur_values(s, L, h->cptr, h->cface, h->csign, h->ldof_ptr, h->face_cell, h->face_lidx, h->lb_ptr,
                        h->Bdiv1, h->dM, bnd, h->S.rowptr, h->S.col, h->Ss.slice_ptr, h->Ss.val);
    launch_diag_inv(s, L.Np, h->Sdiag, h->Ss.val, nullptr, h->dSinv);
    launch_col_scale(s, h->Ss, h->dSinv);
    launch_gershgorin(s, h->Ss, h->dSinv, h->partials, h->cheb.p);
    h->s_ready = true;
    h->s32_ready = false;
  }
  if (f32 && needS && !h->s32_ready) {
    launch_col_scale32(s, h->Ss, h->dSinv, h->dSinv32);
    h->s32_ready = true;
  }
  if (f32 && needA && !h->a32_ready) {
    launch_col_scale32(s, h->As, h->dAinv, h->dAinv32);
    h->a32_ready = true;
  }
  check_launch();
}

void ensure_k(vem_handle h) { ensure_values(h, false, false, false, h->gamma_A); }

SchwarzMesh schwarz_mesh(vem_handle h) {
  return {h->nv,        h->nf,       h->nc,           h->fptr,       h->fvtx,       h->cptr, h->cface,
          h->face_cell, h->face_lidx, h->ldof_ptr,    h->sorted_gid, h->sorted_l,  h->csign};
}

// Block-Reg's Schwarz preconditioner for gamma: A_gamma's values (the lowest order's face system;
// order k builds its face system from the local matrices and needs only A_gamma's pattern), the
// edge patterns on first use, then the face system and the patch inverses when the coefficient,
// gamma or the boundary data changed; FP32 roundings when f32.
void ensure_schwarz(vem_handle h, double gamma, bool f32) {
  const DofLayout L = h->L;
  ensure_values(h, false, L.nint == 0, f32 && L.nint == 0, gamma);
  hipStream_t s = h->stream;
  const SchwarzMesh m = schwarz_mesh(h);
  if (!h->sz.built) schwarz_build(s, h->tmp, m, L, h->A, h->sz);
  if (!h->sz.ready || h->sz.gamma != gamma) {
    const int* bnd = h->bc == VEM_BC_FLUX ? h->is_bnd.p : nullptr;
    schwarz_values(s, m, L, h->lmat_ptr, h->M1, h->lb_ptr, h->Bdiv1, h->nu, 1.0 / gamma, bnd, h->A, h->As, h->sz);
    h->sz.gamma = gamma;
  }
  if (f32 && !h->sz.ready32) schwarz_round32(s, L, h->sz);
  check_launch();
}

void ensure_workspace(vem_handle h, int m) {
  int64_t N = h->L.Nu + h->L.Np;
  if (h->ws_N == N && h->ws_m >= m) return;
  h->Vb.alloc((size_t)(m + 1) * N);
  h->Zb.alloc((size_t)m * N);
  h->xw.alloc(N);
  int64_t nm = std::max<int64_t>(h->L.Nu, h->L.Np);
  h->pr.alloc(nm);
  h->pz.alloc(nm);
  h->ps.alloc(nm);
  h->pp.alloc(nm);
  h->pw0.alloc(nm);
  h->pw1.alloc(nm);
  h->px32.alloc(nm);
  h->pxw.alloc(nm);
  h->ws_N = N;
  h->ws_m = m;
}

// The four inner iterations: FP64 pipelined (the default), FP64 classical, FP32 classical
// (mixed precision, uncapped) and FP32 pipelined (mixed precision, capped).
enum InnerMode { kPipe64 = 0, kClassic64 = 1, kClassic32 = 2, kPipe32 = 3 };

void inner_iter(hipStream_t s, InnerMode mode, int i, const Sell& A, const PcgWork& w, const PcgWork32& w32,
                PcgState* st, double* part) {
  switch (mode) {
    case kPipe64: launch_pcg_iter(s, i, A, w, st, part); break;
    case kClassic64: launch_pcg_iter64c(s, i, A, w, st, part); break;
    case kClassic32: launch_pcg_iter32(s, i, A, w32, st, part); break;
    case kPipe32: launch_pcg_iter32p(s, i, A, w32, st, part); break;
  }
}

// The graph of kGraphIters iterations (2 .. 2+kGraphIters-1) for this matrix and precision,
// captured on the private stream on first use or when a referenced buffer moved.
hipGraphExec_t inner_graph(vem_handle h, const Sell& A, const PcgWork& w, const PcgWork32& w32, InnerMode mode,
                           InnerGraph& g) {
  const bool mixed = mode == kClassic32 || mode == kPipe32;
  const void* vals = mode == kPipe64      ? (const void*)A.val_cs.p
                     : mode == kClassic64 ? (const void*)A.val.p
                     : mode == kPipe32    ? (const void*)A.val32_cs.p
                                          : (const void*)A.val32.p;
  const void* key[8] = {vals, A.col.p, h->pr.p, h->pcg.p,
                        mixed ? (const void*)h->px32.p : (const void*)w.x, mixed ? (const void*)w32.dinv : w.dinv,
                        (const void*)(intptr_t)A.rows, (const void*)(intptr_t)A.nnz};
  if (g.exec && std::equal(key, key + 8, g.key)) return g.exec;
  g.reset();
  if (!h->cap) VEM_HIP(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  VEM_HIP(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
  hipGraph_t graph = nullptr;
  try {
    for (int t = 0; t < kGraphIters; ++t) {
      inner_iter(h->cap, mode, 2 + t, A, w, w32, h->pcg, h->pcgpart);
    }
  } catch (...) {
    (void)hipStreamEndCapture(h->cap, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  VEM_HIP(hipStreamEndCapture(h->cap, &graph));
  hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    g.exec = nullptr;
    throw Error{VEM_EHIP, std::string("hipGraphInstantiate failed: ") + hipGetErrorString(e)};
  }
  std::copy(key, key + 8, g.key);
  return g.exec;
}

// Inner Jacobi-CG: x ~ A^{-1} b to inner_tol.  FP64: pipelined, or classical on request (its
// residual stays closer to the true one on very ill-conditioned blocks).  FP32: pipelined when
// the iterations are capped at kBlindInner or fewer, classical otherwise (over hundreds of FP32
// iterations the pipelined recurrences lose positivity, while a capped solve that meets that
// guard simply stops with its iterate, which flexible GMRES accepts like any inexact solve).
// Iterations are enqueued in chunks between convergence checks; the first
// chunk is sized from the previous solve on the same matrix so that few
// launches find the solve already converged.  With graphs, iterations 0 and
// 1 are launched directly and the rest by replaying a captured run of
// kGraphIters iterations (inner_maxit is then rounded up to that length);
// the iterate is formed in a fixed workspace and copied to x.  Returns the
// iterations performed.
// `side` (a diagonal scaling) is performed by the Chebyshev form's first launch, or by a launch of its
// own before the other forms.
void inner_pcg(vem_handle h, const Sell& A, const double* dinv, const float* dinv32, const double* b, double* x,
               const vem_solve_opts& o, int& expect, InnerGraph& g64, InnerGraph& g32,
               const ScaleJob& side = ScaleJob{}) {
  hipStream_t s = h->stream;
  if (o.inner_form == VEM_INNER_CHEBYSHEV) {
    // a fixed polynomial of degree inner_maxit on [cheb_lo hi, hi]; inner_tol and graphs do not apply
    const double c = o.cheb_lo > 0.0 ? o.cheb_lo : 1.0 / 200.0;
    const double* inv_hi = h->cheb.p + (&A == &h->Ss ? 0 : 1);
    if (o.precision == VEM_MIXED) {
      PcgWork32 w{h->px32, (float*)h->pr.p, (float*)h->pz.p, (float*)h->ps.p, (float*)h->pp.p, (float*)h->pw0.p,
                  (float*)h->pw1.p, dinv32};
      launch_cheb<float>(s, A, w, b, inv_hi, c, o.inner_maxit, h->pcg, side);
      launch_to_f64(s, A.rows, h->px32, x);
    } else {
      PcgWork w{x, h->pr, h->pz, h->ps, h->pp, h->pw0, h->pw1, dinv};
      launch_cheb<double>(s, A, w, b, inv_hi, c, o.inner_maxit, h->pcg, side);
    }
    check_launch();
    return;
  }
  if (side.n > 0) launch_scale_by(s, side.n, side.x, side.d, 1.0, side.y);
  const bool mixed = o.precision == VEM_MIXED;
  const bool classical = o.inner_form == VEM_INNER_CLASSICAL;
  const InnerMode mode = !mixed ? (classical ? kClassic64 : kPipe64)
                                : (o.inner_maxit <= kBlindInner && !classical ? kPipe32 : kClassic32);
  const bool graphs = o.use_graphs != 0;
  PcgWork w{graphs ? h->pxw.p : x, h->pr, h->pz, h->ps, h->pp, h->pw0, h->pw1, dinv};
  // FP32 vectors live in the first half of the FP64 work buffers
  PcgWork32 w32{h->px32, (float*)h->pr.p, (float*)h->pz.p, (float*)h->ps.p, (float*)h->pp.p, (float*)h->pw0.p,
                (float*)h->pw1.p, dinv32};
  hipGraphExec_t exec = graphs ? inner_graph(h, A, w, w32, mode, mixed ? g32 : g64) : nullptr;
  switch (mode) {
    case kPipe64: launch_pcg_init(s, A, w, b, h->pcg, o.inner_tol, o.inner_maxit, h->pcgpart); break;
    case kClassic64: launch_pcg_init64c(s, A, w, b, h->pcg, o.inner_tol, h->pcgpart); break;
    case kClassic32: launch_pcg_init32(s, A, w32, b, h->pcg, o.inner_tol, o.inner_maxit, h->pcgpart); break;
    case kPipe32: launch_pcg_init32p(s, A, w32, b, h->pcg, o.inner_tol, o.inner_maxit, h->pcgpart); break;
  }
  check_launch();
  auto one = [&](int i) { inner_iter(s, mode, i, A, w, w32, h->pcg, h->pcgpart); };
  if (o.inner_maxit <= kBlindInner) {
    // A small cap: enqueue every iteration without looking at the state.  Once the
    // stop test fires, the remaining launches return at once; the iteration count is
    // summed on the device (PcgState::total) and read when the outer solve ends.
    int i = 0;
    while (i < o.inner_maxit) {
      if (exec && i >= 2 && i + kGraphIters <= o.inner_maxit) {
        VEM_HIP(hipGraphLaunch(exec, s));
        i += kGraphIters;
      } else {
        one(i);
        ++i;
      }
    }
    check_launch();
    if (mixed)
      launch_to_f64(s, A.rows, h->px32, x);
    else if (graphs)
      launch_copy(s, A.rows, h->pxw, x);
    return;
  }
  const int step = std::max(1, o.inner_check);
  int chunk = expect > 4 ? (expect * 7) / 8 : step;
  int i = 0;
  for (;;) {
    const int stop = std::min(o.inner_maxit, i + chunk);
    while (i < stop) {
      if (exec && i >= 2) {
        VEM_HIP(hipGraphLaunch(exec, s));
        i += kGraphIters;
      } else {
        one(i);
        ++i;
      }
    }
    check_launch();
    VEM_HIP(hipMemcpyAsync(h->hpcg.p, h->pcg.p, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    sync(h);
    if (h->hpcg.p->done || i >= o.inner_maxit) break;
    chunk = expect > 4 ? std::max(2, std::min(step, expect / 8)) : step;
  }
  if (mixed)
    launch_to_f64(s, A.rows, h->px32, x);
  else if (graphs)
    launch_copy(s, A.rows, h->pxw, x);
  expect = h->hpcg.p->count;
}

// Enqueue the iterations of one inner solve (one(i) enqueues iteration i): all of them without
// polling for a cap of kBlindInner or fewer, else in chunks between convergence checks, the first
// sized from the previous solve on the same block.
template <class One>
void run_inner(vem_handle h, const vem_solve_opts& o, int& expect, One&& one) {
  if (o.inner_maxit <= kBlindInner) {
    for (int i = 0; i < o.inner_maxit; ++i) one(i);
    check_launch();
    return;
  }
  const int step = std::max(1, o.inner_check);
  int chunk = expect > 4 ? (expect * 7) / 8 : step;
  int i = 0;
  for (;;) {
    const int stop = std::min(o.inner_maxit, i + chunk);
    while (i < stop) one(i++);
    check_launch();
    VEM_HIP(hipMemcpyAsync(h->hpcg.p, h->pcg.p, sizeof(PcgState), hipMemcpyDeviceToHost, h->stream));
    sync(h);
    if (h->hpcg.p->done || i >= o.inner_maxit) break;
    chunk = expect > 4 ? std::max(2, std::min(step, expect / 8)) : step;
  }
  expect = h->hpcg.p->count;
}

// z_u ~ A_gamma^{-1} v_u by CG on the face system preconditioned by the edge-patch Schwarz operator:
// the interior DOFs condensed into the right-hand side (order k), CG on the face DOFs (FP64, or
// FP32 with FP64 dot products), then the interior DOFs by back-substitution.
void schwarz_inner(vem_handle h, const vem_solve_opts& o, const double* v, double* z) {
  hipStream_t s = h->stream;
  const DofLayout L = h->L;
  const Schwarz& X = h->sz;
  const Sell& F = schwarz_face_sell(X, h->As, L);
  const SchwarzMesh m = schwarz_mesh(h);
  const int* bnd = h->bc == VEM_BC_FLUX ? h->is_bnd.p : nullptr;
  // iterations enqueued in chunks between polls: launches past convergence return at once
  const bool polled = o.inner_maxit > kBlindInner;
  if (o.precision == VEM_MIXED) {
    PcgWork32 w{h->px32, (float*)h->pr.p, (float*)h->pz.p, (float*)h->ps.p, (float*)h->pp.p, (float*)h->pw0.p,
                (float*)h->pw1.p, nullptr};
    launch_schwarz_rhs<float>(s, m, L, X, bnd, v, w.r);
    launch_scg_init<float>(s, X, w, h->pcg, o.inner_tol, h->pcgpart);
    run_inner(h, o, h->expect_A, [&](int i) { launch_scg_iter<float>(s, i, F, X, w, h->pcg, h->pcgpart, polled); });
    launch_to_f64(s, X.nF, h->px32, z);
  } else {
    PcgWork w{z, h->pr, h->pz, h->ps, h->pp, h->pw0, h->pw1, nullptr};
    launch_schwarz_rhs<double>(s, m, L, X, bnd, v, w.r);
    launch_scg_init<double>(s, X, w, h->pcg, o.inner_tol, h->pcgpart);
    run_inner(h, o, h->expect_A, [&](int i) { launch_scg_iter<double>(s, i, F, X, w, h->pcg, h->pcgpart, polled); });
  }
  if (L.nint > 0) launch_schwarz_back(s, m, L, X, v, z);
  check_launch();
}

// z = P^{-1} v for the chosen block preconditioner
void apply_prec(vem_handle h, const vem_solve_opts& o, const double* v, double* z) {
  hipStream_t s = h->stream;
  const int64_t Nu = h->L.Nu, Np = h->L.Np;
  switch (o.precond) {
    case VEM_PREC_SCHUR: {
      // z_u = diag(M)^{-1} v_u, performed inside the inner solve's first launch where it can be
      const ScaleJob zu{Nu, v, h->dMinv, z};
      const double* rp = v + Nu;
      if (h->bc == VEM_BC_FLUX) {
        // S has the constant pressure in its kernel: the inner CG takes the part of r_p
        // orthogonal to it (its own range)
        double* d = h->scal.p + 4 * kMaxDots;
        launch_dots(s, Np, 1, h->n_p, Np, rp, h->partials, d);
        launch_project(s, Np, rp, h->n_p, d, 1.0 / h->np_nn, h->ptmp);
        rp = h->ptmp;
      }
      inner_pcg(h, h->Ss, h->dSinv, h->dSinv32, rp, z + Nu, o, h->expect_S, h->gS, h->gS32, zu);
      return;
    }
    case VEM_PREC_REG:
      if (o.reg_inner == VEM_REG_SCHWARZ)
        schwarz_inner(h, o, v, z);
      else
        inner_pcg(h, h->As, h->dAinv, h->dAinv32, v, z, o, h->expect_A, h->gA, h->gA32);
      launch_scale_by(s, Np, v + Nu, nullptr, 1.0 / h->gamma_A, z + Nu);
      return;
    default:
      launch_copy(s, Nu + Np, v, z);
  }
}

// Right-hand side with flux boundary data (from the coefficient and the coefficient-free local
// matrices, not from the assembled K): the known fluxes move to the right, the prescribed rows
// carry them, and the pressure part is projected off the constant pressure (this removes the
// quadrature-level mismatch between int f and the boundary flux, so the system is consistent).
const double* flux_rhs(vem_handle h) {
  hipStream_t s = h->stream;
  const DofLayout L = h->L;
  launch_flux_rhs(s, L, h->cptr, h->cface, h->csign, h->face_cell, h->face_lidx, h->lmat_ptr, h->M1, h->lb_ptr,
                  h->Bdiv1, h->nu, h->is_bnd, h->xB, h->rhs, h->rhs_flux);
  double* d = h->scal.p + 4 * kMaxDots;
  double* bp = h->rhs_flux.p + L.Nu;
  launch_dots(s, L.Np, 1, h->n_p, L.Np, bp, h->partials, d);
  launch_project(s, L.Np, bp, h->n_p, d, 1.0 / h->np_nn, bp);
  check_launch();
  return h->rhs_flux.p;
}

// Loads F from f at the cell points, and either the pressure term g from p_D at the boundary points
// or the prescribed boundary fluxes xB from u at the boundary points (structure of arrays).
// The per-tetrahedron sums go to `fixed` when given (at least tet_sum_len(h) doubles), else to the
// handle's grow-only pool.
int64_t tet_sum_len(vem_handle h) { return h->family == VEM_LO ? h->ntet : h->ntet * h->L.npd; }

void set_loads(vem_handle h, const double* f_qp, const double* pD_qp, const double* u_qp, double* fixed = nullptr) {
    hipStream_t s = h->stream;
    const int64_t nqf = (int64_t)h->nbtri * h->npts_face;
    if (u_qp) launch_fill(s, h->L.Nu, 0.0, h->xB);
    launch_fill(s, h->L.Nu, 0.0, h->rhs);
    DBuf<double>& pool = h->tmp.f64[0];
    if (!fixed) pool.reserve(tet_sum_len(h));
    double* tsum = fixed ? fixed : pool.p;
    if (h->family == VEM_LO) {
      launch_load_tets(s, h->ntet, h->npts_cell, h->qw_cell, h->tet_inc, h->tet_a, h->inc_cell, h->xyz, h->fptr,
                       h->fvtx, h->cface, h->csign, h->c_xref, f_qp, tsum);
      launch_load_cells(s, h->nc, h->cell_tet_ptr, tsum, h->rhs.p + h->L.Nu);
      if (pD_qp)
        launch_bnd_rhs(s, (int)h->nbf, h->npts_face, h->qw_face, h->bface, h->btri_ptr, h->xyz, h->fptr, h->fvtx,
                       h->face_cell, pD_qp, h->rhs);
      if (u_qp)
        launch_bnd_flux(s, (int)h->nbf, h->npts_face, nqf, h->qw_face, h->bface, h->btri_ptr, h->xyz, h->fptr,
                        h->fvtx, h->f_normal, h->f_area, u_qp, h->xB);
    } else {
      PaperLoadArgs a{};
      a.s = s;
      a.nc = h->nc;
      a.nb = (int)h->nbf;
      a.npts_cell = h->npts_cell;
      a.npts_face = h->npts_face;
      a.ntet = h->ntet;
      a.ref_cell = h->qref_cell;
      a.w_cell = h->qw_cell;
      a.ref_face = h->qref_face;
      a.w_face = h->qw_face;
      a.tet_inc = h->tet_inc;
      a.tet_a = h->tet_a;
      a.inc_cell = h->inc_cell;
      a.fptr = h->fptr;
      a.fvtx = h->fvtx;
      a.cface = h->cface;
      a.cell_tet_ptr = h->cell_tet_ptr;
      a.bface = h->bface;
      a.btri_ptr = h->btri_ptr;
      a.face_cell = h->face_cell;
      a.csign = h->csign;
      a.xyz = h->xyz;
      a.xref = h->c_xref;
      a.ccen = h->c_cen;
      a.cdiam = h->c_diam;
      a.cvol = h->c_vol;
      a.cmom = h->pk_cmom;
      a.fcen = h->f_cen;
      a.fdiam = h->f_diam;
      a.fe1 = h->f_e1;
      a.fe2 = h->f_e2;
      a.Tf = h->pk_Tf;
      a.fq = f_qp;
      a.pq = pD_qp;
      a.tet_sum = tsum;
      a.rhs_p = h->rhs.p + h->L.Nu;
      a.rhs_u = h->rhs;
      a.uq = u_qp;
      a.fnormal = h->f_normal;
      a.farea = h->f_area;
      a.nq_face_total = nqf;
      a.xB = h->xB;
      launch_paper_loads(h->korder, a);
    }
    check_launch();
    sync(h);
}

void require_disc(vem_handle h) {
  VEM_REQUIRE(h && h->has_disc, VEM_EINVAL, "call vem_set_mesh and vem_discretize first");
}

}  // namespace

// =======================================================================================
extern "C" {

void vem_solve_opts_default(vem_solve_opts* o) {
  if (!o) return;
  o->precond = VEM_PREC_SCHUR;
  o->restart = 30;
  o->maxit = 5000;
  o->use_x0 = 0;
  o->tol = 1e-8;
  o->inner_tol = 1e-6;
  o->inner_maxit = 5000;
  o->inner_check = 32;
  o->gamma = 0.0;
  o->precision = VEM_FP64;
  o->use_graphs = 0;
  o->inner_form = VEM_INNER_PIPELINED;
  o->reg_inner = VEM_REG_SCHWARZ;
  o->cheb_lo = 0.0;
}

vem_status vem_create(vem_handle* out, void* stream) {
  if (!out) return VEM_EINVAL;
  vem_ctx* h = nullptr;
  try {
    h = new vem_ctx();
  } catch (...) {
    return VEM_ENOMEM;
  }
  vem_status st = guarded(h, [&] {
    VEM_HIP(hipGetDevice(&h->device));
    h->stream = (hipStream_t)stream;
    ensure_scratch(h);
    h->noalloc = noalloc_scratch(h->device);
  });
  if (st != VEM_OK) {
    delete h;
    *out = nullptr;
    return st;
  }
  *out = h;
  return VEM_OK;
}

vem_status vem_destroy(vem_handle h) {
  if (!h) return VEM_OK;
  (void)hipStreamSynchronize(h->stream);
  delete h;
  return VEM_OK;
}

const char* vem_status_string(vem_status st) {
  switch (st) {
    case VEM_OK: return "ok";
    case VEM_NOT_CONVERGED: return "not converged within maxit";
    case VEM_EINVAL: return "invalid argument";
    case VEM_EBADMESH: return "bad mesh";
    case VEM_ENOMEM: return "out of memory or size limit";
    case VEM_EHIP: return "HIP runtime error";
    case VEM_EBREAKDOWN: return "Krylov breakdown";
    case VEM_ENAN: return "NaN or Inf in the solve";
    default: return "unknown status";
  }
}

const char* vem_last_error(vem_handle h) { return h ? h->last_error.c_str() : "null handle"; }

vem_status vem_set_mesh(vem_handle h, int64_t nv, const double* xyz, int64_t nf, const int32_t* face_ptr,
                        const int32_t* face_vtx, int64_t nc, const int32_t* cell_ptr, const int32_t* cell_face,
                        const int8_t* cell_face_sign, int mem_kind) {
  if (!h) return VEM_EINVAL;
  return guarded(h, [&] {
    VEM_REQUIRE(nv > 0 && nf > 0 && nc > 0 && nv < INT_MAX && nf < INT_MAX && nc < INT_MAX, VEM_EINVAL,
                "mesh sizes must be positive and below 2^31");
    VEM_REQUIRE(xyz && face_ptr && face_vtx && cell_ptr && cell_face && cell_face_sign, VEM_EINVAL,
                "null mesh array");
    VEM_REQUIRE(mem_kind == VEM_MEM_HOST || mem_kind == VEM_MEM_DEVICE, VEM_EINVAL, "bad mem_kind");
    hipStream_t s = h->stream;
    h->has_mesh = false;
    h->has_disc = false;
    h->sz.built = h->sz.ready = h->sz.ready32 = false;
    if (mem_kind == VEM_MEM_HOST) {
      // offsets validated on the host
      h->h_fptr.assign(face_ptr, face_ptr + nf + 1);
      h->h_cptr.assign(cell_ptr, cell_ptr + nc + 1);
      VEM_REQUIRE(h->h_fptr[0] == 0 && h->h_cptr[0] == 0, VEM_EBADMESH, "offset arrays must start at 0");
      for (int64_t i = 0; i < nf; ++i)
        VEM_REQUIRE(h->h_fptr[i + 1] >= h->h_fptr[i], VEM_EBADMESH, "face_ptr not monotone");
      int maxcf = 0;
      for (int64_t i = 0; i < nc; ++i) {
        VEM_REQUIRE(h->h_cptr[i + 1] >= h->h_cptr[i], VEM_EBADMESH, "cell_ptr not monotone");
        maxcf = std::max(maxcf, h->h_cptr[i + 1] - h->h_cptr[i]);
      }
      h->nfv = h->h_fptr[nf];
      h->ncf = h->h_cptr[nc];
      h->max_cell_faces = maxcf;
      h->fptr.alloc(nf + 1);
      h->cptr.alloc(nc + 1);
      VEM_HIP(hipMemcpyAsync(h->fptr.p, h->h_fptr.data(), (nf + 1) * sizeof(int), hipMemcpyHostToDevice, s));
      VEM_HIP(hipMemcpyAsync(h->cptr.p, h->h_cptr.data(), (nc + 1) * sizeof(int), hipMemcpyHostToDevice, s));
    } else {
      // offsets validated on the device: no copy of the arrays to the host
      h->fptr.alloc(nf + 1);
      h->cptr.alloc(nc + 1);
      VEM_HIP(hipMemcpyAsync(h->fptr.p, face_ptr, (nf + 1) * sizeof(int), hipMemcpyDefault, s));
      VEM_HIP(hipMemcpyAsync(h->cptr.p, cell_ptr, (nc + 1) * sizeof(int), hipMemcpyDefault, s));
      DBuf<int>& chk = h->tmp.i32[0];
      chk.reserve(2);
      fill_i32(s, 2, 0, chk);
      launch_check_offsets(s, nf, h->fptr, nc, h->cptr, chk);
      check_launch();
      h->tmp.ti.alloc(8);
      int* r = h->tmp.ti.p;
      VEM_HIP(hipMemcpyAsync(r, chk.p, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
      VEM_HIP(hipMemcpyAsync(r + 2, h->fptr.p + nf, sizeof(int), hipMemcpyDeviceToHost, s));
      VEM_HIP(hipMemcpyAsync(r + 3, h->cptr.p + nc, sizeof(int), hipMemcpyDeviceToHost, s));
      sync(h);
      VEM_REQUIRE(!(r[0] & 4), VEM_EBADMESH, "offset arrays must start at 0");
      VEM_REQUIRE(!(r[0] & 1), VEM_EBADMESH, "face_ptr not monotone");
      VEM_REQUIRE(!(r[0] & 2), VEM_EBADMESH, "cell_ptr not monotone");
      h->nfv = r[2];
      h->ncf = r[3];
      h->max_cell_faces = r[1];
      h->h_fptr.clear();
      h->h_cptr.clear();
    }
    h->nv = (int)nv;
    h->nf = (int)nf;
    h->nc = (int)nc;
    h->xyz.alloc(3 * nv);
    h->fvtx.alloc(h->nfv);
    h->cface.alloc(h->ncf);
    h->csign.alloc(h->ncf);
    h->inc_cell.alloc(h->ncf);
    VEM_HIP(hipMemcpyAsync(h->xyz.p, xyz, 3 * nv * sizeof(double), hipMemcpyDefault, s));
    VEM_HIP(hipMemcpyAsync(h->fvtx.p, face_vtx, h->nfv * sizeof(int), hipMemcpyDefault, s));
    VEM_HIP(hipMemcpyAsync(h->cface.p, cell_face, h->ncf * sizeof(int), hipMemcpyDefault, s));
    VEM_HIP(hipMemcpyAsync(h->csign.p, cell_face_sign, h->ncf * sizeof(int8_t), hipMemcpyDefault, s));
    // face -> (cell, local index) for both orientations, with validation
    h->face_cnt.alloc(2 * (size_t)nf);
    h->face_cell.alloc(2 * (size_t)nf);
    h->face_lidx.alloc(2 * (size_t)nf);
    h->is_bnd.alloc(nf + 1);
    fill_i32(s, 2 * nf, 0, h->face_cnt);
    fill_i32(s, 2 * nf, -1, h->face_cell);
    fill_i32(s, 2 * nf, -1, h->face_lidx);
    DBuf<int>& derr = h->tmp.i32[0];
    derr.reserve(1);
    fill_i32(s, 1, 0, derr);
    launch_check_mesh(s, h->nv, h->nf, h->nc, h->fptr, h->fvtx, h->cptr, h->cface, h->csign, h->face_cnt,
                      h->face_cell, h->face_lidx, h->inc_cell, derr);
    check_launch();
    int e = read_err(h, derr);
    VEM_REQUIRE(e == 0, VEM_EBADMESH, mesh_err_text(e));
    h->has_mesh = true;
  });
}

vem_status vem_discretize(vem_handle h, int family, int k, int load_points) {
  if (!h) return VEM_EINVAL;
  return guarded(h, [&] {
    VEM_REQUIRE(h->has_mesh, VEM_EINVAL, "call vem_set_mesh first");
    VEM_REQUIRE(family == VEM_LO || (family == VEM_PAPER && k >= 1 && k <= 3), VEM_EINVAL,
                "family must be VEM_LO, or VEM_PAPER with k in 1..3");
    VEM_REQUIRE(load_points >= 1 && load_points <= 6, VEM_EINVAL, "load_points must be in 1..6");
    hipStream_t s = h->stream;
    h->has_disc = false;
    h->sz.built = h->sz.ready = h->sz.ready32 = false;
    const int nf = h->nf, nc = h->nc;
    // ---- a1: geometry
    h->f_area.alloc(nf);
    h->f_normal.alloc(3 * (size_t)nf);
    h->f_cen.alloc(3 * (size_t)nf);
    h->f_diam.alloc(nf);
    h->f_e1.alloc(3 * (size_t)nf);
    h->f_e2.alloc(3 * (size_t)nf);
    h->c_vol.alloc(nc);
    h->c_cen.alloc(3 * (size_t)nc);
    h->c_diam.alloc(nc);
    h->c_xref.alloc(3 * (size_t)nc);
    launch_face_geometry(s, nf, h->xyz, h->fptr, h->fvtx, h->f_area, h->f_normal, h->f_cen, h->f_diam, h->f_e1,
                         h->f_e2);
    launch_cell_geometry(s, nc, h->xyz, h->fptr, h->fvtx, h->cptr, h->cface, h->csign, h->c_vol, h->c_cen,
                         h->c_diam, h->c_xref);
    check_launch();
    DBuf<int>& derr = h->tmp.i32[0];
    derr.reserve(1);
    fill_i32(s, 1, 0, derr);
    fill_i32(s, 1, 0, h->is_bnd.p + nf);
    launch_check_faces(s, nf, h->face_cnt, h->f_area, h->is_bnd, derr);
    launch_check_cells(s, nc, h->c_vol, derr);
    // the error flags and the sum of the cell diameters come back with one synchronisation
    ensure_scratch(h);
    launch_sum(s, nc, h->c_diam, h->partials, h->scal);
    check_launch();
    h->tmp.ti.alloc(8);
    VEM_HIP(hipMemcpyAsync(h->tmp.ti.p, derr.p, sizeof(int), hipMemcpyDeviceToHost, s));
    VEM_HIP(hipMemcpyAsync(h->hbuf.p, h->scal.p, sizeof(double), hipMemcpyDeviceToHost, s));
    sync(h);
    const int e = h->tmp.ti.p[0];
    VEM_REQUIRE(e == 0, VEM_EBADMESH, mesh_err_text(e));
    h->h = h->hbuf.p[0] / nc;
    h->gamma_default = h->h * h->h;

    // ---- quadrature support: tetrahedra of the cells, triangles of the boundary faces
    h->load_n = load_points;
    if (h->qrule_n != load_points) {  // the reference rules depend on n only
      h->qrule_n = 0;
      std::vector<double> p, w;
      tet_reference_rule(load_points, p, w);
      h->npts_cell = (int)w.size();
      h->qref_cell.alloc(p.size());
      h->qw_cell.alloc(w.size());
      VEM_HIP(hipMemcpyAsync(h->qref_cell.p, p.data(), p.size() * sizeof(double), hipMemcpyHostToDevice, s));
      VEM_HIP(hipMemcpyAsync(h->qw_cell.p, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, s));
      sync(h);
      tri_reference_rule(load_points, p, w);
      h->npts_face = (int)w.size();
      h->qref_face.alloc(p.size());
      h->qw_face.alloc(w.size());
      VEM_HIP(hipMemcpyAsync(h->qref_face.p, p.data(), p.size() * sizeof(double), hipMemcpyHostToDevice, s));
      VEM_HIP(hipMemcpyAsync(h->qw_face.p, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, s));
      sync(h);
      h->qrule_n = load_points;
    }
    {
      DBuf<int>& cnt = h->tmp.i32[1];
      cnt.reserve(nc + 1);
      launch_tet_counts(s, nc, h->fptr, h->cptr, h->cface, cnt);
      check_launch();
      h->cell_tet_ptr.alloc(nc + 1);
      DBuf<int>& pos = h->tmp.i32[2];
      pos.reserve(nf + 1);
      // tetrahedron offsets and boundary-face positions: one synchronisation for both totals
      scan_reserve(h->tmp, std::max(nc, nf));
      scan_i32_async(s, h->tmp, cnt, nc, h->cell_tet_ptr, h->tmp.i64[3], 0);
      scan_i32_async(s, h->tmp, h->is_bnd, nf, pos, h->tmp.i64[2], 1);
      sync(h);
      VEM_REQUIRE(h->tmp.tot.p[0] <= INT_MAX, VEM_ENOMEM, "more than 2^31-1 quadrature tetrahedra");
      h->ntet = h->tmp.tot.p[0];
      h->nbf = h->tmp.tot.p[1];
      h->tet_inc.alloc(h->ntet);
      h->tet_a.alloc(h->ntet);
      launch_tets(s, nc, h->fptr, h->cptr, h->cface, h->cell_tet_ptr, h->tet_inc, h->tet_a);
      check_launch();
      h->bface.alloc(h->nbf > 0 ? h->nbf : 1);
      launch_compact_flags(s, nf, h->is_bnd, pos, h->bface);
      DBuf<int>& tc = h->tmp.i32[3];
      tc.reserve(h->nbf + 1);
      launch_bnd_tri_counts(s, (int)h->nbf, h->bface, h->fptr, tc);
      check_launch();
      h->btri_ptr.alloc(h->nbf + 1);
      h->nbtri = h->nbf > 0 ? scan_i32(s, h->tmp, tc, h->nbf, h->btri_ptr) : 0;
      if (h->nbf == 0) fill_i32(s, 1, 0, h->btri_ptr);
    }

    // ---- a2-a4: local matrices (coefficient-free)
    DofLayout L{};
    L.nf = nf;
    L.nc = nc;
    L.nfd = 1;
    L.nint = 0;
    L.npd = 1;
    if (family == VEM_PAPER) {
      PaperSizes z = paper_sizes(k);
      L.nfd = z.nfd;
      L.nint = z.nint;
      L.npd = z.npd;
    }
    L.Nu = (int64_t)nf * L.nfd + (int64_t)nc * L.nint;
    L.Np = (int64_t)nc * L.npd;
    h->L = L;
    h->family = family;
    h->korder = family == VEM_PAPER ? k : 0;
    int64_t tot_ldof = 0;
    {
      DBuf<int64_t>& nd = h->tmp.i64[0];
      DBuf<int64_t>& nm = h->tmp.i64[1];
      DBuf<int64_t>& nb = h->tmp.i64[2];
      nd.reserve(nc + 1);
      nm.reserve(nc + 1);
      nb.reserve(nc + 1);
      launch_cell_sizes(s, L, h->cptr, nd, nm, nb);
      check_launch();
      DBuf<int64_t>& p64 = h->tmp.i64[3];
      p64.reserve(nc + 1);
      h->lmat_ptr.alloc(nc + 1);
      h->lb_ptr.alloc(nc + 1);
      // local DOF, matrix and divergence-block offsets: one synchronisation for the three totals
      scan_reserve(h->tmp, nc);
      scan_i64_async(s, h->tmp, nd, nc, p64, 0);
      scan_i64_async(s, h->tmp, nm, nc, h->lmat_ptr, 1);
      scan_i64_async(s, h->tmp, nb, nc, h->lb_ptr, 2);
      sync(h);
      const int64_t tot = h->tmp.tot.p[0], nmat = h->tmp.tot.p[1], nbd = h->tmp.tot.p[2];
      VEM_REQUIRE(tot <= INT_MAX, VEM_ENOMEM, "too many local DOFs");
      tot_ldof = tot;
      h->ldof_ptr.alloc(nc + 1);
      k_narrow<<<grid_of(nc + 1), 256, 0, s>>>(nc + 1, p64.p, h->ldof_ptr.p);
      h->M1.alloc(nmat);
      h->Bdiv1.alloc(nbd);
      h->sorted_gid.alloc(tot);
      h->sorted_l.alloc(tot);
    }
    if (family == VEM_LO) {
      launch_lo_local(s, h->ncf, h->inc_cell, h->cptr, h->cface, h->csign, h->f_area, h->f_normal, h->f_cen,
                      h->c_vol, h->c_cen, h->lmat_ptr, h->M1, h->lb_ptr, h->Bdiv1);
    } else {
      PaperSizes z = paper_sizes(k);
      if (h->pk_trip_nq != z.nq) {
        h->pk_trip_nq = 0;
        std::vector<double> p2, w2, trip;
        tri_reference_rule(z.nq, p2, w2);
        for (size_t r = 0; r < w2.size(); ++r) {
          trip.push_back(p2[2 * r]);
          trip.push_back(p2[2 * r + 1]);
          trip.push_back(w2[r]);
        }
        h->pk_trip.alloc(trip.size());
        VEM_HIP(hipMemcpyAsync(h->pk_trip.p, trip.data(), trip.size() * sizeof(double), hipMemcpyHostToDevice, s));
        sync(h);  // `trip` is released at the end of this scope
        h->pk_trip_nq = z.nq;
      }
      DBuf<double>& tri = h->pk_trip;
      DBuf<double>& FP = h->tmp.f64[1];
      DBuf<double>& FM = h->tmp.f64[2];
      DBuf<double>& Dg = h->tmp.f64[3];
      DBuf<double>& Pg = h->tmp.f64[4];
      DBuf<double>& Xg = h->tmp.f64[5];
      DBuf<double>& Cg = h->tmp.f64[6];
      FP.reserve((size_t)h->ncf * z.nsm);
      FM.reserve((size_t)h->ncf * z.nfm);
      h->pk_Tf.alloc((size_t)nf * z.nfd * z.nfd);
      h->pk_cmom.alloc((size_t)nc * z.nsm);
      Dg.reserve((size_t)tot_ldof * z.n3);
      Pg.reserve((size_t)tot_ldof * z.n3);
      Xg.reserve((size_t)tot_ldof * z.n3);
      Cg.reserve((size_t)tot_ldof * z.npd);
      PaperLocalArgs a{};
      a.s = s;
      a.nf = nf;
      a.nc = nc;
      a.ninc = h->ncf;
      a.inc_cell = h->inc_cell;
      a.cptr = h->cptr;
      a.cface = h->cface;
      a.fptr = h->fptr;
      a.fvtx = h->fvtx;
      a.ldof_ptr = h->ldof_ptr;
      a.csign = h->csign;
      a.xyz = h->xyz;
      a.farea = h->f_area;
      a.fnormal = h->f_normal;
      a.fcen = h->f_cen;
      a.fdiam = h->f_diam;
      a.fe1 = h->f_e1;
      a.fe2 = h->f_e2;
      a.cvol = h->c_vol;
      a.ccen = h->c_cen;
      a.cdiam = h->c_diam;
      a.tri_ref = tri;
      a.FP = FP;
      a.FM = FM;
      a.Tf = h->pk_Tf;
      a.cmom = h->pk_cmom;
      a.Dg = Dg;
      a.Pg = Pg;
      a.Xg = Xg;
      a.Cg = Cg;
      a.lmat_ptr = h->lmat_ptr;
      a.lb_ptr = h->lb_ptr;
      a.M1 = h->M1;
      a.Bdiv1 = h->Bdiv1;
      launch_paper_local(k, a);
      check_launch();
    }
    launch_ldof_sort(s, L, h->cptr, h->cface, h->ldof_ptr, h->sorted_gid, h->sorted_l);
    check_launch();

    // ---- a5/a6: patterns of K, A_gamma and S
    const int64_t N = L.Nu + L.Np;
    {
      DBuf<int>& lenK = h->tmp.i32[1];
      DBuf<int>& lenA = h->tmp.i32[2];
      DBuf<int>& lenS = h->tmp.i32[3];
      lenK.reserve(N + 1);
      lenA.reserve(L.Nu + 1);
      lenS.reserve(L.Np + 1);
      launch_rowlen(s, L, h->cptr, h->ldof_ptr, h->sorted_gid, h->face_cell, h->face_lidx, h->cface, lenK, lenA,
                    lenS);
      check_launch();
      h->K.rows = N;
      h->A.rows = L.Nu;
      h->S.rows = L.Np;
      h->K.rowptr.alloc(N + 1);
      h->A.rowptr.alloc(L.Nu + 1);
      h->S.rowptr.alloc(L.Np + 1);
      // row offsets of K, A_gamma and S: one synchronisation for the three totals
      scan_reserve(h->tmp, N);
      scan_i32_async(s, h->tmp, lenK, N, h->K.rowptr, h->tmp.i64[0], 0);
      scan_i32_async(s, h->tmp, lenA, L.Nu, h->A.rowptr, h->tmp.i64[1], 1);
      scan_i32_async(s, h->tmp, lenS, L.Np, h->S.rowptr, h->tmp.i64[2], 2);
      sync(h);
      for (int m = 0; m < 3; ++m)
        VEM_REQUIRE(h->tmp.tot.p[m] <= INT_MAX, VEM_ENOMEM, "more than 2^31-1 entries in a sparse pattern");
      h->K.nnz = h->tmp.tot.p[0];
      h->A.nnz = h->tmp.tot.p[1];
      h->S.nnz = h->tmp.tot.p[2];
    }
    h->K.col.alloc(h->K.nnz);
    h->K.val.alloc(h->K.nnz);
    h->A.col.alloc(h->A.nnz);
    h->A.val.alloc(h->A.nnz);
    h->S.col.alloc(h->S.nnz);
    h->S.val.alloc(h->S.nnz);
    h->Kdiag.alloc(L.Nu);
    h->Adiag.alloc(L.Nu);
    h->Sdiag.alloc(L.Np);
    launch_fill_patterns(s, L, h->cptr, h->ldof_ptr, h->sorted_gid, h->face_cell, h->face_lidx, h->cface,
                         h->K.rowptr, h->K.col, h->Kdiag, h->A.rowptr, h->A.col, h->Adiag, h->S.rowptr, h->S.col,
                         h->Sdiag);
    check_launch();
    {
      const Csr* csr[3] = {&h->K, &h->A, &h->S};
      Sell* sell[3] = {&h->Ks, &h->As, &h->Ss};
      build_sells(s, h->tmp, csr, sell, 3);
      // the diagonals are read from the SELL values
      sell_diag_slots(s, L.Nu, h->K, h->Ks, h->Kdiag);  // K: the flux rows only
      sell_diag_slots(s, L.Nu, h->A, h->As, h->Adiag);
      sell_diag_slots(s, L.Np, h->S, h->Ss, h->Sdiag);
      check_launch();
    }
    h->dM.alloc(L.Nu);
    h->dMinv.alloc(L.Nu);
    h->dAinv.alloc(L.Nu);
    h->dSinv.alloc(L.Np);
    h->dAinv32.alloc(L.Nu);
    h->dSinv32.alloc(L.Np);
    h->cheb.alloc(2);
    h->nu.alloc(nc);
    launch_fill(s, nc, 1.0, h->nu);
    h->rhs.alloc(N);
    launch_fill(s, N, 0.0, h->rhs);
    // flux boundary data: prescribed fluxes, the constant pressure and the mean weights
    h->xB.alloc(L.Nu);
    launch_fill(s, L.Nu, 0.0, h->xB);
    h->rhs_flux.alloc(N);
    h->n_p.alloc(L.Np);
    h->pw.alloc(L.Np);
    h->ptmp.alloc(L.Np);
    launch_pressure_constants(s, L, family == VEM_PAPER ? paper_sizes(k).nsm : 0,
                              family == VEM_PAPER ? h->pk_cmom.p : nullptr, h->c_vol, h->n_p, h->pw);
    {
      double* d = h->scal.p + 4 * kMaxDots;
      double two[2];
      launch_dots(s, L.Np, 1, h->n_p, L.Np, h->n_p, h->partials, d);
      launch_dots(s, L.Np, 1, h->pw, L.Np, h->n_p, h->partials, d + 1);
      check_launch();
      VEM_HIP(hipMemcpyAsync(two, d, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      sync(h);
      h->np_nn = two[0];
      h->np_wn = two[1];
    }
    h->gamma_A = h->gamma_default;
    invalidate_values(h);
    h->has_disc = true;
  });
}

vem_status vem_get_sizes(vem_handle h, vem_sizes* o) {
  if (!h || !o) return VEM_EINVAL;
  return guarded(h, [&] {
    require_disc(h);
    std::memset(o, 0, sizeof(*o));
    o->n_vertices = h->nv;
    o->n_faces = h->nf;
    o->n_cells = h->nc;
    o->n_u = h->L.Nu;
    o->n_p = h->L.Np;
    o->n = h->L.Nu + h->L.Np;
    o->nnz_K = h->K.nnz;
    o->nnz_schur = h->S.nnz;
    o->nnz_reg = h->A.nnz;
    o->n_qp_cell = h->ntet * h->npts_cell;
    o->n_qp_face = h->nbtri * h->npts_face;
    o->load_points = h->load_n;
    o->max_cell_faces = h->max_cell_faces;
    o->h = h->h;
    o->gamma = h->gamma_default;
    o->n_face_dofs = (int64_t)h->L.nf * h->L.nfd;
  });
}

vem_status vem_get_quadrature(vem_handle h, double* qp_cell, double* qp_face) {
  if (!h) return VEM_EINVAL;
  return guarded(h, [&] {
    require_disc(h);
    hipStream_t s = h->stream;
    if (qp_cell)
      launch_qp_cell(s, h->ntet, h->npts_cell, h->qref_cell, h->tet_inc, h->tet_a, h->inc_cell, h->xyz, h->fptr,
                     h->fvtx, h->cface, h->c_xref, qp_cell);
    if (qp_face)
      launch_qp_face(s, (int)h->nbf, h->npts_face, (int64_t)h->nbtri * h->npts_face, h->qref_face, h->bface,
                     h->btri_ptr, h->xyz, h->fptr, h->fvtx, qp_face);
    check_launch();
  });
}

vem_status vem_set_coefficient(vem_handle h, const double* nu) {
  if (!h || !nu) return VEM_EINVAL;
  return guarded(h, [&] {
    require_disc(h);
    hipStream_t s = h->stream;
    // staged and checked first, so that a rejected field leaves the previous coefficient in place
    DBuf<double>& stage = h->tmp.f64[7];
    stage.reserve(h->nc);
    VEM_HIP(hipMemcpyAsync(stage.p, nu, h->nc * sizeof(double), hipMemcpyDefault, s));
    DBuf<int>& bad = h->tmp.i32[0];
    bad.reserve(1);
    fill_i32(s, 1, 0, bad);
    launch_check_cells(s, (int)h->nc, stage.p, bad);  // flags a value that is not positive and finite
    check_launch();
    h->tmp.ti.alloc(8);
    VEM_HIP(hipMemcpyAsync(h->tmp.ti.p, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    sync(h);
    VEM_REQUIRE(h->tmp.ti.p[0] == 0, VEM_EINVAL, "coefficient nu must be positive and finite in every cell");
    // stream-ordered: the caller's array has been read by now
    VEM_HIP(hipMemcpyAsync(h->nu.p, stage.p, h->nc * sizeof(double), hipMemcpyDeviceToDevice, s));
    invalidate_values(h);
  });
}

vem_status vem_set_boundary(vem_handle h, int kind) {
  if (!h) return VEM_EINVAL;
  return guarded(h, [&] {
    VEM_REQUIRE(kind == VEM_BC_PRESSURE || kind == VEM_BC_FLUX, VEM_EINVAL, "unknown boundary data kind");
    if (kind != h->bc) {
      h->bc = kind;
      invalidate_values(h);
      if (h->has_disc) {
        launch_fill(h->stream, h->L.Nu + h->L.Np, 0.0, h->rhs);
        launch_fill(h->stream, h->L.Nu, 0.0, h->xB);
        check_launch();
        sync(h);
      }
    }
  });
}

vem_status vem_set_rhs(vem_handle h, const double* f_qp, const double* pD_qp) {
  if (!h || !f_qp) return VEM_EINVAL;
  return guarded(h, [&] {
    require_disc(h);
    VEM_REQUIRE(h->bc == VEM_BC_PRESSURE, VEM_EINVAL, "flux boundary data: use vem_set_rhs_flux");
    set_loads(h, f_qp, pD_qp, nullptr);
  });
}

vem_status vem_set_coefficient_batch(vem_handle h, int64_t nbatch, const double* nu) {
  if (!h || !nu || nbatch < 1) return VEM_EINVAL;
  return guarded(h, [&] {
    require_disc(h);
    hipStream_t s = h->stream;
    const int64_t n = nbatch * h->nc;
    VEM_REQUIRE(n <= INT_MAX, VEM_EINVAL, "nbatch * n_cells exceeds 2^31 - 1");
    DBuf<double>& stage = h->tmp.f64[7];
    stage.reserve(n);
    VEM_HIP(hipMemcpyAsync(stage.p, nu, n * sizeof(double), hipMemcpyDefault, s));
    DBuf<int>& bad = h->tmp.i32[0];
    bad.reserve(1);
    fill_i32(s, 1, 0, bad);
    launch_check_cells(s, (int)n, stage.p, bad);  // every value positive and finite
    check_launch();
    h->tmp.ti.alloc(8);
    VEM_HIP(hipMemcpyAsync(h->tmp.ti.p, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    sync(h);
    VEM_REQUIRE(h->tmp.ti.p[0] == 0, VEM_EINVAL, "coefficient nu must be positive and finite in every cell");
    h->nu_batch.reserve(n);
    VEM_HIP(hipMemcpyAsync(h->nu_batch.p, stage.p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    h->nb_nu = nbatch;
  });
}

vem_status vem_set_rhs_batch(vem_handle h, int64_t nbatch, const double* f_qp, const double* pD_qp) {
  if (!h || !f_qp || nbatch < 1) return VEM_EINVAL;
  return guarded(h, [&] {
    require_disc(h);
    VEM_REQUIRE(h->bc == VEM_BC_PRESSURE, VEM_EINVAL, "batched right-hand sides take pressure boundary data");
    hipStream_t s = h->stream;
    const int64_t N = h->L.Nu + h->L.Np;
    const int64_t nqc = h->ntet * h->npts_cell, nqf = h->nbtri * h->npts_face;
    h->rhs_batch.reserve(nbatch * N);
    // each load goes through the handle's single right-hand side, which is then restored
    DBuf<double>& keep = h->tmp.f64[6];
    keep.reserve(N);
    launch_copy(s, N, h->rhs, keep);
    for (int64_t b = 0; b < nbatch; ++b) {
      set_loads(h, f_qp + b * nqc, pD_qp ? pD_qp + b * nqf : nullptr, nullptr);
      launch_copy(s, N, h->rhs, h->rhs_batch.p + b * N);
    }
    launch_copy(s, N, keep, h->rhs);
    check_launch();
    sync(h);
    h->nb_rhs = nbatch;
  });
}

vem_status vem_set_rhs_noalloc(vem_handle h, const double* f_qp, const double* pD_qp) {
  if (!h || !f_qp) return VEM_EINVAL;
  return guarded(h, [&] {
    require_disc(h);
    VEM_REQUIRE(h->bc == VEM_BC_PRESSURE, VEM_EINVAL, "flux boundary data: use vem_set_rhs_flux");
    VEM_REQUIRE(h->noalloc, VEM_EHIP, "no device scratch bound to this handle");
    const int64_t need = tet_sum_len(h);
    VEM_REQUIRE(need <= kNoAllocDoubles, VEM_ENOMEM,
                "vem_set_rhs_noalloc: the mesh needs " + std::to_string(need) +
                    " doubles of load scratch, more than its fixed " + std::to_string(kNoAllocDoubles) +
                    " (use vem_set_rhs)");
    // every entry the build reads is written by it first: nothing to clear
    set_loads(h, f_qp, pD_qp, nullptr, h->noalloc);
  });
}

vem_status vem_set_rhs_flux(vem_handle h, const double* f_qp, const double* u_qp) {
  if (!h || !f_qp || !u_qp) return VEM_EINVAL;
  return guarded(h, [&] {
    require_disc(h);
    VEM_REQUIRE(h->bc == VEM_BC_FLUX, VEM_EINVAL, "call vem_set_boundary(h, VEM_BC_FLUX) first");
    set_loads(h, f_qp, nullptr, u_qp);
  });
}

vem_status vem_apply(vem_handle h, const double* x, double* y) {
  if (!h || !x || !y) return VEM_EINVAL;
  return guarded(h, [&] {
    require_disc(h);
    ensure_k(h);
    launch_spmv(h->stream, h->Ks, x, y);
    check_launch();
  });
}

vem_status vem_export_csr(vem_handle h, int which, int32_t* rowptr, int32_t* col, double* val) {
  if (!h) return VEM_EINVAL;
  return guarded(h, [&] {
    require_disc(h);
    VEM_REQUIRE(which >= VEM_MAT_K && which <= VEM_MAT_REG_SCHWARZ, VEM_EINVAL, "unknown matrix");
    const bool face = which == VEM_MAT_REG_FACE, schw = which == VEM_MAT_REG_SCHWARZ;
    if (face || schw) {
      ensure_schwarz(h, h->sz.ready ? h->sz.gamma : h->gamma_A, false);
    } else {
      ensure_values(h, which == VEM_MAT_SCHUR, which == VEM_MAT_REG, false, h->gamma_A);
    }
    const bool lo_face = face && h->L.nint == 0;  // the lowest order's face system is A_gamma
    Csr* M = which == VEM_MAT_K       ? &h->K
             : which == VEM_MAT_SCHUR ? &h->S
             : which == VEM_MAT_REG   ? &h->A
             : schw                   ? &h->sz.Pc
             : lo_face                ? &h->A
                                      : &h->sz.Fc;
    const Sell* Ms = which == VEM_MAT_K       ? &h->Ks
                     : which == VEM_MAT_SCHUR ? &h->Ss
                     : which == VEM_MAT_REG   ? &h->As
                     : schw                   ? &h->sz.Ps
                     : lo_face                ? &h->As
                                              : &h->sz.Fs;
    hipStream_t s = h->stream;
    if (val) {
      if (schw || (face && !lo_face))
        schwarz_export(s, h->sz, face, *M);
      else
        sell_to_csr(s, *Ms, *M);
    }
    if (rowptr)
      VEM_HIP(hipMemcpyAsync(rowptr, M->rowptr.p, (M->rows + 1) * sizeof(int), hipMemcpyDefault, s));
    if (col) VEM_HIP(hipMemcpyAsync(col, M->col.p, M->nnz * sizeof(int), hipMemcpyDefault, s));
    if (val) VEM_HIP(hipMemcpyAsync(val, M->val.p, M->nnz * sizeof(double), hipMemcpyDefault, s));
    sync(h);
  });
}

vem_status vem_get_rhs(vem_handle h, double* b) {
  if (!h || !b) return VEM_EINVAL;
  return guarded(h, [&] {
    require_disc(h);
    const double* src = h->bc == VEM_BC_FLUX ? flux_rhs(h) : h->rhs.p;
    VEM_HIP(hipMemcpyAsync(b, src, (h->L.Nu + h->L.Np) * sizeof(double), hipMemcpyDefault, h->stream));
    sync(h);
  });
}

vem_status vem_get_geometry(vem_handle h, double* fa, double* fn, double* fc, double* cv, double* cc, double* cd) {
  if (!h) return VEM_EINVAL;
  return guarded(h, [&] {
    require_disc(h);
    hipStream_t s = h->stream;
    auto cp = [&](double* dst, const double* src, size_t n) {
      if (dst) VEM_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDefault, s));
    };
    cp(fa, h->f_area, h->nf);
    cp(fn, h->f_normal, 3 * (size_t)h->nf);
    cp(fc, h->f_cen, 3 * (size_t)h->nf);
    cp(cv, h->c_vol, h->nc);
    cp(cc, h->c_cen, 3 * (size_t)h->nc);
    cp(cd, h->c_diam, h->nc);
    sync(h);
  });
}

vem_status vem_time_kernel(vem_handle h, int which, int reps, double* avg_ms, double* bytes) {
  if (!h || !avg_ms || reps < 1) return VEM_EINVAL;
  return guarded(h, [&] {
    require_disc(h);
    VEM_REQUIRE(which >= VEM_KERNEL_SPMV && which <= VEM_KERNEL_CHEB_SCHUR32, VEM_EINVAL, "unknown kernel");
    const bool cheb = which == VEM_KERNEL_CHEB_SCHUR || which == VEM_KERNEL_CHEB_SCHUR32;
    const bool schwarz = which == VEM_KERNEL_CG_REG_SCHWARZ || which == VEM_KERNEL_CG_REG_SCHWARZ32;
    const bool pipe32 = which == VEM_KERNEL_CG_SCHUR32P || which == VEM_KERNEL_CG_REG32P;
    const bool f32 = pipe32 || which == VEM_KERNEL_CG_SCHUR32 || which == VEM_KERNEL_CG_REG32 ||
                     which == VEM_KERNEL_CHEB_SCHUR32;
    const bool schur = which == VEM_KERNEL_CG_SCHUR || which == VEM_KERNEL_CG_SCHUR32 ||
                       which == VEM_KERNEL_CG_SCHUR32P || cheb;
    ensure_values(h, which != VEM_KERNEL_SPMV && schur, which != VEM_KERNEL_SPMV && !schur, f32, h->gamma_A);
    if (schwarz) ensure_schwarz(h, h->gamma_A, which == VEM_KERNEL_CG_REG_SCHWARZ32);
    hipStream_t s = h->stream;
    ensure_workspace(h, std::max(1, h->ws_m));
    const int64_t Nu = h->L.Nu, Np = h->L.Np, N = Nu + Np;
    hipEvent_t e0, e1;
    VEM_HIP(hipEventCreate(&e0));
    VEM_HIP(hipEventCreate(&e1));
    double b = 0.0;
    double own_ms = -1.0;  // the Chebyshev products are timed launch by launch (their own time)
    try {
      if (which == VEM_KERNEL_SPMV) {
        launch_spmv(s, h->Ks, h->rhs, h->Vb);  // warm-up
        VEM_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) launch_spmv(s, h->Ks, h->rhs, h->Vb);
        VEM_HIP(hipEventRecord(e1, s));
        b = 12.0 * h->K.nnz + 8.0 * N + 8.0 * N;  // matrix, x once, y once
      } else if (cheb) {
        // one Chebyshev product kernel: reps products (plus the one initial scaling) averaged
        launch_fill(s, h->L.Np, 1.0, h->Vb);
        if (which == VEM_KERNEL_CHEB_SCHUR32) {
          PcgWork32 w{h->px32, (float*)h->pr.p, (float*)h->pz.p, (float*)h->ps.p, (float*)h->pp.p,
                      (float*)h->pw0.p, (float*)h->pw1.p, h->dSinv32};
          own_ms = time_cheb_products<float>(s, h->Ss, w, h->Vb, h->cheb.p, 1.0 / 400.0, reps, h->pcg);
          VEM_HIP(hipEventRecord(e0, s));
          VEM_HIP(hipEventRecord(e1, s));
          b = 8.0 * h->S.nnz + 4.0 * h->S.rows * 4.0;
        } else {
          PcgWork w{h->xw.p, h->pr, h->pz, h->ps, h->pp, h->pw0, h->pw1, h->dSinv};
          own_ms = time_cheb_products<double>(s, h->Ss, w, h->Vb, h->cheb.p, 1.0 / 400.0, reps, h->pcg);
          VEM_HIP(hipEventRecord(e0, s));
          VEM_HIP(hipEventRecord(e1, s));
          // S D^{-1} once; the iterate gathered; the previous iterate and b read; the next written
          b = 12.0 * h->S.nnz + 8.0 * h->S.rows * 4.0;
        }
      } else if (schwarz) {
        const DofLayout L = h->L;
        const Schwarz& X = h->sz;
        const Sell& F = schwarz_face_sell(X, h->As, L);
        const Csr& Fc = L.nint > 0 ? X.Fc : h->A;
        const SchwarzMesh m = schwarz_mesh(h);
        launch_fill(s, L.Nu, 1.0, h->Vb);  // a constant right-hand side
        const double nF = (double)X.nF;
        if (which == VEM_KERNEL_CG_REG_SCHWARZ32) {
          PcgWork32 w{h->px32, (float*)h->pr.p, (float*)h->pz.p, (float*)h->ps.p, (float*)h->pp.p, (float*)h->pw0.p,
                      (float*)h->pw1.p, nullptr};
          launch_schwarz_rhs<float>(s, m, L, X, nullptr, h->Vb, w.r);
          launch_scg_init<float>(s, X, w, h->pcg, 0.0, h->pcgpart);
          launch_scg_iter<float>(s, 0, F, X, w, h->pcg, h->pcgpart);
          launch_scg_iter<float>(s, 1, F, X, w, h->pcg, h->pcgpart);
          VEM_HIP(hipEventRecord(e0, s));
          for (int r = 0; r < reps; ++r) launch_scg_iter<float>(s, 2 + r, F, X, w, h->pcg, h->pcgpart);
          VEM_HIP(hipEventRecord(e1, s));
          // face blocks: one 4-byte index per block and two block offsets per face
          b = X.blocked ? 4.0 * (Fc.nnz + X.Pc.nnz) + 4.0 * (X.Fb.nblk + X.Pb.nblk) + 16.0 * (X.Fb.nf + 1) +
                              4.0 * nF * 13.0
                        : 8.0 * (Fc.nnz + X.Pc.nnz) + 4.0 * nF * 13.0;
        } else {
          PcgWork w{h->xw.p, h->pr, h->pz, h->ps, h->pp, h->pw0, h->pw1, nullptr};
          launch_schwarz_rhs<double>(s, m, L, X, nullptr, h->Vb, w.r);
          launch_scg_init<double>(s, X, w, h->pcg, 0.0, h->pcgpart);
          launch_scg_iter<double>(s, 0, F, X, w, h->pcg, h->pcgpart);
          launch_scg_iter<double>(s, 1, F, X, w, h->pcg, h->pcgpart);
          VEM_HIP(hipEventRecord(e0, s));
          for (int r = 0; r < reps; ++r) launch_scg_iter<double>(s, 2 + r, F, X, w, h->pcg, h->pcgpart);
          VEM_HIP(hipEventRecord(e1, s));
          // both matrices once; [product] z gathered, p and q read and written; [update] q gathered,
          // r, z and x read and written, p read: 13 vector accesses per row
          b = X.blocked ? 8.0 * (Fc.nnz + X.Pc.nnz) + 4.0 * (X.Fb.nblk + X.Pb.nblk) + 16.0 * (X.Fb.nf + 1) +
                              8.0 * nF * 13.0
                        : 12.0 * (Fc.nnz + X.Pc.nnz) + 8.0 * nF * 13.0;
        }
      } else {
        Sell& A = schur ? h->Ss : h->As;
        const Csr& C = schur ? h->S : h->A;
        const double* dinv = schur ? h->dSinv.p : h->dAinv.p;
        const float* dinv32 = schur ? h->dSinv32.p : h->dAinv32.p;
        // a constant right-hand side: never zero, whatever the loads are
        launch_fill(s, A.rows, 1.0, h->Vb);
        const double* rhs = h->Vb;
        PcgWork w{h->xw.p, h->pr, h->pz, h->ps, h->pp, h->pw0, h->pw1, dinv};
        PcgWork32 w32{h->px32, (float*)h->pr.p, (float*)h->pz.p, (float*)h->ps.p, (float*)h->pp.p,
                      (float*)h->pw0.p, (float*)h->pw1.p, dinv32};
        // tol = 0: the solve never stops, every timed launch does a full iteration
        if (pipe32) {
          launch_pcg_init32p(s, A, w32, rhs, h->pcg, 0.0, INT_MAX, h->pcgpart);
          launch_pcg_iter32p(s, 0, A, w32, h->pcg, h->pcgpart);
          launch_pcg_iter32p(s, 1, A, w32, h->pcg, h->pcgpart);
          VEM_HIP(hipEventRecord(e0, s));
          for (int r = 0; r < reps; ++r) launch_pcg_iter32p(s, 2 + r, A, w32, h->pcg, h->pcgpart);
          VEM_HIP(hipEventRecord(e1, s));
          // as the FP64 iteration below, with 4-byte values and vector elements
          b = 8.0 * C.nnz + 4.0 * C.rows * 13.0;
        } else if (f32) {
          launch_pcg_init32(s, A, w32, rhs, h->pcg, 0.0, INT_MAX, h->pcgpart);
          launch_pcg_iter32(s, 0, A, w32, h->pcg, h->pcgpart);
          launch_pcg_iter32(s, 1, A, w32, h->pcg, h->pcgpart);
          VEM_HIP(hipEventRecord(e0, s));
          for (int r = 0; r < reps; ++r) launch_pcg_iter32(s, 2 + r, A, w32, h->pcg, h->pcgpart);
          VEM_HIP(hipEventRecord(e1, s));
          // one classical CG iteration (two launches): FP32 values + int32 columns once; z and p
          // gathered, p and Ap written; x, r, Ap, p, D^{-1} read and x, r, z written (12 FP32 accesses per row)
          b = 8.0 * C.nnz + 4.0 * C.rows * 12.0;
        } else {
          launch_pcg_init(s, A, w, rhs, h->pcg, 0.0, INT_MAX, h->pcgpart);
          launch_pcg_iter(s, 0, A, w, h->pcg, h->pcgpart);
          launch_pcg_iter(s, 1, A, w, h->pcg, h->pcgpart);
          VEM_HIP(hipEventRecord(e0, s));
          for (int r = 0; r < reps; ++r) launch_pcg_iter(s, 2 + r, A, w, h->pcg, h->pcgpart);
          VEM_HIP(hipEventRecord(e1, s));
          // matrix once; w gathered; dinv, r, z, s, p, x read; z, s, p, x, r, w written
          b = 12.0 * C.nnz + 8.0 * C.rows * 13.0;
        }
      }
      check_launch();
      VEM_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      VEM_HIP(hipEventElapsedTime(&ms, e0, e1));
      VEM_HIP(hipMemcpyAsync(h->hpcg.p, h->pcg.p, sizeof(PcgState), hipMemcpyDeviceToHost, s));
      sync(h);
      VEM_REQUIRE(which == VEM_KERNEL_SPMV || h->hpcg.p->done == 0, VEM_EBREAKDOWN,
                  "inner CG stopped during the timing loop");
      *avg_ms = own_ms >= 0.0 ? own_ms : (double)ms / reps;
      if (bytes) *bytes = b;
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  });
}

}  // extern "C"

static vem_status solve_impl(vem_handle h, const vem_solve_opts* opts, const double* user_rhs, double* u, double* p,
                             vem_solve_info* info) {
  if (!h || !u || !p) return VEM_EINVAL;
  vem_status result = VEM_OK;
  vem_status st = guarded(h, [&] {
    require_disc(h);
    const double* rhs = user_rhs ? user_rhs : h->rhs.p;
    vem_solve_opts o;
    if (opts)
      o = *opts;
    else
      vem_solve_opts_default(&o);
    VEM_REQUIRE(o.restart >= 1 && o.restart <= kMaxRestart, VEM_EINVAL, "restart must be in 1..32");
    VEM_REQUIRE(o.tol > 0 && o.maxit >= 1, VEM_EINVAL, "tol must be > 0 and maxit >= 1");
    VEM_REQUIRE(o.precond >= VEM_PREC_SCHUR && o.precond <= VEM_PREC_NONE, VEM_EINVAL, "unknown preconditioner");
    VEM_REQUIRE(o.inner_tol > 0 && o.inner_maxit >= 1, VEM_EINVAL, "inner_tol must be > 0 and inner_maxit >= 1");
    VEM_REQUIRE(o.precision == VEM_FP64 || o.precision == VEM_MIXED, VEM_EINVAL, "unknown precision mode");
    VEM_REQUIRE(o.inner_form == VEM_INNER_PIPELINED || o.inner_form == VEM_INNER_CLASSICAL ||
                    o.inner_form == VEM_INNER_CHEBYSHEV,
                VEM_EINVAL, "unknown inner CG form");
    VEM_REQUIRE(o.inner_form != VEM_INNER_CHEBYSHEV || (o.inner_maxit <= 4096 && o.cheb_lo < 1.0), VEM_EINVAL,
                "Chebyshev inner form: inner_maxit (the degree) at most 4096 and cheb_lo below 1");
    VEM_REQUIRE(o.reg_inner == VEM_REG_JACOBI || o.reg_inner == VEM_REG_SCHWARZ, VEM_EINVAL,
                "unknown Block-Reg inner preconditioner");
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = h->stream;
    const int m = o.restart;
    const int64_t Nu = h->L.Nu, Np = h->L.Np, N = Nu + Np;
    const double gam = o.gamma > 0 ? o.gamma : h->gamma_default;
    // the Schwarz form asks for A_gamma's values itself where it needs them (the lowest order)
    const bool schwarz = o.precond == VEM_PREC_REG && o.reg_inner == VEM_REG_SCHWARZ;
    ensure_values(h, o.precond == VEM_PREC_SCHUR, o.precond == VEM_PREC_REG && !schwarz, o.precision == VEM_MIXED,
                  gam);
    if (schwarz) ensure_schwarz(h, gam, o.precision == VEM_MIXED);
    if (!user_rhs && h->bc == VEM_BC_FLUX) rhs = flux_rhs(h);
    ensure_workspace(h, m);
    double* V = h->Vb;
    double* Z = h->Zb;
    double* x = h->xw;
    double* dh = h->scal.p;                 // h = V^T w          (<= kMaxDots)
    double* dh2 = h->scal.p + kMaxDots;     // reorthogonalisation + ||w'||^2
    double* dn = h->scal.p + 2 * kMaxDots;  // ||r||^2
    double* dy = h->scal.p + 3 * kMaxDots;  // combination coefficients
    double* hb = h->hbuf.p;

    // the inner solves add their iterations to PcgState::total
    VEM_HIP(hipMemsetAsync(&h->pcg.p->total, 0, sizeof(int), s));
    // ||b||
    launch_dots(s, N, 1, rhs, N, rhs, h->partials, dn);
    check_launch();
    VEM_HIP(hipMemcpyAsync(hb, dn, sizeof(double), hipMemcpyDeviceToHost, s));
    sync(h);
    const double bnorm = std::sqrt(hb[0]);
    VEM_REQUIRE(std::isfinite(bnorm), VEM_ENAN, "right-hand side is not finite");

    if (o.use_x0) {
      VEM_HIP(hipMemcpyAsync(x, u, Nu * sizeof(double), hipMemcpyDeviceToDevice, s));
      VEM_HIP(hipMemcpyAsync(x + Nu, p, Np * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
      launch_fill(s, N, 0.0, x);
    }
    vem_solve_info inf{};
    if (bnorm == 0.0) {
      launch_fill(s, N, 0.0, x);
    }
    // r0 = b - K x0.  From x0 = 0 it is b itself, whose norm is known: no product, no second
    // synchronisation (dn already holds ||b||^2 for the first normalisation).
    double beta = bnorm;
    if (o.use_x0) {
      launch_residual(s, h->Ks, x, rhs, V, h->partials, dn);
      check_launch();
      VEM_HIP(hipMemcpyAsync(hb, dn, sizeof(double), hipMemcpyDeviceToHost, s));
      sync(h);
      beta = std::sqrt(hb[0]);
    } else {
      launch_copy(s, N, rhs, V);
      check_launch();
    }
    const double bref = bnorm > 0 ? bnorm : 1.0;
    int its = 0, restarts = 0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), yv(m);
    auto Hc = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
    bool nan_seen = false;
    while (beta / bref > o.tol && its < o.maxit && bnorm > 0) {
      // V0 = r / beta
      launch_scale_to(s, N, V, dn, V);
      std::fill(H.begin(), H.end(), 0.0);
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      int jend = 0;
      // One Arnoldi step, enqueued without waiting: everything the next step needs stays on
      // the device, so step j+1 is enqueued before the host reads step j's scalars and the
      // device never idles on the host's Givens rotations.  A step enqueued past the
      // convergence point is discarded (its outputs are never read).
      //   Classical Gram-Schmidt twice, in two passes over V: the first pass of step j also
      // finishes v_j, i.e. applies step j-1's second projection and normalisation to the w'
      // that step left in V[j].  The preconditioner of step j therefore takes that w' rather
      // than v_j; flexible GMRES allows any z_j, since K z_j = V H e_j holds by construction of
      // the orthogonalisation of K z_j, and w' differs from ||w'|| v_j by a rounding-level
      // component in span(V).
      auto enqueue_step = [&](int j) {
        double* vj = V + (size_t)j * N;
        double* zj = Z + (size_t)j * N;
        double* w = V + (size_t)(j + 1) * N;
        apply_prec(h, o, vj, zj);
        launch_spmv(s, h->Ks, zj, w);
        // h at scal[0], its correction at scal[kMaxDots], ||w||^2 between the passes at
        // scal[kMaxDots + j + 1]; the reductions also write them to the step's pinned host slot
        // (same offsets), so no copy is enqueued
        double* hc = h->hcol_dev + (size_t)j * kColSlot;
        if (j == 0)
          launch_dots(s, N, 1, V, N, w, h->partials, dh, hc);
        else
          launch_dots_fix(s, N, j + 1, V, N, dh2, w, h->partials, dh, hc);
        launch_update_dots(s, N, j + 1, V, N, dh, w, h->partials, dh2, hc + kMaxDots);
        check_launch();
        VEM_HIP(hipEventRecord(h->step_done[j & 1], s));
      };
      enqueue_step(0);
      for (int j = 0; j < m; ++j) {
        if (j + 1 < m && its + 1 < o.maxit) enqueue_step(j + 1);
        VEM_HIP(hipEventSynchronize(h->step_done[j & 1]));
        const double* col = h->hcol.p + (size_t)j * kColSlot;
        double hh = 0.0;
        for (int i = 0; i <= j; ++i) {
          Hc(i, j) = col[i] + col[kMaxDots + i];
          hh += col[kMaxDots + i] * col[kMaxDots + i];
        }
        // the norm the device divided by: ||w||^2 - |V^T w|^2 of the second pass
        const double hn2 = col[kMaxDots + j + 1] - hh;
        double hn = std::isfinite(hn2) ? std::sqrt(hn2 > 0.0 ? hn2 : 0.0) : hn2;
        Hc(j + 1, j) = hn;
        for (int i = 0; i <= j + 1; ++i)
          if (!std::isfinite(Hc(i, j))) nan_seen = true;
        if (nan_seen) break;
        for (int i = 0; i < j; ++i) {
          double t = cs[i] * Hc(i, j) + sn[i] * Hc(i + 1, j);
          Hc(i + 1, j) = -sn[i] * Hc(i, j) + cs[i] * Hc(i + 1, j);
          Hc(i, j) = t;
        }
        double den = std::hypot(Hc(j, j), Hc(j + 1, j));
        if (den == 0.0) {
          jend = j;
          break;
        }
        cs[j] = Hc(j, j) / den;
        sn[j] = Hc(j + 1, j) / den;
        Hc(j, j) = den;
        Hc(j + 1, j) = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        ++its;
        jend = j + 1;
        if (std::fabs(g[j + 1]) / bref <= o.tol || its >= o.maxit || hn == 0.0) break;
      }
      if (nan_seen) break;
      if (jend > 0) {
        for (int i = jend - 1; i >= 0; --i) {
          double t = g[i];
          for (int k = i + 1; k < jend; ++k) t -= Hc(i, k) * yv[k];
          yv[i] = t / Hc(i, i);
        }
        std::memcpy(hb + 3 * kMaxDots, yv.data(), jend * sizeof(double));
        VEM_HIP(hipMemcpyAsync(dy, hb + 3 * kMaxDots, jend * sizeof(double), hipMemcpyHostToDevice, s));
        launch_combine(s, N, jend, Z, N, dy, x);
      }
      ++restarts;
      launch_residual(s, h->Ks, x, rhs, V, h->partials, dn);
      check_launch();
      VEM_HIP(hipMemcpyAsync(hb, dn, sizeof(double), hipMemcpyDeviceToHost, s));
      sync(h);
      double nb = std::sqrt(hb[0]);
      if (!std::isfinite(nb)) {
        nan_seen = true;
        break;
      }
      if (jend == 0 && nb >= beta) {
        beta = nb;
        break;  // no progress possible (breakdown at the first step)
      }
      beta = nb;
    }
    VEM_REQUIRE(!nan_seen, VEM_ENAN, "NaN or Inf met in the Krylov iteration");
    if (h->bc == VEM_BC_FLUX) {
      // of the pressures that solve the system (they differ by the constant), the one with zero mean
      double* d = h->scal.p + 4 * kMaxDots;
      launch_dots(s, Np, 1, h->pw, Np, x + Nu, h->partials, d);
      launch_project(s, Np, x + Nu, h->n_p, d, 1.0 / h->np_wn, x + Nu);
      check_launch();
    }
    VEM_HIP(hipMemcpyAsync(u, x, Nu * sizeof(double), hipMemcpyDeviceToDevice, s));
    VEM_HIP(hipMemcpyAsync(p, x + Nu, Np * sizeof(double), hipMemcpyDeviceToDevice, s));
    VEM_HIP(hipMemcpyAsync(h->hpcg.p, h->pcg.p, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    sync(h);
    const int64_t inner = o.precond == VEM_PREC_NONE ? 0 : h->hpcg.p->total;
    auto t1 = std::chrono::steady_clock::now();
    inf.iterations = its;
    inf.restarts = restarts;
    inf.inner_iterations = inner;
    inf.relres = bnorm > 0 ? beta / bnorm : 0.0;
    inf.solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    result = (bnorm == 0.0 || inf.relres <= o.tol) ? VEM_OK : VEM_NOT_CONVERGED;
    inf.status = result;
    if (info) *info = inf;
  });
  return st != VEM_OK ? st : result;
}

extern "C" {

vem_status vem_solve(vem_handle h, const vem_solve_opts* opts, double* u, double* p, vem_solve_info* info) {
  return solve_impl(h, opts, nullptr, u, p, info);
}

vem_status vem_solve_rhs(vem_handle h, const vem_solve_opts* opts, const double* rhs, double* u, double* p,
                         vem_solve_info* info) {
  if (!h || !rhs) return VEM_EINVAL;
  // With flux data K is singular (the constant pressure spans its kernel) and its prescribed rows
  // fix boundary DOFs; a caller right-hand side is neither projected nor meaningful there.
  if (h->bc == VEM_BC_FLUX) {
    h->last_error = "vem_solve_rhs supports pressure boundary data only";
    return VEM_EINVAL;
  }
  return solve_impl(h, opts, rhs, u, p, info);
}

vem_status vem_solve_batch(vem_handle h, const vem_solve_opts* opts, int64_t nbatch, double* u, double* p,
                           vem_solve_info* info) {
  if (!h || !u || !p || nbatch < 1) return VEM_EINVAL;
  if (!h->has_disc || (h->nb_nu != 0 && h->nb_nu != nbatch) || (h->nb_rhs > 1 && h->nb_rhs != nbatch) ||
      (h->nb_nu == 0 && h->nb_rhs <= 1) || (h->nb_rhs > 0 && h->bc != VEM_BC_PRESSURE)) {
    h->last_error = "vem_solve_batch: set nbatch coefficient fields and/or nbatch right-hand sides first";
    return VEM_EINVAL;
  }
  const int64_t nc = h->nc, Nu = h->L.Nu, Np = h->L.Np, N = Nu + Np;
  // the handle's own coefficient is restored afterwards
  vem_status st = guarded(h, [&] {
    DBuf<double>& keep = h->tmp.f64[5];
    keep.reserve(nc);
    launch_copy(h->stream, nc, h->nu, keep);
    check_launch();
  });
  if (st != VEM_OK) return st;
  vem_status worst = VEM_OK;
  for (int64_t b = 0; b < nbatch && worst >= 0; ++b) {
    if (h->nb_nu > 0) {
      st = guarded(h, [&] {
        launch_copy(h->stream, nc, h->nu_batch.p + b * nc, h->nu);
        check_launch();
        invalidate_values(h);
      });
      if (st != VEM_OK) {
        worst = st;
        break;
      }
    }
    const double* rhs = h->nb_rhs > 1 ? h->rhs_batch.p + b * N : h->nb_rhs == 1 ? h->rhs_batch.p : nullptr;
    vem_solve_info inf{};
    st = solve_impl(h, opts, rhs, u + b * Nu, p + b * Np, &inf);
    if (info) info[b] = inf;
    if (st < 0)
      worst = st;
    else if (st > worst)
      worst = st;
  }
  // the handle's coefficient back in place, also after a failed system
  if (h->nb_nu > 0) {
    const std::string err = h->last_error;
    st = guarded(h, [&] {
      launch_copy(h->stream, nc, h->tmp.f64[5], h->nu);
      check_launch();
      invalidate_values(h);
      sync(h);
    });
    if (worst < 0) h->last_error = err;  // report the system's error, not the restore's
    if (st != VEM_OK && worst >= 0) return st;
  }
  return worst;
}

vem_status vem_coefficient_gradient(vem_handle h, const double* u, const double* lam, double* g) {
  if (!h || !u || !lam || !g) return VEM_EINVAL;
  // The gradient formula assumes every flux DOF is free (pressure data): with flux data the
  // prescribed DOFs would contribute terms that do not depend on the coefficient.
  if (h->bc == VEM_BC_FLUX) {
    h->last_error = "vem_coefficient_gradient supports pressure boundary data only";
    return VEM_EINVAL;
  }
  return guarded(h, [&] {
    require_disc(h);
    launch_coef_grad(h->stream, h->L, h->cptr, h->cface, h->csign, h->lmat_ptr, h->M1, h->nu, u, lam, g);
    check_launch();
  });
}

}  // extern "C"
