// SELL-64 (sliced ELLPACK) copies of the assembled CSR matrices.
//
// A slice is 64 consecutive rows, one wavefront: the slice is padded to its
// longest row and stored column-major, so entry k of the 64 rows is one
// contiguous 512-byte load of values and a 256-byte load of column indices.
// A thread owns a row; its loads do not depend on a row pointer and are
// independent of each other, which keeps many loads in flight per wave.
// Padding entries carry value 0 and the row's own column; a matrix of short rows may have every
// slice padded to its longest row (a fixed entry count per row).  The CSR pattern
// is built first; the value kernels then write straight into the SELL slots
// (entry k of row r at slice_ptr[r/64] + r%64 + 64k: coalesced across a
// wave), and src[] maps every slot back to its CSR entry (-1 for padding)
// for the CSR export.  Entries of a row keep their CSR order, so a row's sum
// is formed in the same order as a sequential CSR product.
#include "vem_internal.h"

namespace vem {
namespace {

// slice lengths; *max_len (zeroed before) receives the longest, one atomic per wavefront
__global__ void k_sell_len(int64_t rows, int64_t nslices, const int* __restrict__ rowptr, int* slice_len,
                           int64_t* slice_sz, int* max_len) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int m = 0;
  if (s < nslices) {
    int64_t r0 = s * 64, r1 = r0 + 64 < rows ? r0 + 64 : rows;
    for (int64_t r = r0; r < r1; ++r) {
      int l = rowptr[r + 1] - rowptr[r];
      m = l > m ? l : m;
    }
    slice_len[s] = m;
    slice_sz[s] = (int64_t)m * 64;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const int mo = __shfl_xor(m, o, 64);
    m = mo > m ? mo : m;
  }
  if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(max_len, m);
}

__global__ void k_sell_fill(int64_t rows, const int* __restrict__ rowptr, const int* __restrict__ col,
                            const int64_t* __restrict__ slice_ptr, const int* __restrict__ slice_len, int* scol,
                            int* src, double* sval) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t nrow_pad = ((rows + 63) / 64) * 64;
  if (r >= nrow_pad) return;
  int64_t s = r >> 6;
  int lane = (int)(r & 63);
  int64_t base = slice_ptr[s] + lane;
  int len = slice_len[s];
  int b = 0, e = 0;
  if (r < rows) {
    b = rowptr[r];
    e = rowptr[r + 1];
  }
  for (int k = 0; k < len; ++k) {
    int64_t o = base + (int64_t)k * 64;
    if (b + k < e) {
      scol[o] = col[b + k];
      src[o] = b + k;
    } else {
      scol[o] = r < rows ? (int)r : 0;
      src[o] = -1;
      sval[o] = 0.0;  // padding: the value kernels write only the real entries
    }
  }
}

// Every slice padded to one length: slice_len[s] = len and slice_ptr[s] = 64 len s (s <= nslices).
__global__ void k_sell_uniform(int64_t nslices, int len, int* __restrict__ slice_len, int64_t* __restrict__ ptr) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s > nslices) return;
  if (s < nslices) slice_len[s] = len;
  ptr[s] = s * 64 * len;
}

// CSR values from the SELL slots (for the export)
__global__ void k_sell_to_csr(int64_t n, const int* __restrict__ src, const double* __restrict__ sval,
                              double* __restrict__ val) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int j = src[i];
  if (j >= 0) val[j] = sval[i];
}

// CSR positions of the diagonal entries -> their SELL slots, in place
__global__ void k_sell_diag(int64_t rows, const int* __restrict__ rowptr, const int* __restrict__ slice_ptr,
                            int* diag) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  diag[r] = slice_ptr[r >> 6] + (int)(r & 63) + 64 * (diag[r] - rowptr[r]);
}

__global__ void k_narrow64(int64_t n, const int64_t* __restrict__ in, int* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (int)in[i];
}

inline int grid256(int64_t n) { return (int)((n + 255) / 256); }

// rows of at most this many entries may be padded to one length per matrix
constexpr int kSellFixedMax = 8;

}  // namespace

void build_sells(hipStream_t s, Scratch& tmp, const Csr* const* A, Sell* const* S, int count) {
  VEM_REQUIRE(count >= 0 && count <= 3, VEM_EINVAL, "at most three SELL builds at once");
  int64_t maxsl = 1;
  for (int m = 0; m < count; ++m) maxsl = std::max<int64_t>(maxsl, (A[m]->rows + 63) / 64);
  scan_reserve(tmp, maxsl);
  DBuf<int>& mlen = tmp.i32[0];
  mlen.reserve(3);
  VEM_HIP(hipMemsetAsync(mlen.p, 0, 3 * sizeof(int), s));
  tmp.ti.alloc(8);
  for (int m = 0; m < count; ++m) {
    Sell& B = *S[m];
    B.rows = A[m]->rows;
    B.nslices = (B.rows + 63) / 64;
    B.slice_len.alloc(B.nslices);
    DBuf<int64_t>& sz = tmp.i64[2 * m];
    DBuf<int64_t>& ptr = tmp.i64[2 * m + 1];
    sz.reserve(B.nslices + 1);
    ptr.reserve(B.nslices + 1);
    k_sell_len<<<grid256(B.nslices), 256, 0, s>>>(B.rows, B.nslices, A[m]->rowptr, B.slice_len, sz, mlen.p + m);
    VEM_HIP(hipGetLastError());
    scan_i64_async(s, tmp, sz, B.nslices, ptr, m);
  }
  VEM_HIP(hipMemcpyAsync(tmp.ti.p, mlen.p, count * sizeof(int), hipMemcpyDeviceToHost, s));
  VEM_HIP(hipStreamSynchronize(s));
  // Short rows: where padding every slice to the longest adds at most 1/16 of the slots, it is done,
  // and the products take a fixed number of entries per row with no per-slice masks (the 64^3 cube's
  // S: 7 per row, 0.9% more slots).
  int64_t totals[3];
  for (int m = 0; m < count; ++m) {
    Sell& B = *S[m];
    B.max_len = tmp.ti.p[m];
    totals[m] = tmp.tot.p[m];
    const int64_t even = B.nslices * 64 * (int64_t)B.max_len;
    B.fixed_len = 0;
    if (B.max_len > 0 && B.max_len <= kSellFixedMax && even <= totals[m] + totals[m] / 16) {
      B.fixed_len = B.max_len;
      totals[m] = even;
      k_sell_uniform<<<grid256(B.nslices + 1), 256, 0, s>>>(B.nslices, B.max_len, B.slice_len, tmp.i64[2 * m + 1]);
      VEM_HIP(hipGetLastError());
    }
  }
  for (int m = 0; m < count; ++m) {
    Sell& B = *S[m];
    const int64_t total = totals[m];
    VEM_REQUIRE(total < INT32_MAX, VEM_ENOMEM, "padded matrix exceeds 2^31-1 entries");
    DBuf<int64_t>& ptr = tmp.i64[2 * m + 1];
    B.nnz = total;
    B.slice_ptr.alloc(B.nslices + 1);
    k_narrow64<<<grid256(B.nslices + 1), 256, 0, s>>>(B.nslices + 1, ptr, B.slice_ptr);
    B.col.alloc(total);
    B.src.alloc(total);
    B.val.alloc(total);
    const int64_t nrow_pad = B.nslices * 64;
    k_sell_fill<<<grid256(nrow_pad), 256, 0, s>>>(B.rows, A[m]->rowptr, A[m]->col, ptr, B.slice_len, B.col, B.src,
                                                   B.val);
    VEM_HIP(hipGetLastError());
  }
}

void sell_to_csr(hipStream_t s, const Sell& S, Csr& A) {
  if (S.nnz > 0) k_sell_to_csr<<<grid256(S.nnz), 256, 0, s>>>(S.nnz, S.src, S.val, A.val);
}

void sell_diag_slots(hipStream_t s, int64_t ndiag, const Csr& A, const Sell& S, int* diag) {
  VEM_REQUIRE(ndiag >= 0 && ndiag <= A.rows, VEM_EINVAL, "more diagonal entries than rows");
  if (ndiag > 0) k_sell_diag<<<grid256(ndiag), 256, 0, s>>>(ndiag, A.rowptr, S.slice_ptr, diag);
}

}  // namespace vem
