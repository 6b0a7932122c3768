// Sparse products of the truncated SVD (Table 1, the SpMM rows of Algorithms
// 1 and 2): C = A X and C = A^T X for a CSR matrix A and a dense block X of
// w columns (w = b for LancSVD, w = r for RandSVD).
//
// The paper runs both through cuSPARSE and measures the transposed product as
// its bottleneck.  Here A^T is kept explicitly as a second CSR matrix, built
// once on the device (cqr_csr_transpose), so both products are the same
// row-parallel gather: row i of C is the sum over the nonzeros (i, c) of
// a_ic times row c of X.  X is first copied into row-major order (rows of
// w padded to 16, 32 or 64 doubles), so each nonzero gathers one contiguous
// row of X (128 bytes at w = 16); TW = padded width lanes work on one row of
// C, lane j on column j, and the sum runs over the row's nonzeros in storage
// order, so results are reproducible bit for bit.  HBM-bound: per product
// the nonzeros (12 bytes each), the row pointers, one read of X and one write
// of C.
#include "internal.h"
#include "../../include/cqr.h"

namespace cqr {
namespace {

constexpr int kSpThreads = 256;

// Xr (rows x wp, row-major) = X (rows x w, column-major, ldx), zero padding.
// A block moves 64 rows through LDS: column-wise coalesced reads, row-wise
// coalesced writes.
__global__ void __launch_bounds__(256)
to_rowmajor_kernel(int64_t rows, int w, int wp, const double* __restrict__ X, int64_t ldx, double* __restrict__ Xr) {
  __shared__ double sT[64][65];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  for (int idx = tid; idx < 64 * wp; idx += 256) {
    const int i = idx % 64, j = idx / 64;
    const int64_t row = r0 + i;
    sT[j][i] = (row < rows && j < w) ? X[row + (int64_t)j * ldx] : 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < 64 * wp; idx += 256) {
    const int j = idx % wp, i = idx / wp;
    const int64_t row = r0 + i;
    if (row < rows) Xr[row * wp + j] = sT[j][i];
  }
}

// C (rows x w, ldc) = A Xr with A in CSR (rows x *), Xr row-major (* x TW).
// TW lanes per row of C; the row's column indices and values are loaded by
// the lanes together, TW at a time, and broadcast within the group.
template <int TW>
__global__ void __launch_bounds__(kSpThreads)
csr_spmm_kernel(int64_t rows, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                const double* __restrict__ val, const double* __restrict__ Xr, int w, double* __restrict__ C,
                int64_t ldc) {
  constexpr int RPB = kSpThreads / TW;
  const int tid = threadIdx.x;
  const int j = tid % TW;
  const int64_t row = (int64_t)blockIdx.x * RPB + tid / TW;
  const bool ok = row < rows;
  const int beg = ok ? rowptr[row] : 0;
  const int end = ok ? rowptr[row + 1] : 0;
  double acc0 = 0.0, acc1 = 0.0;
  for (int k0 = beg; k0 < end; k0 += TW) {
    const int kk = k0 + j;
    const int myc = kk < end ? col[kk] : 0;
    const double myv = kk < end ? val[kk] : 0.0;
    const int cnt = (end - k0) < TW ? (end - k0) : TW;
    int t = 0;
    for (; t + 1 < cnt; t += 2) {
      const int c0 = __shfl(myc, t, TW), c1 = __shfl(myc, t + 1, TW);
      const double v0 = __shfl(myv, t, TW), v1 = __shfl(myv, t + 1, TW);
      acc0 += v0 * Xr[(int64_t)c0 * TW + j];
      acc1 += v1 * Xr[(int64_t)c1 * TW + j];
    }
    if (t < cnt) {
      const int c0 = __shfl(myc, t, TW);
      const double v0 = __shfl(myv, t, TW);
      acc0 += v0 * Xr[(int64_t)c0 * TW + j];
    }
  }
  if (ok && j < w) C[row + (int64_t)j * ldc] = acc0 + acc1;
}

// ---------------------------------------------------------------- transpose
__global__ void fill_i32_kernel(int64_t n, int32_t* p) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void count_cols_kernel(int64_t nnz, const int32_t* __restrict__ col, int32_t* cnt) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[col[k]], 1);
}

// ptr[0] = 0, ptr[i + 1] = cnt[0] + ... + cnt[i] (one workgroup; each thread
// scans a contiguous chunk).  Also clears cnt (reused as the fill counters).
__global__ void __launch_bounds__(1024) scan_kernel(int64_t n, int32_t* cnt, int32_t* ptr) {
  __shared__ int64_t sPart[1024];
  const int tid = threadIdx.x;
  const int64_t chunk = (n + 1023) / 1024;
  const int64_t i0 = tid * chunk, i1 = (i0 + chunk < n) ? i0 + chunk : n;
  int64_t s = 0;
  for (int64_t i = i0; i < i1; ++i) s += cnt[i];
  sPart[tid] = s;
  __syncthreads();
  if (tid == 0) {
    int64_t acc = 0;
    for (int t = 0; t < 1024; ++t) {
      const int64_t v = sPart[t];
      sPart[t] = acc;
      acc += v;
    }
    ptr[0] = 0;
  }
  __syncthreads();
  int64_t acc = sPart[tid];
  for (int64_t i = i0; i < i1; ++i) {
    acc += cnt[i];
    ptr[i + 1] = (int32_t)acc;
    cnt[i] = 0;
  }
}

__global__ void scatter_kernel(int64_t m, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                               const double* __restrict__ val, const int32_t* __restrict__ tptr, int32_t* fill,
                               int32_t* tcol, double* tval) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      const int c = col[k];
      const int pos = tptr[c] + atomicAdd(&fill[c], 1);
      tcol[pos] = (int32_t)i;
      tval[pos] = val[k];
    }
  }
}

// Each row of A^T sorted by column (= row of A): a unique order, whatever
// order the atomics of the scatter gave.
__global__ void sort_rows_kernel(int64_t n, const int32_t* __restrict__ tptr, int32_t* tcol, double* tval) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    const int b = tptr[c], e = tptr[c + 1];
    for (int k = b + 1; k < e; ++k) {
      const int32_t key = tcol[k];
      const double v = tval[k];
      int p = k - 1;
      while (p >= b && tcol[p] > key) {
        tcol[p + 1] = tcol[p];
        tval[p + 1] = tval[p];
        --p;
      }
      tcol[p + 1] = key;
      tval[p + 1] = v;
    }
  }
}

int width_pad(int64_t w) { return w <= 16 ? 16 : (w <= 32 ? 32 : 64); }

hipError_t spmm_rows(int64_t rows, int64_t inner, const int32_t* rowptr, const int32_t* col, const double* val,
                     int64_t w, const double* X, int64_t ldx, double* C, int64_t ldc, double* xrm, int64_t nnz,
                     hipStream_t st) {
  for (int64_t j0 = 0; j0 < w; j0 += 64) {
    const int wc = (int)((w - j0) < 64 ? (w - j0) : 64);
    const int wp = width_pad(wc);
    hipLaunchKernelGGL(to_rowmajor_kernel, dim3((unsigned)((inner + 63) / 64)), dim3(256), 0, st, inner, wc, wp,
                       X + j0 * ldx, ldx, xrm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int slot = prof_begin(st);
    const int64_t rpb = kSpThreads / wp;
    const dim3 grid((unsigned)((rows + rpb - 1) / rpb));
    if (wp == 16)
      hipLaunchKernelGGL(csr_spmm_kernel<16>, grid, dim3(kSpThreads), 0, st, rows, rowptr, col, val, xrm, wc,
                         C + j0 * ldc, ldc);
    else if (wp == 32)
      hipLaunchKernelGGL(csr_spmm_kernel<32>, grid, dim3(kSpThreads), 0, st, rows, rowptr, col, val, xrm, wc,
                         C + j0 * ldc, ldc);
    else
      hipLaunchKernelGGL(csr_spmm_kernel<64>, grid, dim3(kSpThreads), 0, st, rows, rowptr, col, val, xrm, wc,
                         C + j0 * ldc, ldc);
    e = hipGetLastError();
    prof_end(slot, ROLE_SPMM, st, 2.0 * (double)nnz * wc,
             12.0 * (double)nnz + 4.0 * (double)(rows + 1) + 8.0 * (double)wc * (double)(rows + inner));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

size_t spmm_scratch_doubles(int64_t m, int64_t n) { return (size_t)(m > n ? m : n) * 64; }

hipError_t spmm(const SparseCsr& S, bool trans, int64_t w, const double* X, int64_t ldx, double* C, int64_t ldc,
                hipStream_t st) {
  if (trans) return spmm_rows(S.n, S.m, S.trowptr, S.tcol, S.tval, w, X, ldx, C, ldc, S.xrm, S.nnz, st);
  return spmm_rows(S.m, S.n, S.rowptr, S.col, S.val, w, X, ldx, C, ldc, S.xrm, S.nnz, st);
}

}  // namespace cqr

using namespace cqr;

extern "C" {

int cqr_csr_transpose_workspace_size(int64_t n, size_t* bytes) {
  if (n < 1) return -1;
  if (!bytes) return -2;
  *bytes = ((size_t)n * sizeof(int32_t) + 255) & ~(size_t)255;
  return CQR_OK;
}

int cqr_csr_transpose(int64_t m, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col, const double* val,
                      int32_t* trowptr, int32_t* tcol, double* tval, void* work, size_t work_bytes, void* stream) {
  if (m < 1) return -1;
  if (n < 1) return -2;
  if (nnz < 0 || nnz > INT32_MAX) return -3;
  if (!rowptr) return -4;
  if (!col && nnz > 0) return -5;
  if (!val && nnz > 0) return -6;
  if (!trowptr) return -7;
  if (!tcol && nnz > 0) return -8;
  if (!tval && nnz > 0) return -9;
  if (!work || work_bytes < (size_t)n * sizeof(int32_t)) return CQR_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  int32_t* cnt = (int32_t*)work;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096)), dim3(256), 0,
                     st, n, cnt);
  hipLaunchKernelGGL(count_cols_kernel, dim3(2048), dim3(256), 0, st, nnz, col, cnt);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, n, cnt, trowptr);
  hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((m + 255) / 256 < 4096 ? (m + 255) / 256 : 4096)), dim3(256), 0,
                     st, m, rowptr, col, val, trowptr, cnt, tcol, tval);
  hipLaunchKernelGGL(sort_rows_kernel, dim3((unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096)), dim3(256),
                     0, st, n, trowptr, tcol, tval);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? CQR_OK : CQR_ERR_HIP_BASE - (int)e;
}

int cqr_spmm_workspace_size(int64_t m, int64_t n, size_t* bytes) {
  if (m < 1) return -1;
  if (n < 1) return -2;
  if (!bytes) return -3;
  *bytes = spmm_scratch_doubles(m, n) * sizeof(double);
  return CQR_OK;
}

int cqr_spmm(int trans, int64_t m, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
             const double* val, int64_t w, const double* X, int64_t ldx, double* C, int64_t ldc, void* work,
             size_t work_bytes, void* stream) {
  if (trans != 0 && trans != 1) return -1;
  if (m < 1) return -2;
  if (n < 1) return -3;
  if (nnz < 0 || nnz > INT32_MAX) return -4;
  if (!rowptr) return -5;
  if (!col && nnz > 0) return -6;
  if (!val && nnz > 0) return -7;
  if (w < 1) return -8;
  const int64_t rows = trans ? n : m, inner = trans ? m : n;
  if (!X) return -9;
  if (ldx < inner) return -10;
  if (!C) return -11;
  if (ldc < rows) return -12;
  if (!work || work_bytes < spmm_scratch_doubles(m, n) * sizeof(double)) return CQR_ERR_WORKSPACE;
  SparseCsr S{m, n, nnz, rowptr, col, val, rowptr, col, val, (double*)work};
  const hipError_t e = spmm(S, trans != 0, w, X, ldx, C, ldc, (hipStream_t)stream);
  return e == hipSuccess ? CQR_OK : CQR_ERR_HIP_BASE - (int)e;
}

}  // extern "C"
