// Small dense kernels: the b x b Cholesky factorisation with the inverse of
// its factor (Table 1 POTRF, run on the GPU instead of the host), block
// copies, and the two kernels of the triangular solve.
#include "internal.h"

namespace cqr {
namespace {

// One workgroup of 16 x 16 threads (4 waves, one per SIMD) factors W (b x b,
// b <= 16 TS) as L L^T and inverts L.  Thread (ty, tx) = (tid / 16, tid % 16)
// keeps the TS x TS register tile of rows ty*TS.. and columns tx*TS.. .
//
// Factorisation, right-looking, one barrier per column k: the owners of
// column k publish its current values; every thread then takes the pivot
// d = W(k,k), forms l = sqrt(d), scales the column by 1/l and applies the
// rank-1 update to its tile.  A pivot that is not > 0 (NaN included) marks a
// breakdown; the kernel still runs to the end and reports it in status.
// L is then parked in LDS and the same registers hold X = L^{-1}, built
// right-looking from X = I with one barrier per k: row k of X is scaled by
// 1/L(k,k) and L(i,k) times it is subtracted from every row i > k.
// Published columns/rows are double-buffered in LDS by the parity of k.
template <int TS>
__global__ void __launch_bounds__(256)
chol_inv_kernel(int b, const double* __restrict__ W, int64_t ldw, double* __restrict__ LT, double* __restrict__ XT,
                int* status, int code, int blk) {
  constexpr int TG = 16, NB = TG * TS;
  if (status[0] != 0) return;
  __shared__ double colbuf[2][NB];
  __shared__ double rowbuf[2][NB];
  __shared__ double sL[NB][NB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x, ty = tid / TG, tx = tid % TG;
  if (tid == 0) bad = 0;
  double w[TS][TS];
#pragma unroll
  for (int r = 0; r < TS; ++r)
#pragma unroll
    for (int c = 0; c < TS; ++c) {
      const int i = ty * TS + r, j = tx * TS + c;
      w[r][c] = (i < b && j < b) ? W[i + (int64_t)j * ldw] : (i == j ? 1.0 : 0.0);
    }
  __syncthreads();

  for (int kb = 0; kb < TG && kb * TS < b; ++kb) {
#pragma unroll
    for (int kk = 0; kk < TS; ++kk) {
      const int k = kb * TS + kk;
      const int buf = k & 1;
      if (tx == kb) {
#pragma unroll
        for (int r = 0; r < TS; ++r) colbuf[buf][ty * TS + r] = w[r][kk];
      }
      __syncthreads();
      const double d = colbuf[buf][k];
      if (tid == 0 && k < b && !(d > 0.0)) bad = 1;
      const double l = sqrt(d);
      const double rl = 1.0 / l;
      // Column entries of rows/columns <= k enter the update as exact zeros,
      // which leaves those tile entries unchanged without per-element branches.
      double lim[TS], ljm[TS];
#pragma unroll
      for (int r = 0; r < TS; ++r) lim[r] = (ty * TS + r > k) ? colbuf[buf][ty * TS + r] * rl : 0.0;
#pragma unroll
      for (int c = 0; c < TS; ++c) ljm[c] = (tx * TS + c > k) ? colbuf[buf][tx * TS + c] * rl : 0.0;
#pragma unroll
      for (int r = 0; r < TS; ++r)
#pragma unroll
        for (int c = 0; c < TS; ++c) w[r][c] -= lim[r] * ljm[c];
      if (tx == kb) {
#pragma unroll
        for (int r = 0; r < TS; ++r) {
          const int i = ty * TS + r;
          w[r][kk] = (i > k) ? lim[r] : ((i == k) ? l : w[r][kk]);
        }
      }
    }
  }
  // Park L (lower part; zero above) in LDS and write L^T out.
#pragma unroll
  for (int r = 0; r < TS; ++r)
#pragma unroll
    for (int c = 0; c < TS; ++c) {
      const int i = ty * TS + r, j = tx * TS + c;
      const double v = (i >= j) ? w[r][c] : 0.0;
      sL[i][j] = v;
      if (i < b && j < b) LT[j + (int64_t)i * b] = v;  // LT(j, i) = L(i, j)
    }
  // The same registers now hold X, starting from I.
#pragma unroll
  for (int r = 0; r < TS; ++r)
#pragma unroll
    for (int c = 0; c < TS; ++c) w[r][c] = (ty * TS + r == tx * TS + c) ? 1.0 : 0.0;
  __syncthreads();

  for (int kb = 0; kb < TG && kb * TS < b; ++kb) {
#pragma unroll
    for (int kk = 0; kk < TS; ++kk) {
      const int k = kb * TS + kk;
      const int buf = k & 1;
      if (ty == kb) {
#pragma unroll
        for (int c = 0; c < TS; ++c) rowbuf[buf][tx * TS + c] = w[kk][c];
      }
      __syncthreads();
      const double rl = 1.0 / sL[k][k];
      double xk[TS];
#pragma unroll
      for (int c = 0; c < TS; ++c) xk[c] = rowbuf[buf][tx * TS + c] * rl;
#pragma unroll
      for (int r = 0; r < TS; ++r) {
        const int i = ty * TS + r;
        const double lik = (i > k) ? sL[i][k] : 0.0;
#pragma unroll
        for (int c = 0; c < TS; ++c) w[r][c] -= lik * xk[c];
      }
      if (ty == kb) {
#pragma unroll
        for (int c = 0; c < TS; ++c) w[kk][c] = xk[c];
      }
    }
  }

#pragma unroll
  for (int r = 0; r < TS; ++r)
#pragma unroll
    for (int c = 0; c < TS; ++c) {
      const int i = ty * TS + r, j = tx * TS + c;
      if (i < b && j < b) XT[j + (int64_t)i * b] = (i >= j) ? w[r][c] : 0.0;  // XT(j, i) = X(i, j)
    }
  __syncthreads();
  if (tid == 0 && bad) {
    status[1] = blk;
    status[0] = code;
  }
}

__global__ void __launch_bounds__(256)
copy_kernel(int64_t rows, int64_t cols, const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
            int64_t ldd, const int* __restrict__ gate) {
  if (gate != nullptr && *gate != 0) return;
  const int64_t total = rows * cols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx % rows, j = idx / rows;
    dst[i + j * ldd] = src[i + j * lds];
  }
}

__global__ void __launch_bounds__(256)
zero_kernel(int64_t rows, int64_t cols, double* __restrict__ X, int64_t ldx) {
  const int64_t total = rows * cols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx % rows, j = idx / rows;
    X[i + j * ldx] = 0.0;
  }
}

// y = Q^T x for square Q (n x n): one wave per column, fixed-order reduction.
__global__ void __launch_bounds__(256)
gemv_t_kernel(int64_t n, const double* __restrict__ Q, int64_t ldq, const double* __restrict__ x,
              double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  const double* q = Q + j * ldq;
  double acc = 0.0;
  for (int64_t i = lane; i < n; i += 64) acc += q[i] * x[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) y[j] = acc;
}

constexpr int kTrsvNB = 64;

// Back substitution on the diagonal block R[i0:i0+nb, i0:i0+nb] of upper R:
// y[i0:i0+nb] := R_blk^{-1} y[i0:i0+nb].  One 64-thread workgroup.
__global__ void __launch_bounds__(kTrsvNB)
trsv_diag_kernel(int64_t i0, int nb, const double* __restrict__ R, int64_t ldr, double* __restrict__ y) {
  __shared__ double sR[kTrsvNB][kTrsvNB + 1];
  __shared__ double xs;
  const int t = threadIdx.x;
  for (int c = 0; c < nb; ++c)
    if (t < nb) sR[t][c] = R[(i0 + t) + (i0 + c) * ldr];
  double v = (t < nb) ? y[i0 + t] : 0.0;
  __syncthreads();
  for (int i = nb - 1; i >= 0; --i) {
    if (t == i) {
      v = v / sR[i][i];
      xs = v;
    }
    __syncthreads();
    if (t < i) v -= sR[t][i] * xs;
    __syncthreads();
  }
  if (t < nb) y[i0 + t] = v;
}

// y[0:i0] -= R[0:i0, i0:i0+nb] y[i0:i0+nb].
__global__ void __launch_bounds__(256)
trsv_update_kernel(int64_t i0, int nb, const double* __restrict__ R, int64_t ldr, double* __restrict__ y) {
  __shared__ double xs[kTrsvNB];
  if (threadIdx.x < nb) xs[threadIdx.x] = y[i0 + threadIdx.x];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= i0) return;
  double acc = 0.0;
  for (int c = 0; c < nb; ++c) acc += R[r + (i0 + c) * ldr] * xs[c];
  y[r] -= acc;
}

unsigned grid_for(int64_t total) {
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  return (unsigned)blocks;
}

}  // namespace

hipError_t chol_inv(int b, const double* W, int64_t ldw, double* LT, double* XT, int* status, int code, int blk,
                    hipStream_t s) {
  if (b < 1 || b > 128) return hipErrorInvalidValue;
  const double bb = (double)b;
  const int slot = prof_begin(s);
  if (b <= 16)
    hipLaunchKernelGGL(chol_inv_kernel<1>, dim3(1), dim3(256), 0, s, b, W, ldw, LT, XT, status, code, blk);
  else if (b <= 32)
    hipLaunchKernelGGL(chol_inv_kernel<2>, dim3(1), dim3(256), 0, s, b, W, ldw, LT, XT, status, code, blk);
  else if (b <= 64)
    hipLaunchKernelGGL(chol_inv_kernel<4>, dim3(1), dim3(256), 0, s, b, W, ldw, LT, XT, status, code, blk);
  else
    hipLaunchKernelGGL(chol_inv_kernel<8>, dim3(1), dim3(256), 0, s, b, W, ldw, LT, XT, status, code, blk);
  hipError_t e = hipGetLastError();
  prof_end(slot, ROLE_CHOL, s, bb * bb * bb / 3.0, 8.0 * 3.0 * bb * bb);
  return e;
}

hipError_t copy_matrix(int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst, int64_t ldd,
                       const int* gate, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const int slot = prof_begin(s);
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, s, rows, cols, src, lds, dst, ldd, gate);
  hipError_t e = hipGetLastError();
  prof_end(slot, ROLE_COPY, s, 0.0, 16.0 * (double)rows * cols);
  return e;
}

hipError_t zero_matrix(int64_t rows, int64_t cols, double* X, int64_t ldx, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, s, rows, cols, X, ldx);
  return hipGetLastError();
}

hipError_t gemv_t(int64_t n, const double* Q, int64_t ldq, const double* x, double* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int slot = prof_begin(s);
  hipLaunchKernelGGL(gemv_t_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, Q, ldq, x, y);
  hipError_t e = hipGetLastError();
  prof_end(slot, ROLE_GEMV, s, 2.0 * (double)n * n, 8.0 * ((double)n * n + 2.0 * n));
  return e;
}

hipError_t trsv_upper(int64_t n, const double* R, int64_t ldr, double* y, hipStream_t s) {
  for (int64_t i0 = ((n - 1) / kTrsvNB) * kTrsvNB; i0 >= 0 && n > 0; i0 -= kTrsvNB) {
    const int nb = (int)((n - i0) < kTrsvNB ? (n - i0) : kTrsvNB);
    int slot = prof_begin(s);
    hipLaunchKernelGGL(trsv_diag_kernel, dim3(1), dim3(kTrsvNB), 0, s, i0, nb, R, ldr, y);
    hipError_t e = hipGetLastError();
    prof_end(slot, ROLE_TRSV_DIAG, s, (double)nb * nb, 8.0 * (double)nb * nb / 2.0);
    if (e != hipSuccess) return e;
    if (i0 > 0) {
      slot = prof_begin(s);
      hipLaunchKernelGGL(trsv_update_kernel, dim3((unsigned)((i0 + 255) / 256)), dim3(256), 0, s, i0, nb, R, ldr, y);
      e = hipGetLastError();
      prof_end(slot, ROLE_TRSV_UPD, s, 2.0 * (double)i0 * nb, 8.0 * (double)i0 * nb);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace cqr
