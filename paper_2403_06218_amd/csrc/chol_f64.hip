// Small dense kernels: the b x b Cholesky factorisation with the inverse of
// its factor (Table 1 POTRF, run on the GPU instead of the host), block
// copies, and the matrix-vector product Q^T b of the solve.
#include "internal.h"
#include "wave_chol.h"

namespace cqr {
namespace {

typedef double chol_d4 __attribute__((ext_vector_type(4)));
typedef float chol_f4 __attribute__((ext_vector_type(4)));

// The 16 x 16 x 4 MFMA of the compute type: both take A(l mod 16, l / 16) and
// B(l / 16, l mod 16) from lane l; they differ in where the result lands.
template <typename T>
struct CholMf;
template <>
struct CholMf<double> {
  using V = chol_d4;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // Row of accumulator element v in lane group g = lane / 16 (column lane % 16).
  static __device__ __forceinline__ int crow(int g, int v) { return g + 4 * v; }
};
template <>
struct CholMf<float> {
  using V = chol_f4;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int crow(int g, int v) { return 4 * g + v; }
};

constexpr int kCB = 128;       // largest block width
constexpr int kCLD = kCB + 1;  // LDS row stride (odd: column walks are conflict-free)

// One workgroup (8 waves) factors W (b x b, b <= 128) as L L^T and inverts L,
// in the arithmetic of T (FP64, or FP32 for the low-precision form, whose
// factors carry BF16/FP8 rounding anyway; input and outputs are FP64 either
// way), blocked by panels of 16 columns, with the whole matrix held once in LDS:
// the lower triangle (with the diagonal) holds L, the strict upper triangle
// holds X^T for X = L^{-1}, and sD the diagonal of X (1 / L_ii).  Rows and
// columns b .. 16 ceil(b/16) - 1 are padded with the identity.  Only the lower
// triangle of W is read.
//
// Panel p (columns c0 = 16p .. c0+15), left-looking, in two phases:
//   1. wave 0 factors the diagonal tile, which already holds every earlier
//      panel's update, in registers (row broadcasts) and forms its inverse
//      X_pp: the serial part of the step.  Meanwhile waves 1-7 take one task
//      each (there are at most 7): the tiles below it, A(t, p) -= L(t, 0:p)
//      L(p, 0:p)^T, the next diagonal tile's update from panels 0 .. p-1, and
//      the tiles of block row p-1 of X = L^{-1}: X_i,0:i = -X_ii (L_i,0:i
//      X_0:i,0:i) (all MFMA); then they write out L's panel p-1 and X's block
//      row p-2, both final.
//   2. the rows below take L = A X_pp^T (MFMA); the wave that formed L(p+1, p)
//      gives the next diagonal tile its update from panel p.
// The last block row of X follows the loop.  A pivot that is not > 0 (NaN
// included) marks a breakdown; the kernel runs to the end and reports it in
// status.
template <typename T>
__global__ void __launch_bounds__(512)
chol_inv_kernel(int b, const double* __restrict__ W, int64_t ldw, double* __restrict__ LT, double* __restrict__ XT,
                int64_t ldo, int* status, int code, int blk) {
  constexpr int NT = 512;
  using M = CholMf<T>;
  using V = typename M::V;
  __shared__ T sA[kCB * kCLD];
  __shared__ T sD[kCB];
  __shared__ int bad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int nb = (b + 15) & ~15, P = nb >> 4;
  if (tid == 0) bad = 0;
  // Thread t loads row t % 128 of columns t / 128, +4, +8, ... on and below
  // the diagonal: all of its loads are issued before the first LDS store, so
  // their latencies overlap.
  const int ri = tid & (kCB - 1), rj = tid >> 7;
  {
    double v[kCB / 4];
#pragma unroll
    for (int u = 0; u < kCB / 4; ++u) {
      const int j = rj + 4 * u;
      v[u] = (ri < b && j <= ri) ? W[ri + (int64_t)j * ldw] : (ri == j ? 1.0 : 0.0);
    }
    // W is always readable: its loads are issued before the status test.
    if (status[0] != 0) return;
#pragma unroll
    for (int u = 0; u < kCB / 4; ++u) {
      const int j = rj + 4 * u;
      if (ri < nb && j <= ri) sA[ri * kCLD + j] = (T)v[u];
    }
  }
  __syncthreads();

  // A(t, u) -= L(t, k0:k1) L(u, k0:k1)^T over whole panels, with four
  // independent accumulators (k mod 16) to shorten the dependent chain.
  auto tile_update = [&](int t, int u, int k0, int k1) {
    V acc[4] = {V{}, V{}, V{}, V{}};
    for (int kb = k0; kb < k1; kb += 16) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        acc[q] = M::mma(sA[(16 * t + li) * kCLD + kb + 4 * q + lg], sA[(16 * u + li) * kCLD + kb + 4 * q + lg], acc[q]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
      sA[(16 * t + M::crow(lg, v)) * kCLD + 16 * u + li] -= (acc[0][v] + acc[1][v]) + (acc[2][v] + acc[3][v]);
  };
  // Tile jt of block row i of X (one wave): T = L[r0:r0+16, 0:r0] X[0:r0, jt]
  // (X lower: the sum starts at the diagonal tile), then X(i, jt) = -X_ii T,
  // stored transposed above the diagonal.  T stays in registers: element v of
  // the product's accumulator is row crow(lg, v) of T, which the second
  // product takes as the B operand of its step v (any k order shared by A and
  // B gives the same product).
  auto inverse_tile = [&](int i, int jt) {
    const int r0 = 16 * i;
    V acc[4] = {V{}, V{}, V{}, V{}};
    const int j = 16 * jt + li;
    for (int k0 = 16 * jt; k0 < r0; k0 += 16) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + 4 * q + lg;
        const T bx = (k > j) ? sA[j * kCLD + k] : ((k == j) ? sD[k] : T(0));
        acc[q] = M::mma(sA[(r0 + li) * kCLD + k], bx, acc[q]);
      }
    }
    V tv;
#pragma unroll
    for (int v = 0; v < 4; ++v) tv[v] = (acc[0][v] + acc[1][v]) + (acc[2][v] + acc[3][v]);
    V x = V{};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = M::crow(lg, v);
      const T ax = (li > k) ? sA[(r0 + k) * kCLD + r0 + li] : ((li == k) ? sD[r0 + k] : T(0));
      x = M::mma(ax, tv[v], x);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) sA[(16 * jt + li) * kCLD + r0 + M::crow(lg, v)] = -x[v];
  };

  // Output rows LT(j, :) for the 16-row panel jp (L's column panel jp, final
  // once that panel's rows below are formed) and output columns XT(:, i)
  // for X's block row ip (final once its off-diagonal tiles are formed), by
  // threads t0 .. t0 + nt - 1.  Column i of LT holds L(i, 0:i), column i of
  // XT holds X(i, 0:i); the rest is zero.
  auto store_lt_panel = [&](int jp, int t0, int nt) {
    for (int e = tid - t0; e < 16 * b; e += nt) {
      const int j = 16 * jp + (e & 15), i = e >> 4;
      if (j < b) LT[j + (int64_t)i * ldo] = (i >= j) ? (double)sA[i * kCLD + j] : 0.0;
    }
  };
  auto store_xt_row = [&](int ip, int t0, int nt) {
    for (int e = tid - t0; e < 16 * kCB; e += nt) {
      const int j = e & (kCB - 1), i = 16 * ip + (e >> 7);
      if (i < b && j < b)
        XT[j + (int64_t)i * ldo] = (i > j) ? (double)sA[j * kCLD + i] : ((i == j) ? (double)sD[i] : 0.0);
    }
  };

  for (int p = 0; p < P; ++p) {
    const int c0 = 16 * p;
    if (wave == 0) {
      // Lane i < 16 holds row i of the diagonal block.
      T a[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) a[j] = (lane < 16 && j <= lane) ? sA[(c0 + lane) * kCLD + c0 + j] : T(0);
      // The factor and X_pp = L_pp^{-1} (row i: linv_i times row i of
      // U^{-1}, formed during the factorisation), X stored transposed above
      // the diagonal.
      T lii, linv, y[16];
      const bool ok = wave_chol_inv<T, 16>(a, y, lii, linv, lane);
      if (lane == 0 && !ok) bad = 1;
      if (lane < 16) {
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (j < lane) {
            sA[(c0 + lane) * kCLD + c0 + j] = a[j];
            sA[(c0 + j) * kCLD + c0 + lane] = y[j] * linv;
          }
        sA[(c0 + lane) * kCLD + c0 + lane] = lii;
        sD[c0 + lane] = linv;
      }
    } else {
      // Tasks of this step, one per wave 1..7 (at most 7 exist): tiles t =
      // p+1 .. P-1 of the panel, then the next diagonal tile's update from
      // panels 0 .. p-1, then the tiles jt = 0 .. p-2 of X's block row p-1.
      const int task = wave - 1;
      const int ncol = (p > 0) ? P - 1 - p : 0;
      const int ndiag = (p > 0 && p + 1 < P) ? 1 : 0;
      if (task < ncol) tile_update(p + 1 + task, p, 0, c0);
      else if (task < ncol + ndiag) tile_update(p + 1, p + 1, 0, c0);
      else if (p >= 2 && task - ncol - ndiag < p - 1) inverse_tile(p - 1, task - ncol - ndiag);
      // L's panel p-1 and X's block row p-2 are final.
      if (p >= 1) store_lt_panel(p - 1, 64, NT - 64);
      if (p >= 2) store_xt_row(p - 2, 64, NT - 64);
    }
    __syncthreads();
    for (int t = p + 1 + wave; t < P; t += NT / 64) {
      V acc = V{};
#pragma unroll
      for (int kk = 0; kk < 16; kk += 4) {
        const int k = kk + lg;
        // B(k, j) = X_pp(j, k) with j = li.
        const T bx = (li > k) ? sA[(c0 + k) * kCLD + c0 + li] : ((li == k) ? sD[c0 + k] : T(0));
        acc = M::mma(sA[(16 * t + li) * kCLD + c0 + k], bx, acc);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) sA[(16 * t + M::crow(lg, v)) * kCLD + c0 + li] = acc[v];
      // This wave formed L(p+1, p): the next diagonal tile's update from panel
      // p (its own LDS writes above are ordered before these reads).
      if (t == p + 1) tile_update(p + 1, p + 1, c0, c0 + 16);
    }
    __syncthreads();
  }
  // The last block row of X.
  if (P >= 2)
    for (int jt = wave; jt < P - 1; jt += NT / 64) inverse_tile(P - 1, jt);
  __syncthreads();

  // What the loop has not written: L's last panel and X's last two block rows.
  store_lt_panel(P - 1, 0, NT);
  if (P >= 2) store_xt_row(P - 2, 0, NT);
  store_xt_row(P - 1, 0, NT);
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

unsigned grid_for(int64_t total) {
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  return (unsigned)blocks;
}

}  // namespace

// The same contract for b <= 16 in one wave, registers only: lane i < 16
// holds row i of W, factors it and forms row i of X = L^{-1} with
// wave_chol_inv, and writes column i of LT and of XT.
__global__ void __launch_bounds__(64)
chol_inv16_kernel(int b, const double* __restrict__ W, int64_t ldw, double* __restrict__ LT, double* __restrict__ XT,
                  int64_t ldo, int* status, int code, int blk) {
  if (status[0] != 0) return;
  const int lane = threadIdx.x;
  double a[16];
#pragma unroll
  for (int j = 0; j < 16; ++j)
    a[j] = (lane < b && j <= lane) ? W[lane + (int64_t)j * ldw] : ((lane == j) ? 1.0 : 0.0);
  double lii, linv, y[16];
  const bool ok = wave_chol_inv<double, 16>(a, y, lii, linv, lane);
  // LT(j, i) = L(i, j) and XT(j, i) = X(i, j) = linv_i (U^{-1})_ij.
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    if (lane < b && j < b) {
      LT[j + (int64_t)lane * ldo] = (j < lane) ? a[j] : ((j == lane) ? lii : 0.0);
      XT[j + (int64_t)lane * ldo] = (j < lane) ? y[j] * linv : ((j == lane) ? linv : 0.0);
    }
  }
  if (lane == 0 && !ok) {
    status[1] = blk;
    status[0] = code;
  }
}

static hipError_t chol_inv_ld(int b, const double* W, int64_t ldw, double* LT, double* XT, int64_t ldo, int* status,
                       int code, int blk, bool f32, hipStream_t s) {
  if (b < 1 || b > kCB) return hipErrorInvalidValue;
  const double bb = (double)b;
  const int slot = prof_begin(s);
  if (b <= 16)
    hipLaunchKernelGGL(chol_inv16_kernel, dim3(1), dim3(64), 0, s, b, W, ldw, LT, XT, ldo, status, code, blk);
  else if (f32)
    hipLaunchKernelGGL(chol_inv_kernel<float>, dim3(1), dim3(512), 0, s, b, W, ldw, LT, XT, ldo, status, code, blk);
  else
    hipLaunchKernelGGL(chol_inv_kernel<double>, dim3(1), dim3(512), 0, s, b, W, ldw, LT, XT, ldo, status, code, blk);
  hipError_t e = hipGetLastError();
  prof_end(slot, ROLE_CHOL, s, bb * bb * bb / 3.0, 8.0 * 3.0 * bb * bb);
  return e;
}

hipError_t chol_inv(int b, const double* W, int64_t ldw, double* LT, double* XT, int* status, int code, int blk,
                    hipStream_t s, bool f32) {
  return chol_inv_ld(b, W, ldw, LT, XT, b, status, code, blk, f32, s);
}

// 2 x 2 block form for kCB < b <= 2 kCB, with b1 = kCB and b2 = b - kCB:
//   L11 L11^T = W11;  U12 = L21^T = X11 W12;  S = W22 - U12^T U12;  L22 L22^T = S;
//   X21^T = -X11^T U12 X22^T.
// Writes LT = [L11^T U12; 0 L22^T] and XT = [X11^T X21^T; 0 X22^T] (ld b).
// W's trailing block is overwritten by S; tmp holds b1 x b2 doubles.  With f32
// the two diagonal factorisations and the four products take FP32 arithmetic
// (FP64 data throughout).
hipError_t chol_inv_wide(int b, double* W, int64_t ldw, double* LT, double* XT, double* tmp, int* status, int code,
                         int blk, hipStream_t s, bool f32, bool lower_zero) {
  if (b <= kCB) return chol_inv(b, W, ldw, LT, XT, status, code, blk, s, f32);
  if (b > 2 * kCB) return hipErrorInvalidValue;
  const int b1 = kCB, b2 = b - kCB;
  const double d1 = b1, d2 = b2;
  hipError_t e;
  double* W12 = W + (int64_t)b1 * ldw;
  double* W22 = W12 + b1;
  double* U12 = LT + (int64_t)b1 * b;   // LT[0:b1, b1:b]
  double* X12 = XT + (int64_t)b1 * b;   // XT[0:b1, b1:b] = X21^T
  if ((e = chol_inv_ld(b1, W, ldw, LT, XT, b, status, code, blk, f32, s)) != hipSuccess) return e;
  // U12 = X11 W12 = (XT11)^T W12.
  if ((e = gemm_tn(ROLE_CHOL, b1, b2, b1, 1.0, XT, b, W12, ldw, 0.0, U12, b, nullptr, 0, status, s,
                   d1 * d1 * d2, f32)) != hipSuccess)
    return e;
  // S = W22 - U12^T U12 (in place).
  if ((e = gemm_tn(ROLE_CHOL, b2, b2, b1, -1.0, U12, b, U12, b, 1.0, W22, ldw, nullptr, 0, status, s,
                   2.0 * d1 * d2 * d2, f32)) != hipSuccess)
    return e;
  if ((e = chol_inv_ld(b2, W22, ldw, LT + b1 + (int64_t)b1 * b, XT + b1 + (int64_t)b1 * b, b, status, code, blk,
                       f32, s)) != hipSuccess)
    return e;
  // X21^T = -(XT11 U12) XT22.
  if ((e = gemm_nn(ROLE_CHOL, b1, b2, b1, 1.0, XT, b, U12, b, 0.0, tmp, b1, status, s, d1 * d1 * d2, f32)) !=
      hipSuccess)
    return e;
  if ((e = gemm_nn(ROLE_CHOL, b1, b2, b2, -1.0, tmp, b1, XT + b1 + (int64_t)b1 * b, b, 0.0, X12, b, status, s,
                   2.0 * d1 * d2 * d2, f32)) != hipSuccess)
    return e;
  // Strictly lower blocks of LT and XT (nothing else writes them, so a
  // caller whose buffers start zero need not clear them again).
  if (lower_zero) return hipSuccess;
  if ((e = zero_matrix(b2, b1, LT + b1, b, s)) != hipSuccess) return e;
  return zero_matrix(b2, b1, XT + b1, b, s);
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


}  // namespace cqr
