// Adjoint of the solve x = A^{-1} b with A = Q R (stored factors of the
// batched form): for an upstream gradient g = dL/dx,
//   lambda = A^{-T} g = Q (R^{-T} g),   dL/dA = -lambda x^T,   dL/db = lambda.
// One 1024-thread workgroup per matrix: the triangular solve R^T z = g is
// blocked by 32 (a dot product per column against the finished part of z, one
// wave per column, then the 32 x 32 triangle in one wave with readlane);
// lambda = Q z is accumulated block by block (one thread per row, four
// accumulators added in a fixed order) by the waves that are idle during each
// triangle; the rank-1 product is written column by column (coalesced), the
// columns split between the two halves of the workgroup.  HBM-bound on
// reading Q and R and writing dA.
#include "internal.h"
#include "../../include/cqr.h"

namespace cqr {
namespace {

template <typename T>
__device__ __forceinline__ T rlane(T x, int l);
template <>
__device__ __forceinline__ double rlane<double>(double x, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}
template <>
__device__ __forceinline__ float rlane<float>(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

template <typename T>
__device__ __forceinline__ T wsum(T x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

constexpr int kAdjNMax = 512;
constexpr int kAdjThreads = 1024;

struct AdjArgs {
  const int32_t* n;
  void* const* Q;
  const int32_t* ldq;
  void* const* R;
  const int32_t* ldr;
  void* const* x;
  void* const* g;
  void* const* dA;
  const int32_t* ldda;
  void* const* db;
};

template <typename T>
__global__ __launch_bounds__(kAdjThreads) void adjoint_kernel(AdjArgs a) {
  constexpr int NW = kAdjThreads / 64;
  __shared__ T sz[kAdjNMax];  // g, then z = R^{-T} g
  __shared__ T sx[kAdjNMax];
  __shared__ T sl[kAdjNMax];  // lambda
  const int m = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = a.n[m];
  const int ldq = a.ldq[m], ldr = a.ldr[m], ldda = a.ldda[m];
  if (n < 1 || n > kAdjNMax || ldq < n || ldr < n || ldda < n) return;
  const T* Q = (const T*)a.Q[m];
  const T* R = (const T*)a.R[m];
  const T* x = (const T*)a.x[m];
  const T* g = (const T*)a.g[m];
  T* dA = (T*)a.dA[m];
  T* db = (T*)a.db[m];
  if (!Q || !R || !x || !g || !dA || !db) return;
  for (int r = tid; r < n; r += kAdjThreads) {
    sz[r] = g[r];
    sx[r] = x[r];
  }
  __syncthreads();
  // R^T z = g, column block by column block.  While wave 0 solves the
  // diagonal triangle of block s, waves 8-15 (one row each) add the previous
  // block's terms of lambda = Q z, whose z entries are final: the stream
  // through Q runs under the latency of the substitution.
  const int lr = tid - kAdjThreads / 2;  // row of lambda owned by waves 8-15
  const bool lrow = lr >= 0 && lr < n;
  T l0 = T(0), l1 = T(0), l2 = T(0), l3 = T(0);
  auto lambda_block = [&](int c0, int c1) {  // columns c0 .. c1-1, c1 - c0 <= 32
    if (!lrow) return;
    const T* qr = Q + lr;
    T qv[32];
#pragma unroll
    for (int u = 0; u < 32; ++u) qv[u] = (c0 + u < c1) ? qr[(size_t)(c0 + u) * ldq] : T(0);
#pragma unroll
    for (int u = 0; u < 32; u += 4) {
      if (c0 + u < c1) l0 += qv[u] * sz[c0 + u];
      if (c0 + u + 1 < c1) l1 += qv[u + 1] * sz[c0 + u + 1];
      if (c0 + u + 2 < c1) l2 += qv[u + 2] * sz[c0 + u + 2];
      if (c0 + u + 3 < c1) l3 += qv[u + 3] * sz[c0 + u + 3];
    }
  };
  for (int s = 0; s < n; s += 32) {
    const int w = min(32, n - s);
    if (s > 0) {
      for (int i = wave; i < w; i += NW) {
        const T* rc = R + (size_t)(s + i) * ldr;
        T rv[kAdjNMax / 64];
#pragma unroll
        for (int u = 0; u < kAdjNMax / 64; ++u) {
          const int p = lane + 64 * u;
          rv[u] = (p < s) ? rc[p] : T(0);
        }
        T d = T(0);
#pragma unroll
        for (int u = 0; u < kAdjNMax / 64; ++u) {
          const int p = lane + 64 * u;
          if (p < s) d += rv[u] * sz[p];
        }
        d = wsum(d);
        if (lane == 0) sz[s + i] -= d;
      }
      __syncthreads();
    }
    if (wave == 0) {
      // Lane j holds column j of the diagonal block: rcol[p] = R(s + p, s + j).
      T rcol[32];
      const T* rc = R + (size_t)(s + lane) * ldr + s;
#pragma unroll
      for (int p = 0; p < 32; ++p) rcol[p] = (lane < w && p < w) ? rc[p] : T(0);
      T gj = (lane < w) ? sz[s + lane] : T(0);
#pragma unroll
      for (int p = 0; p < 32; ++p) {
        if (p < w) {
          const T zp = rlane(gj, p) / rlane(rcol[p], p);
          if (lane == p) gj = zp;
          else if (lane > p) gj -= rcol[p] * zp;
        }
      }
      if (lane < w) sz[s + lane] = gj;
    } else if (s > 0) {
      lambda_block(s - 32, s);
    }
    __syncthreads();
  }
  // The last block's terms; db = lambda.
  lambda_block(((n - 1) / 32) * 32, n);
  if (lrow) {
    const T lam = (l0 + l1) + (l2 + l3);
    sl[lr] = lam;
    db[lr] = lam;
  }
  __syncthreads();
  // dA = -lambda x^T: thread (r, h) writes row r of the columns c = h mod 2.
  {
    const int r = tid % kAdjNMax, h = tid / kAdjNMax;
    if (r < n) {
      const T lr = -sl[r];
      for (int c = h; c < n; c += 2) dA[(size_t)r + (size_t)c * ldda] = lr * sx[c];
    }
  }
}

}  // namespace
}  // namespace cqr

using namespace cqr;

extern "C" {

int cqr_batched_solve_backward(int64_t count, int dtype, const int32_t* n, void* const* Q, const int32_t* ldq,
                               void* const* R, const int32_t* ldr, void* const* x, void* const* g, void* const* dA,
                               const int32_t* ldda, void* const* db, void* stream) {
  if (count < 0 || count > INT32_MAX) return -1;
  if (dtype != CQR_F64 && dtype != CQR_F32) return -2;
  if (count == 0) return CQR_OK;
  if (!n) return -3;
  if (!Q) return -4;
  if (!ldq) return -5;
  if (!R) return -6;
  if (!ldr) return -7;
  if (!x) return -8;
  if (!g) return -9;
  if (!dA) return -10;
  if (!ldda) return -11;
  if (!db) return -12;
  hipStream_t st = (hipStream_t)stream;
  AdjArgs aa{n, Q, ldq, R, ldr, x, g, dA, ldda, db};
  const int slot = prof_begin(st);
  if (dtype == CQR_F64)
    hipLaunchKernelGGL(adjoint_kernel<double>, dim3((unsigned)count), dim3(kAdjThreads), 0, st, aa);
  else
    hipLaunchKernelGGL(adjoint_kernel<float>, dim3((unsigned)count), dim3(kAdjThreads), 0, st, aa);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return CQR_ERR_HIP_BASE - (int)e;
  prof_end(slot, ROLE_ADJOINT, st, 0.0, 0.0);
  return CQR_OK;
}

}  // extern "C"
