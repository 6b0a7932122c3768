// Breakdown fallback of CGS-CQR2 on the device: when the Cholesky factorisation
// of a block's Gram matrix breaks down (a pivot that is not > 0), Section 3 of
// the paper reverts that block to classical Gram-Schmidt with
// re-orthogonalisation (CGS2).  Here the failed block is restored from its
// saved input and redone one column at a time as Algorithm 5 with b = 1,
// against the s earlier basis columns P and the block's own finished columns:
//
//   for each column v = Q[:, c], basis X = [P, Q[:, 0:c]] (s + c columns):
//     pass t = 1, 2:  h_t = X^T v;  v -= X h_t;  l_t = ||v||_2;  v /= l_t
//     R[c, c] = l_2 l_1,  [H; R][0:s+c, c] = h_1 + h_2 l_1       (S11, S12)
//   A remainder of zero (or NaN) norm in either pass gives a zero column,
//   R[c, c] = 0 and the first pass's h_1 as its coefficients.
//
// One persistent launch does the whole block: a grid of workgroups that are
// all resident at once steps through the columns together, separated by grid
// barriers (an arrival counter in global memory; every wait is bounded).  Per
// pass: the dot products (one wave per basis column, fixed-order reduction),
// a barrier, the update of the workgroup's rows and its share of ||v||^2, a
// barrier, every workgroup summing the shares in the same order (so all take
// the same breakdown decision), the scaling of its rows, a barrier.
//
// The launch is gated on the status word the Cholesky kernels set: with no
// breakdown every workgroup exits at once, so the fallback costs one empty
// launch per block and the factorisation needs no host round trip (it can be
// captured in a hipGraph).  The last workgroup to finish clears the status
// word and the barrier counters, and records info and the block's flags.
#include "internal.h"
#include "../../include/cqr.h"

namespace cqr {
namespace {

constexpr int kFbThreads = 256;
constexpr int kFbRowsPerThread = 1;  // target rows per thread when choosing the grid

template <typename TP>
struct FbArgs {
  int64_t q, s, w;
  const TP* P;      // q x s basis (ldp), may be null when s == 0 (FP64, or the FP32 finished columns
                    // of the low-precision form)
  int64_t ldp;
  double* Q;        // q x w block (ldq), in place
  int64_t ldq;
  double* H;        // s x w projections (ldh), may be null when s == 0
  int64_t ldh;
  double* R;        // w x w triangle (ldr)
  int64_t ldr;
  const double* save;  // q x w input copy (ld ldsave), or null when the block is intact
  int64_t ldsave;
  int* status;         // gate: status[0] != 0 means a breakdown in this block
  int32_t* info;       // device, may be null: first fallback block (1-based), or CQR_INFO_WAIT_ABANDONED
  int32_t* flags;      // device, may be null: flags[blk]
  int blk;
  unsigned* ctr;       // [0] barrier arrivals, [1] finished workgroups, [2] abandoned-wait flag
  double* part;        // gridDim.x doubles
  double* hbuf;        // 4 (s + w) doubles: [column parity][pass][s + w]
  uint64_t wait_ticks; // bound of one barrier wait in 100 MHz ticks
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// x^T v over q rows for one wave: four accumulators per lane, combined in a
// fixed order, then the wave sum.
template <typename TX>
__device__ __forceinline__ double column_dot(const TX* __restrict__ x, const double* __restrict__ v, int64_t q,
                                             int lane) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t i = lane;
  for (; i + 192 < q; i += 256) {
    acc[0] += (double)x[i] * v[i];
    acc[1] += (double)x[i + 64] * v[i + 64];
    acc[2] += (double)x[i + 128] * v[i + 128];
    acc[3] += (double)x[i + 192] * v[i + 192];
  }
  for (int u = 0; i < q; i += 64, ++u) acc[u] += (double)x[i] * v[i];
  return wave_sum((acc[0] + acc[1]) + (acc[2] + acc[3]));
}

// Grid barrier number `epoch` (1, 2, ...): every workgroup adds one arrival;
// thread 0 waits until all gridDim.x * epoch arrivals are in (bounded).  Once
// any wait has been abandoned the result is void anyway, so later barriers do
// not wait at all: the launch then ends within about one wait bound.
template <typename TP>
__device__ void grid_barrier(const FbArgs<TP>& a, unsigned epoch) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(&a.ctr[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = epoch * gridDim.x;
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(&a.ctr[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(&a.ctr[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
      if (wall_clock64() - t0 > a.wait_ticks) {
        __hip_atomic_store(&a.ctr[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

template <typename TP>
__global__ void __launch_bounds__(kFbThreads) cgs2_fallback_kernel(FbArgs<TP> a) {
  if (a.status[0] == 0) return;
  __shared__ double sRed[kFbThreads / 64];
  __shared__ double sNorm;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t G = gridDim.x;
  const int64_t chunk = (a.q + G - 1) / G;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = (r0 + chunk < a.q) ? r0 + chunk : a.q;
  const int64_t sw = a.s + a.w;
  unsigned epoch = 0;

  // Restore the block and clear its outputs.
  if (a.save)
    for (int64_t c = 0; c < a.w; ++c)
      for (int64_t i = r0 + tid; i < r1; i += kFbThreads) a.Q[i + c * a.ldq] = a.save[i + c * a.ldsave];
  for (int64_t idx = (int64_t)blockIdx.x * kFbThreads + tid; idx < a.s * a.w; idx += G * kFbThreads)
    a.H[idx % a.s + (idx / a.s) * a.ldh] = 0.0;
  for (int64_t idx = (int64_t)blockIdx.x * kFbThreads + tid; idx < a.w * a.w; idx += G * kFbThreads)
    a.R[idx % a.w + (idx / a.w) * a.ldr] = 0.0;
  grid_barrier(a, ++epoch);

  bool anyzero = false;
  for (int64_t c = 0; c < a.w; ++c) {
    double* v = a.Q + c * a.ldq;
    const int64_t nb = a.s + c;
    double* h1 = a.hbuf + (c & 1) * 2 * sw;
    double* h2 = h1 + sw;
    double l1 = 0.0, l2 = 0.0;
    bool zero = false;
    for (int t = 0; t < 2 && !zero; ++t) {
      double* h = t ? h2 : h1;
      // h = X^T v: one wave per basis column, four accumulators per lane.
      for (int64_t j = (int64_t)blockIdx.x * (kFbThreads / 64) + wave; j < nb; j += G * (kFbThreads / 64)) {
        const double d = (j < a.s) ? column_dot(a.P + j * a.ldp, v, a.q, lane)
                                   : column_dot(a.Q + (j - a.s) * a.ldq, v, a.q, lane);
        if (lane == 0) h[j] = d;
      }
      grid_barrier(a, ++epoch);
      // v -= X h on this workgroup's rows, and its share of ||v||^2.
      double pn = 0.0;
      for (int64_t i = r0 + tid; i < r1; i += kFbThreads) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        int64_t j = 0;
        for (; j + 4 <= a.s; j += 4) {
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[u] += (double)a.P[i + (j + u) * a.ldp] * h[j + u];
        }
        for (; j < a.s; ++j) acc[0] += (double)a.P[i + j * a.ldp] * h[j];
        for (int64_t k = 0; k < c; ++k) acc[1] += a.Q[i + k * a.ldq] * h[a.s + k];
        const double nv = v[i] - ((acc[0] + acc[1]) + (acc[2] + acc[3]));
        v[i] = nv;
        pn += nv * nv;
      }
      pn = wave_sum(pn);
      if (lane == 0) sRed[wave] = pn;
      __syncthreads();
      if (tid == 0) a.part[blockIdx.x] = (sRed[0] + sRed[1]) + (sRed[2] + sRed[3]);
      grid_barrier(a, ++epoch);
      // ||v||^2: every workgroup sums the shares in the same order.
      if (wave == 0) {
        double sacc = 0.0;
        for (int64_t g = lane; g < G; g += 64) sacc += a.part[g];
        sacc = wave_sum(sacc);
        if (lane == 0) sNorm = sacc;
      }
      __syncthreads();
      const double nrm2 = sNorm;
      if (!(nrm2 > 0.0)) {
        zero = true;
        for (int64_t i = r0 + tid; i < r1; i += kFbThreads) v[i] = 0.0;
      } else {
        const double lt = sqrt(nrm2);
        if (t == 0)
          l1 = lt;
        else
          l2 = lt;
        const double inv = 1.0 / lt;
        for (int64_t i = r0 + tid; i < r1; i += kFbThreads) v[i] *= inv;
      }
      grid_barrier(a, ++epoch);
    }
    // Coefficients of column c (S12 with b = 1) and the diagonal (S11).
    for (int64_t idx = (int64_t)blockIdx.x * kFbThreads + tid; idx < nb; idx += G * kFbThreads) {
      const double val = zero ? h1[idx] : h1[idx] + h2[idx] * l1;
      if (idx < a.s)
        a.H[idx + c * a.ldh] = val;
      else
        a.R[(idx - a.s) + c * a.ldr] = val;
    }
    if (blockIdx.x == 0 && tid == 0) a.R[c + c * a.ldr] = zero ? 0.0 : l2 * l1;
    anyzero = anyzero || zero;
  }

  // The last workgroup to finish records the outcome and clears the words.
  __syncthreads();
  if (tid == 0) {
    const unsigned t = __hip_atomic_fetch_add(&a.ctr[1], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (t == (unsigned)G - 1u) {
      const bool abandoned = __hip_atomic_load(&a.ctr[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
      if (a.flags) a.flags[a.blk] |= CQR_FLAG_FALLBACK | (anyzero ? CQR_FLAG_ZERO_COL : 0);
      if (a.info) {
        if (abandoned)
          a.info[0] = CQR_INFO_WAIT_ABANDONED;
        else if (a.info[0] == 0)
          a.info[0] = a.blk + 1;
      }
      a.ctr[0] = 0u;
      a.ctr[1] = 0u;
      a.ctr[2] = 0u;
      a.status[1] = 0;
      a.status[0] = 0;
    }
  }
}

int g_fb_grid = 0;  // workgroups of the fallback kernel: one per CU, found once

// One 256-thread workgroup per CU, with a few hundred bytes of LDS and no
// register pressure, is always resident at once on an idle device, so the
// grid barriers never wait for a workgroup that cannot start.
int fb_max_grid() {
  if (g_fb_grid > 0) return g_fb_grid;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  g_fb_grid = cus;
  return g_fb_grid;
}

__global__ void force_breakdown_kernel(int* status, int blk) {
  if (status[0] == 0) {
    status[0] = 1;
    status[1] = blk;
  }
}

template <typename TP>
hipError_t launch_fallback(int64_t q, int64_t s, int64_t w, const TP* P, int64_t ldp, double* Q, int64_t ldq,
                           double* H, int64_t ldh, double* R, int64_t ldr, const double* save, int64_t ldsave,
                           int* status, int32_t* info, int32_t* flags, int blk, void* fbwork, hipStream_t st) {
  if (q <= 0 || w <= 0) return hipSuccess;
  int gmax = fb_max_grid();
  if (gmax <= 0) return hipErrorInvalidConfiguration;
  if (gmax > 1024) gmax = 1024;
  int64_t g = (q + kFbThreads * kFbRowsPerThread - 1) / (kFbThreads * kFbRowsPerThread);
  if (g > gmax) g = gmax;
  if (g < 1) g = 1;
  FbArgs<TP> a;
  a.q = q;
  a.s = s;
  a.w = w;
  a.P = P;
  a.ldp = ldp > 0 ? ldp : 1;
  a.Q = Q;
  a.ldq = ldq;
  a.H = H;
  a.ldh = ldh > 0 ? ldh : 1;
  a.R = R;
  a.ldr = ldr;
  a.save = save;
  a.ldsave = ldsave > 0 ? ldsave : 1;
  a.status = status;
  a.info = info;
  a.flags = flags;
  a.blk = blk;
  a.ctr = (unsigned*)fbwork;
  a.part = (double*)((char*)fbwork + 256);
  a.hbuf = (double*)((char*)fbwork + 256 + 1024 * sizeof(double));
  a.wait_ticks = wait_limit_ticks();
  const int slot = prof_begin(st);
  hipLaunchKernelGGL(cgs2_fallback_kernel<TP>, dim3((unsigned)g), dim3(kFbThreads), 0, st, a);
  const hipError_t e = hipGetLastError();
  prof_end(slot, ROLE_FALLBACK, st, 0.0, 0.0);
  return e;
}

}  // namespace

// Workspace of the fallback for a basis of up to sw = s + w columns:
// counters (256 bytes, first, so that their place does not depend on sw),
// the per-workgroup shares of ||v||^2 (1024 doubles), then the coefficient
// buffers (4 sw doubles).
size_t fallback_workspace_bytes(int64_t sw) {
  return 256 + 1024 * sizeof(double) + (((size_t)4 * (size_t)(sw > 0 ? sw : 1) * sizeof(double) + 255) & ~(size_t)255);
}

hipError_t cgs2_fallback(int64_t q, int64_t s, int64_t w, const double* P, int64_t ldp, double* Q, int64_t ldq,
                         double* H, int64_t ldh, double* R, int64_t ldr, const double* save, int64_t ldsave,
                         int* status, int32_t* info, int32_t* flags, int blk, void* fbwork, hipStream_t st) {
  return launch_fallback<double>(q, s, w, P, ldp, Q, ldq, H, ldh, R, ldr, save, ldsave, status, info, flags, blk,
                                 fbwork, st);
}

hipError_t cgs2_fallback_f32basis(int64_t q, int64_t s, int64_t w, const float* P, int64_t ldp, double* Q,
                                  int64_t ldq, double* H, int64_t ldh, double* R, int64_t ldr, const double* save,
                                  int64_t ldsave, int* status, int32_t* info, int32_t* flags, int blk, void* fbwork,
                                  hipStream_t st) {
  return launch_fallback<float>(q, s, w, P, ldp, Q, ldq, H, ldh, R, ldr, save, ldsave, status, info, flags, blk,
                                fbwork, st);
}

hipError_t force_breakdown(int* status, int blk, hipStream_t st) {
  hipLaunchKernelGGL(force_breakdown_kernel, dim3(1), dim3(1), 0, st, status, blk);
  return hipGetLastError();
}

}  // namespace cqr
