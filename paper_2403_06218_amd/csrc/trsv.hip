// Back substitution R x = c for an upper triangular R (n x n, FP64 or FP32
// entries, FP64 arithmetic), the last step of the solve x = R^{-1} Q^T b.
//
// Rows are cut into 64-row blocks.  Block I needs the finished x_J of every
// block J > I:  x_I = R_II^{-1} (c_I - sum_{J > I} R_IJ x_J).  Two launches:
//
//   trsv_inv_kernel       the inverses R_II^{-1} of all diagonal blocks at
//                         once (independent; one wave per block), FP64;
//   trsv_lookback_kernel  the whole substitution in one launch: one workgroup
//                         per row block, which adds R_IJ x_J for each J as
//                         soon as block J has published x_J, then multiplies
//                         by R_II^{-1} and publishes x_I.
//
// Ordering and progress.  A workgroup takes a ticket t from a global counter
// and owns block I = nblk - 1 - t, so the blocks it waits for are owned by
// workgroups that took smaller tickets, i.e. that are already running: the
// chain always advances whatever order the hardware dispatches workgroups in.
// Blocks finish strictly from the last to the first; a single counter `done`
// holds how many have finished (release store by the finishing workgroup,
// relaxed polling plus an acquire fence by the waiting ones, agent scope, so
// the x values cross XCDs through memory).  Both counters only grow: launch
// number k of a sequence passes base = k * nblk, and the inverse launch
// clears them at the start of a sequence.  Every wait is bounded (in time, on
// the device's constant-rate clock): past the bound the workgroup sets an
// error word, carries on and publishes NaN for its block (so that every block
// that depends on it is NaN too), so every workgroup exits.
#include "internal.h"
#include "wave_chol.h"

namespace cqr {
namespace {

constexpr int kTB = 64;                   // rows per block
constexpr int kTThreads = 256;            // lookback workgroup: 4 waves x 16 columns of each block

template <typename TR>
__global__ void __launch_bounds__(kTB)
trsv_inv_kernel(int64_t n, const TR* __restrict__ R, int64_t ldr, double* __restrict__ Dinv,
                unsigned* __restrict__ ctr) {
  __shared__ double sR[kTB][kTB + 1];
  __shared__ double sInv[kTB];
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kTB;
  const int nb = (int)((n - r0) < kTB ? (n - r0) : kTB);
  if (blockIdx.x == 0 && t < 3) ctr[t] = 0u;
  // Lane t loads row t; rows and columns past nb are the identity.
#pragma unroll 8
  for (int c = 0; c < kTB; ++c)
    sR[t][c] = (t < nb && c < nb) ? ((c >= t) ? (double)R[(r0 + t) + (r0 + c) * ldr] : 0.0) : (t == c ? 1.0 : 0.0);
  __syncthreads();
  sInv[t] = 1.0 / sR[t][t];
  __syncthreads();
  // Lane j forms column j of the inverse: X(i, j) for i = j, j-1, ..., 0
  // (X(i, j) = 0 for i > j), every lane reading the same row of R.
  double x[kTB];
#pragma unroll
  for (int i = kTB - 1; i >= 0; --i) {
    double s = (i == t) ? 1.0 : 0.0;
#pragma unroll
    for (int k = i + 1; k < kTB; ++k) s -= sR[i][k] * x[k];
    x[i] = (i <= t) ? s * sInv[i] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kTB; ++i) sR[i][t] = x[i];
  __syncthreads();
  // Column-major 64 x 64 per block, written one column per step (coalesced).
  double* D = Dinv + (int64_t)blockIdx.x * kTB * kTB;
#pragma unroll 8
  for (int j = 0; j < kTB; ++j) D[t + kTB * j] = sR[t][j];
}

template <typename TR>
__global__ void __launch_bounds__(kTThreads)
trsv_lookback_kernel(int64_t n, const TR* __restrict__ R, int64_t ldr, const double* __restrict__ Dinv,
                     double* y, unsigned* ctr, unsigned base, uint64_t wait_ticks) {
  __shared__ unsigned sTicket;
  __shared__ int sGaveUp;
  __shared__ double sPart[kTThreads / 64][kTB];
  __shared__ double sV[kTB];
  __shared__ unsigned sDone[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const unsigned nblk = (unsigned)((n + kTB - 1) / kTB);
  if (tid == 0) {
    sTicket = atomicAdd(&ctr[0], 1u);
    sGaveUp = 0;
  }
  __syncthreads();
  const unsigned tk = sTicket - base;
  // Tickets past this launch's range cannot occur while launches of one
  // sequence are stream-ordered and pass consecutive bases; report and stop.
  if (tk >= nblk) {
    if (tid == 0) __hip_atomic_store(&ctr[2], 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const int I = (int)(nblk - 1u - tk);
  const int64_t r0 = (int64_t)I * kTB;
  const int64_t row = r0 + lane;
  const bool rowok = row < n;
  // This thread's share of R_II^{-1} (row `lane`, columns 16 wave .. +16) and c_I.
  const double* D = Dinv + (int64_t)I * kTB * kTB;
  double dv[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) dv[c] = D[lane + kTB * (16 * wave + c)];
  const double cI = (wave == 0 && rowok) ? y[row] : 0.0;

  // Off-diagonal part: lane = row of block I, wave = 16 of the 64 columns of
  // each block J; the R tile of the next J is loaded before waiting on it.
  TR rt[16];
  auto load_tile = [&](int J) {
    const int64_t c0 = (int64_t)J * kTB + 16 * wave;
#pragma unroll
    for (int c = 0; c < 16; ++c) rt[c] = (c0 + c < n) ? R[row + (c0 + c) * ldr] : TR(0);
  };
  double acc = 0.0;
  int next = (int)nblk - 1;
  if (next > I) load_tile(next);
  // Wave 0 polls (one request per wave), takes the acquire fence and hands
  // the count it saw to the other waves through LDS behind a barrier; the
  // slot alternates so that a fast wave 0 never overwrites a count that a
  // slower wave has yet to read.
  const uint64_t t0 = wall_clock64();
  int par = 0;
  while (next > I) {
    // Block `next` is finished once done - base >= nblk - next.
    const unsigned want = nblk - (unsigned)next;
    if (wave == 0) {
      unsigned d = __builtin_amdgcn_readfirstlane(
          __hip_atomic_load(&ctr[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - base);
      bool late = false;
      while (d < want) {
        if (wall_clock64() - t0 > wait_ticks) {
          late = true;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
        d = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&ctr[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - base);
      }
      if (late) {
        if (lane == 0) {
          __hip_atomic_store(&ctr[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          sGaveUp = 1;
        }
        d = want;
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (lane == 0) sDone[par] = d;
    }
    __syncthreads();
    const unsigned d = sDone[par];
    par ^= 1;
    // Blocks nblk - d .. nblk - 1 are finished; take all that are due.
    int lo = (int)nblk - (int)(d > nblk ? nblk : d);
    if (lo < I + 1) lo = I + 1;
    for (int J = next; J >= lo; --J) {
      const int64_t xi = (int64_t)J * kTB + 16 * wave + (lane & 15);
      const double xv = (xi < n) ? y[xi] : 0.0;
      TR cur[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) cur[c] = rt[c];
      if (J - 1 > I) load_tile(J - 1);
#pragma unroll
      for (int c = 0; c < 16; ++c) acc += (double)cur[c] * row_bcast(xv, c);  // xv repeats every 16 lanes
    }
    next = lo - 1;
  }

  // v = c_I - sum, then x_I = R_II^{-1} v; partial sums combined in a fixed order.
  sPart[wave][lane] = acc;
  __syncthreads();
  if (wave == 0) sV[lane] = cI - ((sPart[0][lane] + sPart[1][lane]) + (sPart[2][lane] + sPart[3][lane]));
  __syncthreads();
  double px = 0.0;
#pragma unroll
  for (int c = 0; c < 16; ++c) px += dv[c] * sV[16 * wave + c];
  sPart[wave][lane] = px;
  __syncthreads();
  if (wave == 0 && rowok)
    y[row] = sGaveUp ? __builtin_nan("") : (sPart[0][lane] + sPart[1][lane]) + (sPart[2][lane] + sPart[3][lane]);
  __syncthreads();
  if (tid == 0) __hip_atomic_store(&ctr[1], base + nblk - (unsigned)I, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

size_t trsv_workspace_bytes(int64_t n) {
  const int64_t nblk = (n + kTB - 1) / kTB;
  return (((size_t)(nblk > 0 ? nblk : 1) * kTB * kTB * sizeof(double) + 255) & ~(size_t)255) + 256;
}

int64_t trsv_blocks(int64_t n) { return (n + kTB - 1) / kTB; }

hipError_t trsv_prepare(int64_t n, bool f32, const void* R, int64_t ldr, void* work, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nblk = trsv_blocks(n);
  double* Dinv = (double*)work;
  unsigned* ctr = (unsigned*)((char*)work + trsv_workspace_bytes(n) - 256);
  const int slot = prof_begin(s);
  if (f32)
    hipLaunchKernelGGL(trsv_inv_kernel<float>, dim3((unsigned)nblk), dim3(kTB), 0, s, n, (const float*)R, ldr, Dinv,
                       ctr);
  else
    hipLaunchKernelGGL(trsv_inv_kernel<double>, dim3((unsigned)nblk), dim3(kTB), 0, s, n, (const double*)R, ldr,
                       Dinv, ctr);
  const hipError_t e = hipGetLastError();
  prof_end(slot, ROLE_TRSV_INV, s, (double)nblk * kTB * kTB * kTB / 3.0,
           (f32 ? 4.0 : 8.0) * (double)nblk * kTB * kTB / 2.0 + 8.0 * (double)nblk * kTB * kTB);
  return e;
}

hipError_t trsv_solve(int64_t n, bool f32, const void* R, int64_t ldr, void* work, double* y, int64_t seq,
                      hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nblk = trsv_blocks(n);
  if ((seq + 1) * nblk >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const double* Dinv = (const double*)work;
  unsigned* ctr = (unsigned*)((char*)work + trsv_workspace_bytes(n) - 256);
  const unsigned base = (unsigned)(seq * nblk);
  const int slot = prof_begin(s);
  if (f32)
    hipLaunchKernelGGL(trsv_lookback_kernel<float>, dim3((unsigned)nblk), dim3(kTThreads), 0, s, n, (const float*)R,
                       ldr, Dinv, y, ctr, base, wait_limit_ticks());
  else
    hipLaunchKernelGGL(trsv_lookback_kernel<double>, dim3((unsigned)nblk), dim3(kTThreads), 0, s, n,
                       (const double*)R, ldr, Dinv, y, ctr, base, wait_limit_ticks());
  const hipError_t e = hipGetLastError();
  const double dn = (double)n;
  prof_end(slot, ROLE_TRSV, s, dn * dn, (f32 ? 4.0 : 8.0) * dn * dn / 2.0 + 8.0 * dn * kTB + 16.0 * dn);
  return e;
}

const unsigned* trsv_error_word(int64_t n, const void* work) {
  return (const unsigned*)((const char*)work + trsv_workspace_bytes(n) - 256) + 2;
}

namespace {
__global__ void trsv_status_kernel(const unsigned* err, int32_t* status) { status[0] = err[0] != 0u ? 1 : 0; }
}  // namespace

hipError_t trsv_status(int64_t n, const void* work, int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(trsv_status_kernel, dim3(1), dim3(1), 0, s, trsv_error_word(n, work), status);
  return hipGetLastError();
}

}  // namespace cqr
