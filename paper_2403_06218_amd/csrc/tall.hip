// CGS-CQR2 (Algorithm 5) and CholeskyQR2 (Algorithm 4) of one narrow block
// (w <= 16 columns) of a tall matrix, as row-streaming kernels.
//
// For a tall q x r matrix with a narrow block width every step of a block is
// a sweep over the q rows with little arithmetic per byte, so the block is
// bound by HBM traffic and by the number of sweeps.  Here each sweep does
// everything that one pass over the rows allows:
//
//   tall_proj_kernel          H = P^T X                        (S1)
//   tall_update_gram_kernel   Y = X - P H, then W = Y^T Y       (S2+S3, S7+S8)
//   tall_trsm_proj_kernel     T = X L^{-T}, then Hb = P^T T     (S5+S6; S10 alone)
//
// P (q x s, the finished basis) has s <= 128 columns.  A workgroup (8 waves)
// owns a contiguous range of rows and walks it in 16-row tiles, one tile per
// wave at a time, with FP64 MFMA (16x16x4): the 16 rows of a tile are the
// reduction dimension of the P^T products and the N dimension of the
// (transposed) products with small right factors.  In the 16x16x4 layout
// lane l supplies A(l%16, l/16) and B(l/16, l%16) and holds C(l/16 + 4v,
// l%16) in element v; every global load and store is arranged so that a
// lane touches one row (16 consecutive rows per instruction), and a tile is
// moved to the rows-as-reduction form through LDS only where a product
// reduces over rows.
//
// The reductions over rows end in per-workgroup partial sums, combined by
// tall_reduce_kernel in a fixed order (results do not depend on timing).
// Every kernel is gated on the breakdown status word like the GEMMs.
#include "internal.h"

namespace cqr {
namespace {

typedef double td4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ td4 tmma(double a, double b, td4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kTallThreads = 512;
constexpr int kTallWaves = kTallThreads / 64;
constexpr int kTallGroups = 512;  // target number of workgroups (two per CU)
constexpr int64_t kTallMinRows = 16384;

// Partial (M x 16, M = 16 MT) of workgroup g: element (m, n) at
// part[g * 256 MT + m + 16 MT n].  Waves add their tiles in wave order.
template <int MT>
__device__ __forceinline__ void tall_store_partial(const td4 (&acc)[MT], double* sred, double* part, int g,
                                                   int lane, int wave, int tid) {
  const int li = lane & 15, lg = lane >> 4;
  for (int t = 0; t < MT; ++t) {
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) sred[wave * 256 + (lg + 4 * v) + 16 * li] = acc[t][v];
    __syncthreads();
    if (tid < 256) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < kTallWaves; ++k) s += sred[k * 256 + tid];
      const int m = tid & 15, n = tid >> 4;
      part[(int64_t)g * 256 * MT + (16 * t + m) + (int64_t)16 * MT * n] = s;
    }
  }
}

// Global accesses use the coalesced form "row li, column lg + 4 v" (16
// consecutive rows of 4 columns per instruction).  tr16 turns a wave's
// 16 x 16 tile held that way into the form "row 4 v + lg, column li" (the
// reduction-over-rows operand of the 16x16x4 MFMA) through the wave's own
// LDS scratch; LDS operations of one wave complete in order, so no barrier.
__device__ __forceinline__ void tr16(const double (&in)[4], double (&out)[4], double* tb, int li, int lg) {
#pragma unroll
  for (int v = 0; v < 4; ++v) tb[li * 17 + lg + 4 * v] = in[v];
#pragma unroll
  for (int v = 0; v < 4; ++v) out[v] = tb[(4 * v + lg) * 17 + li];
}

// S1: partial H = P[rows]^T X[rows] (s x w).
template <int MT>
__global__ void __launch_bounds__(kTallThreads)
tall_proj_kernel(int64_t q, int s, int w, const double* __restrict__ P, int64_t ldp, const double* __restrict__ X,
                 int64_t ldx, int64_t ch, double* __restrict__ part, const int* __restrict__ gate) {
  if (gate != nullptr && *gate != 0) return;
  __shared__ double sred[kTallWaves * 256];
  __shared__ double stb[kTallWaves * 16 * 17];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  double* tb = stb + wave * 16 * 17;
  const int64_t r0 = (int64_t)blockIdx.x * ch, r1 = (r0 + ch < q) ? r0 + ch : q;
  td4 acc[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) acc[t] = td4{0.0, 0.0, 0.0, 0.0};
  for (int64_t row0 = r0 + 16 * wave; row0 < r1; row0 += 16 * kTallWaves) {
    const int64_t row = row0 + li;
    const bool rok = row < r1;
    double xl[4], pl[MT][4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = lg + 4 * v;
      xl[v] = (rok && c < w) ? X[row + c * ldx] : 0.0;
#pragma unroll
      for (int t = 0; t < MT; ++t) pl[t][v] = (rok && 16 * t + c < s) ? P[row + (16 * t + c) * ldp] : 0.0;
    }
    double xv[4];
    tr16(xl, xv, tb, li, lg);
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      double pv[4];
      tr16(pl[t], pv, tb, li, lg);
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[t] = tmma(pv[v], xv[v], acc[t]);
    }
  }
  tall_store_partial<MT>(acc, sred, part, blockIdx.x, lane, wave, tid);
}

// S2 + S3 (S7 + S8): Y[rows] = X[rows] - P[rows] H (skipped when s == 0; Y may
// be X), then the partial W = Y[rows]^T Y[rows] (w x w).  The update is
// formed transposed, (P H)^T = H^T P^T, so that its result is held row per
// lane like the coalesced loads and stores.
template <int MT>
__global__ void __launch_bounds__(kTallThreads)
tall_update_gram_kernel(int64_t q, int s, int w, const double* __restrict__ P, int64_t ldp,
                        const double* __restrict__ H, int64_t ldh, const double* X, int64_t ldx, double* Y,
                        int64_t ldy, int64_t ch, double* __restrict__ part, const int* __restrict__ gate) {
  if (gate != nullptr && *gate != 0) return;
  __shared__ double sred[kTallWaves * 256];
  __shared__ double stb[kTallWaves * 16 * 17];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  double* tb = stb + wave * 16 * 17;
  const int64_t r0 = (int64_t)blockIdx.x * ch, r1 = (r0 + ch < q) ? r0 + ch : q;
  // A operand of H^T P^T, k-step (t, v): H(16 t + 4 v + lg, li).
  double ha[MT][4];
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = 16 * t + 4 * v + lg;
      ha[t][v] = (k < s && li < w) ? H[k + li * ldh] : 0.0;
    }
  td4 g[1] = {td4{0.0, 0.0, 0.0, 0.0}};
  for (int64_t row0 = r0 + 16 * wave; row0 < r1; row0 += 16 * kTallWaves) {
    const int64_t row = row0 + li;
    const bool rok = row < r1;
    // Element v: row `row`, column lg + 4 v.
    double x[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = lg + 4 * v;
      x[v] = (rok && c < w) ? X[row + c * ldx] : 0.0;
    }
    if (s > 0) {
      // B operand, k-step (t, v): P(row, 16 t + 4 v + lg).
      double pb[MT][4];
#pragma unroll
      for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = 16 * t + 4 * v + lg;
          pb[t][v] = (rok && c < s) ? P[row + c * ldp] : 0.0;
        }
      td4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int t = 0; t < MT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) c = tmma(ha[t][v], pb[t][v], c);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int col = lg + 4 * v;
        x[v] -= c[v];
        if (rok && col < w) Y[row + col * ldy] = x[v];
      }
    }
    double xt[4];
    tr16(x, xt, tb, li, lg);
#pragma unroll
    for (int v = 0; v < 4; ++v) g[0] = tmma(xt[v], xt[v], g[0]);
  }
  tall_store_partial<1>(g, sred, part, blockIdx.x, lane, wave, tid);
}

// S5 (S10): T[rows] = X[rows] XT (XT = (L^{-1})^T, w x w), formed transposed
// (XT^T X^T) so that T is held row per lane; with PROJ also the partial
// Hb = P[rows]^T T[rows] of the next pass (S6).  X and T may be the same
// array (each tile is read before it is written, by the same wave).
template <int MT, bool PROJ>
__global__ void __launch_bounds__(kTallThreads)
tall_trsm_proj_kernel(int64_t q, int s, int w, const double* X, int64_t ldx, const double* __restrict__ XT,
                      double* T, int64_t ldt, const double* __restrict__ P, int64_t ldp, int64_t ch,
                      double* __restrict__ part, const int* __restrict__ gate) {
  if (gate != nullptr && *gate != 0) return;
  __shared__ double sred[kTallWaves * 256];
  __shared__ double stb[kTallWaves * 16 * 17];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  double* tb = stb + wave * 16 * 17;
  const int64_t r0 = (int64_t)blockIdx.x * ch, r1 = (r0 + ch < q) ? r0 + ch : q;
  // A operand of XT^T X^T, k-step v: XT(4 v + lg, li).
  double xa[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int k = 4 * v + lg;
    xa[v] = (k < w && li < w) ? XT[k + li * w] : 0.0;
  }
  td4 acc[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) acc[t] = td4{0.0, 0.0, 0.0, 0.0};
  for (int64_t row0 = r0 + 16 * wave; row0 < r1; row0 += 16 * kTallWaves) {
    const int64_t row = row0 + li;
    const bool rok = row < r1;
    // B operand, k-step v: X(row, 4 v + lg).
    double xb[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = 4 * v + lg;
      xb[v] = (rok && c < w) ? X[row + c * ldx] : 0.0;
    }
    double pl[MT][4];
    if constexpr (PROJ) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = lg + 4 * v;
#pragma unroll
        for (int t = 0; t < MT; ++t) pl[t][v] = (rok && 16 * t + c < s) ? P[row + (16 * t + c) * ldp] : 0.0;
      }
    }
    td4 c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int v = 0; v < 4; ++v) c = tmma(xa[v], xb[v], c);
    // Element v of c: T(row, lg + 4 v).
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int col = lg + 4 * v;
      if (rok && col < w) T[row + col * ldt] = c[v];
    }
    if constexpr (PROJ) {
      double cv[4], tt[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) cv[v] = c[v];
      tr16(cv, tt, tb, li, lg);
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        double pv[4];
        tr16(pl[t], pv, tb, li, lg);
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[t] = tmma(pv[v], tt[v], acc[t]);
      }
    }
  }
  if constexpr (PROJ) tall_store_partial<MT>(acc, sred, part, blockIdx.x, lane, wave, tid);
}

// dst(m, n) = sum over g of the partials (m < M, n < N; partial layout as in
// tall_store_partial with Mp = 16 MT rows), in a fixed order: thread (o, z)
// of a workgroup sums groups z, z + 16, ... of output o, then the 16 sums
// are added in z order.
__global__ void __launch_bounds__(256)
tall_reduce_kernel(int M, int N, int Mp, int G, const double* __restrict__ part, double* __restrict__ dst,
                   int64_t ldd, const int* __restrict__ gate) {
  if (gate != nullptr && *gate != 0) return;
  __shared__ double sz[16][17];
  const int o_loc = threadIdx.x & 15, z = threadIdx.x >> 4;
  const int o = blockIdx.x * 16 + o_loc;  // index into the Mp x 16 partial
  const int64_t stride = (int64_t)Mp * 16;
  double s = 0.0;
  if (o < Mp * 16) {
    int gg = z;
    for (; gg + 48 < G; gg += 64) {
      const double a0 = part[(int64_t)gg * stride + o], a1 = part[(int64_t)(gg + 16) * stride + o];
      const double a2 = part[(int64_t)(gg + 32) * stride + o], a3 = part[(int64_t)(gg + 48) * stride + o];
      s += a0;
      s += a1;
      s += a2;
      s += a3;
    }
    for (; gg < G; gg += 16) s += part[(int64_t)gg * stride + o];
  }
  sz[o_loc][z] = s;
  __syncthreads();
  if (z == 0 && o < Mp * 16) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) t += sz[o_loc][k];
    const int m = o % Mp, n = o / Mp;
    if (m < M && n < N) dst[m + n * ldd] = t;
  }
}

int tall_mt(int s) { return s <= 16 ? 1 : s <= 32 ? 2 : s <= 48 ? 3 : s <= 64 ? 4 : 8; }

int64_t tall_rows_per_group(int64_t q) {
  const int64_t tiles = (q + 15) / 16;
  const int64_t per = (tiles + kTallGroups - 1) / kTallGroups;
  return 16 * (per > 0 ? per : 1);
}

hipError_t tall_reduce(int M, int N, int MT, int G, const double* part, double* dst, int64_t ldd, const int* gate,
                       hipStream_t st) {
  const int Mp = 16 * MT;
  const int slot = prof_begin(st);
  hipLaunchKernelGGL(tall_reduce_kernel, dim3((unsigned)((Mp * 16 + 15) / 16)), dim3(256), 0, st, M, N, Mp, G, part,
                     dst, ldd, gate);
  const hipError_t e = hipGetLastError();
  prof_end(slot, ROLE_REDUCE, st, 0.0, 8.0 * (double)G * Mp * 16);
  return e;
}

}  // namespace

bool tall_eligible(int64_t q, int64_t w, int64_t s) {
  return q >= kTallMinRows && w >= 1 && w <= 16 && s >= 0 && s <= 128;
}

hipError_t tall_proj(int64_t q, int s, int w, const double* P, int64_t ldp, const double* X, int64_t ldx, double* H,
                     int64_t ldh, double* part, size_t part_cap, const int* gate, hipStream_t st) {
  const int MT = tall_mt(s);
  const int64_t ch = tall_rows_per_group(q);
  const int G = (int)((q + ch - 1) / ch);
  if ((size_t)G * 256 * MT > part_cap) return hipErrorInvalidValue;
  const int slot = prof_begin(st);
  const dim3 grid((unsigned)G), block(kTallThreads);
  switch (MT) {
    case 1: hipLaunchKernelGGL(tall_proj_kernel<1>, grid, block, 0, st, q, s, w, P, ldp, X, ldx, ch, part, gate); break;
    case 2: hipLaunchKernelGGL(tall_proj_kernel<2>, grid, block, 0, st, q, s, w, P, ldp, X, ldx, ch, part, gate); break;
    case 3: hipLaunchKernelGGL(tall_proj_kernel<3>, grid, block, 0, st, q, s, w, P, ldp, X, ldx, ch, part, gate); break;
    case 4: hipLaunchKernelGGL(tall_proj_kernel<4>, grid, block, 0, st, q, s, w, P, ldp, X, ldx, ch, part, gate); break;
    default: hipLaunchKernelGGL(tall_proj_kernel<8>, grid, block, 0, st, q, s, w, P, ldp, X, ldx, ch, part, gate); break;
  }
  hipError_t e = hipGetLastError();
  prof_end(slot, ROLE_PROJ, st, 2.0 * (double)q * s * w, 8.0 * (double)q * (s + w));
  if (e != hipSuccess) return e;
  return tall_reduce(s, w, MT, G, part, H, ldh, gate, st);
}

hipError_t tall_update_gram(int64_t q, int s, int w, const double* P, int64_t ldp, const double* H, int64_t ldh,
                            const double* X, int64_t ldx, double* Y, int64_t ldy, double* W, double* part,
                            size_t part_cap, const int* gate, hipStream_t st) {
  const int MT = tall_mt(s);
  const int64_t ch = tall_rows_per_group(q);
  const int G = (int)((q + ch - 1) / ch);
  if ((size_t)G * 256 > part_cap) return hipErrorInvalidValue;
  const int slot = prof_begin(st);
  const dim3 grid((unsigned)G), block(kTallThreads);
  switch (MT) {
    case 1: hipLaunchKernelGGL(tall_update_gram_kernel<1>, grid, block, 0, st, q, s, w, P, ldp, H, ldh, X, ldx, Y, ldy, ch, part, gate); break;
    case 2: hipLaunchKernelGGL(tall_update_gram_kernel<2>, grid, block, 0, st, q, s, w, P, ldp, H, ldh, X, ldx, Y, ldy, ch, part, gate); break;
    case 3: hipLaunchKernelGGL(tall_update_gram_kernel<3>, grid, block, 0, st, q, s, w, P, ldp, H, ldh, X, ldx, Y, ldy, ch, part, gate); break;
    case 4: hipLaunchKernelGGL(tall_update_gram_kernel<4>, grid, block, 0, st, q, s, w, P, ldp, H, ldh, X, ldx, Y, ldy, ch, part, gate); break;
    default: hipLaunchKernelGGL(tall_update_gram_kernel<8>, grid, block, 0, st, q, s, w, P, ldp, H, ldh, X, ldx, Y, ldy, ch, part, gate); break;
  }
  hipError_t e = hipGetLastError();
  prof_end(slot, ROLE_UPDATE, st, 2.0 * (double)q * w * (s + w),
           8.0 * (double)q * (s + (s > 0 ? 2.0 : 1.0) * w));
  if (e != hipSuccess) return e;
  return tall_reduce(w, w, 1, G, part, W, w, gate, st);
}

hipError_t tall_trsm_proj(int64_t q, int s, int w, const double* X, int64_t ldx, const double* XT, double* T,
                          int64_t ldt, const double* P, int64_t ldp, double* Hb, int64_t ldhb, double* part,
                          size_t part_cap, const int* gate, hipStream_t st) {
  const bool proj = s > 0 && Hb != nullptr;
  const int MT = tall_mt(s);
  const int64_t ch = tall_rows_per_group(q);
  const int G = (int)((q + ch - 1) / ch);
  if (proj && (size_t)G * 256 * MT > part_cap) return hipErrorInvalidValue;
  const int slot = prof_begin(st);
  const dim3 grid((unsigned)G), block(kTallThreads);
  if (!proj) {
    hipLaunchKernelGGL((tall_trsm_proj_kernel<1, false>), grid, block, 0, st, q, 0, w, X, ldx, XT, T, ldt, P, ldp, ch,
                       part, gate);
  } else {
    switch (MT) {
      case 1: hipLaunchKernelGGL((tall_trsm_proj_kernel<1, true>), grid, block, 0, st, q, s, w, X, ldx, XT, T, ldt, P, ldp, ch, part, gate); break;
      case 2: hipLaunchKernelGGL((tall_trsm_proj_kernel<2, true>), grid, block, 0, st, q, s, w, X, ldx, XT, T, ldt, P, ldp, ch, part, gate); break;
      case 3: hipLaunchKernelGGL((tall_trsm_proj_kernel<3, true>), grid, block, 0, st, q, s, w, X, ldx, XT, T, ldt, P, ldp, ch, part, gate); break;
      case 4: hipLaunchKernelGGL((tall_trsm_proj_kernel<4, true>), grid, block, 0, st, q, s, w, X, ldx, XT, T, ldt, P, ldp, ch, part, gate); break;
      default: hipLaunchKernelGGL((tall_trsm_proj_kernel<8, true>), grid, block, 0, st, q, s, w, X, ldx, XT, T, ldt, P, ldp, ch, part, gate); break;
    }
  }
  hipError_t e = hipGetLastError();
  prof_end(slot, ROLE_TRSM, st, (double)q * w * w + (proj ? 2.0 * (double)q * s * w : 0.0),
           8.0 * (double)q * (2.0 * w + (proj ? s : 0)));
  if (e != hipSuccess || !proj) return e;
  return tall_reduce(s, w, MT, G, part, Hb, ldhb, gate, st);
}

}  // namespace cqr
