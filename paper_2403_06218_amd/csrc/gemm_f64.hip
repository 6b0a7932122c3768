// FP64 GEMM kernels on the CDNA4 matrix cores (v_mfma_f64_16x16x4_f64).
//
// These carry the matrix products of Algorithms 4 and 5 (Table 1: the GEMMs
// of steps S1/S2/S3/S6/S7/S8, the TRSMs of S5/S10 as a product with the
// inverted triangular factor, and the small products of S11/S12).
//
// Tiling: a 256-thread workgroup (4 wave64s in a 2 x 2 grid) computes an
// MT x NT tile of C; each wave owns (MT/2) x (NT/2) as 16 x 16 MFMA subtiles
// accumulated in registers.  K is walked in KT-deep stages staged through LDS:
// the next stage's global loads are issued into registers before the current
// stage's MFMAs, then written to LDS behind a barrier.
//
// LDS layout (both operands): element (k, x) of a KT x X stage lives at
//   k * (X + 16) + (x ^ ((k >> 1) & 7)).
// The row stride X + 16 puts the two 16-lane halves of each 32-lane MFMA
// operand read in opposite halves of the 64 banks; the XOR swizzle keeps the
// k-contiguous global->LDS writes (16 consecutive k of one column per 16
// lanes) conflict-free as well.
//
// MFMA lane layout (measured on gfx950): lane l supplies A(l%16, l/16) and
// B(l/16, l%16) and holds C(l/16 + 4v, l%16) in accumulator element v.  Rows
// of A are fed through the permutation p(i) = 4 (i % 4) + i / 4, so that lane
// l's four accumulator elements are the four consecutive rows 4 (l/16) .. +3
// of its column, stored contiguously.
#include "internal.h"

namespace cqr {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

// Stage depth and the occupancy the register budget is sized for (waves per
// SIMD); both can be overridden at build time for tuning sweeps.
#ifndef CQR_GEMM_KT
#define CQR_GEMM_KT 16
#endif
#ifndef CQR_GEMM_OCC
#define CQR_GEMM_OCC 2
#endif

template <int X>
__device__ __forceinline__ int lds_index(int k, int x) {
  return k * (X + 16) + (x ^ ((k >> 1) & 7));
}

// C = alpha * op(A) B + beta * C, or raw partial sums into `part` (split-K).
// TA: A is stored K x M (op(A) = A^T); otherwise M x K.  B is K x N.
// blockIdx.x: M tile, blockIdx.y: N tile, blockIdx.z: K split of length kchunk.
template <int ROLE, bool TA, int MT, int NT, int KT>
__global__ void __launch_bounds__(kThreads, CQR_GEMM_OCC)
gemm_f64_kernel(int64_t M, int64_t N, int64_t K, double alpha, const double* __restrict__ A, int64_t lda,
                const double* __restrict__ B, int64_t ldb, double beta, double* C, int64_t ldc, int64_t kchunk,
                double* __restrict__ part, const int* __restrict__ gate) {
  if (gate != nullptr && *gate != 0) return;
  constexpr int WM = 2, WN = 2;
  constexpr int WTM = MT / WM, WTN = NT / WN;
  constexpr int SM = WTM / 16, SN = WTN / 16;
  constexpr int KQ = KT / 4;
  constexpr int APT = MT * KT / kThreads, BPT = NT * KT / kThreads;
  static_assert(SM >= 1 && SN >= 1 && APT * kThreads == MT * KT && BPT * kThreads == NT * KT, "tile shape");
  __shared__ double sA[KT * (MT + 16)];
  __shared__ double sB[KT * (NT + 16)];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int li = lane & 15, lg = lane >> 4;
  const int prow = 4 * (li & 3) + (li >> 2);
  const int64_t m0 = (int64_t)blockIdx.x * MT;
  const int64_t n0 = (int64_t)blockIdx.y * NT;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = (K < kbeg + kchunk) ? K : kbeg + kchunk;
  const int nst = (kend > kbeg) ? (int)((kend - kbeg + KT - 1) / KT) : 0;

  // Global->register staging.  Every thread loads APT elements of A and BPT of
  // B per stage.  Element t of a thread sits at a wave-uniform base (kept in
  // SGPRs) plus one per-thread 32-bit byte offset, so the loads use the
  // scalar-base + vector-offset addressing form.
  constexpr int ASTEP = TA ? (kThreads / KT) : (kThreads / MT);  // per-t step along m (TA) or k
  constexpr int BSTEP = kThreads / KT;                            // per-t step along n
  const int a_k0 = TA ? (tid % KT) : (tid / MT);
  const int a_m0 = TA ? (tid / KT) : (tid % MT);
  const int b_k0 = tid % KT;
  const int b_n0 = tid / KT;
  const uint32_t a_boff = 8u * (TA ? (uint32_t)a_k0 + (uint32_t)a_m0 * (uint32_t)lda
                                   : (uint32_t)a_m0 + (uint32_t)a_k0 * (uint32_t)lda);
  const uint32_t b_boff = 8u * ((uint32_t)b_k0 + (uint32_t)b_n0 * (uint32_t)ldb);
  // Byte distance between a thread's consecutive elements t and t+1; the
  // host guarantees every in-tile offset fits in 32 bits.
  const uint32_t a_tstride = 8u * (uint32_t)ASTEP * (uint32_t)lda;
  const uint32_t b_tstride = 8u * (uint32_t)BSTEP * (uint32_t)ldb;
  const int64_t a_kstride = TA ? (int64_t)KT : (int64_t)KT * lda;
  const double* a_first = A + (TA ? (kbeg + m0 * lda) : (m0 + kbeg * lda));
  const double* b_first = B + (kbeg + n0 * ldb);
  const int64_t mrem64 = M - m0, nrem64 = N - n0;
  const int mrem = mrem64 > MT ? MT : (int)mrem64;
  const int nrem = nrem64 > NT ? NT : (int)nrem64;

  double ra[APT], rb[BPT];
  auto gload = [&](int st) {
    const int64_t kst = (int64_t)st * KT;
    const int64_t krem64 = kend - kbeg - kst;
    const int krem = krem64 > KT ? KT : (int)krem64;
    const double* abase = a_first + (int64_t)st * a_kstride;
    const double* bbase = b_first + kst;
#pragma unroll
    for (int t = 0; t < APT; ++t) {
      const int kk = TA ? a_k0 : a_k0 + t * ASTEP;
      const int mm = TA ? a_m0 + t * ASTEP : a_m0;
      ra[t] = (kk < krem && mm < mrem) ? *(const double*)((const char*)abase + (a_boff + t * a_tstride)) : 0.0;
    }
#pragma unroll
    for (int t = 0; t < BPT; ++t) {
      const int nn = b_n0 + t * BSTEP;
      rb[t] = (b_k0 < krem && nn < nrem) ? *(const double*)((const char*)bbase + (b_boff + t * b_tstride)) : 0.0;
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int t = 0; t < APT; ++t) {
      const int kk = TA ? a_k0 : a_k0 + t * ASTEP;
      const int mm = TA ? a_m0 + t * ASTEP : a_m0;
      sA[lds_index<MT>(kk, mm)] = ra[t];
    }
#pragma unroll
    for (int t = 0; t < BPT; ++t) sB[lds_index<NT>(b_k0, b_n0 + t * BSTEP)] = rb[t];
  };

  d4 acc[SM][SN];
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  if (nst > 0) {
    gload(0);
    sstore();
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const bool more = st + 1 < nst;
    if (more) gload(st + 1);
#pragma unroll
    for (int kq = 0; kq < KQ; ++kq) {
      const int k = 4 * kq + lg;
      double af[SM], bf[SN];
#pragma unroll
      for (int i = 0; i < SM; ++i) af[i] = sA[lds_index<MT>(k, wm * WTM + i * 16 + prow)];
#pragma unroll
      for (int j = 0; j < SN; ++j) bf[j] = sB[lds_index<NT>(k, wn * WTN + j * 16 + li)];
#pragma unroll
      for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      __syncthreads();
      sstore();
      __syncthreads();
    }
  }

  const int64_t zoff = (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) {
      const int64_t n = n0 + wn * WTN + j * 16 + li;
      const int64_t mb = m0 + wm * WTM + i * 16 + 4 * lg;
      if (n >= N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = mb + v;
        if (m >= M) continue;
        const double val = acc[i][j][v];
        if (part != nullptr) {
          part[zoff + m + n * M] = val;
        } else {
          double c = alpha * val;
          if (beta != 0.0) c += beta * C[m + n * ldc];
          C[m + n * ldc] = c;
        }
      }
    }
}

// C = alpha * sum_z part[z] + beta * C, summed in split order (deterministic).
__global__ void __launch_bounds__(256)
splitk_reduce_kernel(int64_t M, int64_t N, int nsplit, const double* __restrict__ part, double alpha, double beta,
                     double* C, int64_t ldc, const int* __restrict__ gate) {
  if (gate != nullptr && *gate != 0) return;
  const int64_t total = M * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int z = 0; z < nsplit; ++z) s += part[(int64_t)z * total + idx];
    const int64_t m = idx % M, n = idx / M;
    double c = alpha * s;
    if (beta != 0.0) c += beta * C[m + n * ldc];
    C[m + n * ldc] = c;
  }
}

constexpr int kKT = CQR_GEMM_KT;
constexpr int64_t kMaxLd = 4000000;

template <int ROLE, bool TA, int MT, int NT>
hipError_t launch_tile(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                       const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int64_t kchunk, int nsplit,
                       double* part, const int* gate, hipStream_t s) {
  const dim3 grid((unsigned)((M + MT - 1) / MT), (unsigned)((N + NT - 1) / NT), (unsigned)nsplit);
  hipLaunchKernelGGL((gemm_f64_kernel<ROLE, TA, MT, NT, kKT>), grid, dim3(kThreads), 0, s, M, N, K, alpha, A,
                     lda, B, ldb, beta, C, ldc, kchunk, part, gate);
  return hipGetLastError();
}

// Tile shapes, largest first.  A launch wants at least kMinWG workgroups
// (two resident per CU on 256 CUs); the largest tile that still gives that
// many is used, else the one that gives the most.
constexpr int kMinWG = 512;

int64_t tiles_for(int64_t M, int64_t N, int mt, int nt) { return ((M + mt - 1) / mt) * ((N + nt - 1) / nt); }

void pick_tile(int64_t M, int64_t N, int nsplit, int* mt, int* nt) {
  static const int cand[4][2] = {{128, 128}, {128, 64}, {64, 128}, {64, 64}};
  int best = 3;
  for (int c = 0; c < 4; ++c) {
    if ((cand[c][0] == 128 && M <= 64) || (cand[c][1] == 128 && N <= 64)) continue;
    if (tiles_for(M, N, cand[c][0], cand[c][1]) * nsplit >= kMinWG) {
      best = c;
      break;
    }
  }
  *mt = cand[best][0];
  *nt = cand[best][1];
}

template <int ROLE, bool TA>
hipError_t launch_gemm(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                       const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int64_t kchunk, int nsplit,
                       double* part, const int* gate, hipStream_t s) {
  int mt, nt;
  pick_tile(M, N, nsplit, &mt, &nt);
  if (mt == 128 && nt == 128)
    return launch_tile<ROLE, TA, 128, 128>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, nsplit, part,
                                           gate, s);
  if (mt == 128)
    return launch_tile<ROLE, TA, 128, 64>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, nsplit, part, gate,
                                          s);
  if (nt == 128)
    return launch_tile<ROLE, TA, 64, 128>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, nsplit, part, gate,
                                          s);
  return launch_tile<ROLE, TA, 64, 64>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, nsplit, part, gate, s);
}

// Tiles of the largest shape that fits (M, N): the split-K count is chosen
// against this before the final tile choice.
int64_t tiles_of(int64_t M, int64_t N) {
  return tiles_for(M, N, M > 64 ? 128 : 64, N > 64 ? 128 : 64);
}

// The kernels address a thread's elements inside one tile with 32-bit byte
// offsets: 8 * (KT + 128 * ld) must stay below 2^32.
bool ld_ok(int64_t ld) { return ld > 0 && ld <= kMaxLd; }

}  // namespace

int choose_splits(int64_t M, int64_t N, int64_t K, size_t part_cap) {
  const int64_t tiles = tiles_of(M, N);
  const int64_t target = kMinWG;
  if (tiles >= target || K <= 4 * kKT) return 1;
  int64_t splits = (target + tiles - 1) / tiles;
  const int64_t by_k = K / (4 * kKT);  // every split walks at least 4 stages
  if (splits > by_k) splits = by_k;
  const int64_t by_cap = (int64_t)(part_cap / (size_t)(M * N));
  if (splits > by_cap) splits = by_cap;
  return splits < 1 ? 1 : (int)splits;
}

hipError_t gemm_tn(Role role, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* part, size_t part_cap,
                   const int* gate, hipStream_t s, double flops) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (!ld_ok(lda) || !ld_ok(ldb)) return hipErrorInvalidValue;
  int nsplit = (part != nullptr) ? choose_splits(M, N, K, part_cap) : 1;
  int64_t kchunk = K;
  if (nsplit > 1) {
    kchunk = (K + nsplit - 1) / nsplit;
    kchunk = (kchunk + kKT - 1) / kKT * kKT;
    nsplit = (int)((K + kchunk - 1) / kchunk);
  }
  if (kchunk < 1) kchunk = 1;
  const double bytes = 8.0 * ((double)K * M + (double)K * N + (double)M * N * (beta != 0.0 ? 2.0 : 1.0));
  const int slot = prof_begin(s);
  hipError_t e;
  double* p = nsplit > 1 ? part : nullptr;
  if (role == ROLE_GRAM)
    e = launch_gemm<ROLE_GRAM, true>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, nsplit, p, gate, s);
  else
    e = launch_gemm<ROLE_PROJ, true>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, nsplit, p, gate, s);
  prof_end(slot, role, s, flops, bytes);
  if (e != hipSuccess || nsplit == 1) return e;
  const int64_t total = M * N;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  const int slot2 = prof_begin(s);
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, s, M, N, nsplit, part, alpha, beta,
                     C, ldc, gate);
  e = hipGetLastError();
  prof_end(slot2, ROLE_REDUCE, s, 0.0, 8.0 * (double)total * (nsplit + (beta != 0.0 ? 2 : 1)));
  return e;
}

hipError_t gemm_nn(Role role, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double beta, double* C, int64_t ldc, const int* gate, hipStream_t s,
                   double flops) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (!ld_ok(lda) || !ld_ok(ldb)) return hipErrorInvalidValue;
  const double bytes = 8.0 * ((double)K * M + (double)K * N + (double)M * N * (beta != 0.0 ? 2.0 : 1.0));
  const int64_t kchunk = K > 0 ? K : 1;
  const int slot = prof_begin(s);
  hipError_t e;
  switch (role) {
    case ROLE_UPDATE:
      e = launch_gemm<ROLE_UPDATE, false>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, 1, nullptr, gate, s);
      break;
    case ROLE_TRSM:
      e = launch_gemm<ROLE_TRSM, false>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, 1, nullptr, gate, s);
      break;
    default:
      e = launch_gemm<ROLE_SMALL, false>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, 1, nullptr, gate, s);
      break;
  }
  prof_end(slot, role, s, flops, bytes);
  return e;
}

}  // namespace cqr
