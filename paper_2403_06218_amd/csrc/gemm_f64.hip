// FP64 GEMM kernels on the CDNA4 matrix cores (v_mfma_f64_16x16x4_f64).
//
// These carry the matrix products of Algorithms 4 and 5 (Table 1: the GEMMs
// of steps S1/S2/S3/S6/S7/S8, the TRSMs of S5/S10 as a product with the
// inverted triangular factor, and the small products of S11/S12).
//
// Tiling (both kernels): a 256-thread workgroup (4 wave64s in a 2 x 2 grid)
// computes an MT x NT tile of C; each wave owns (MT/2) x (NT/2) as 16 x 16
// MFMA subtiles accumulated in registers, and K is walked in 16-deep stages
// staged through LDS.
//
// gemm_dma_kernel (used whenever operands are 16-byte aligned with even
// leading dimensions and K is a multiple of 16): each stage is copied
// global -> LDS by the LDS-DMA load (global_load_lds_dwordx4, 16 bytes per
// lane, no registers), into an S-slot ring with one barrier per stage; every
// ring slot is a separate LDS object so the compiler can tell a stage's reads
// from the DMA writes still in flight to the other slots.  Layouts:
//   k-contiguous operand (A of A^T B, and B): column x holds 8 chunks of two
//     k values; chunk c of column x sits at slot c ^ ((x >> 1) & 7), so the 16
//     lanes of an MFMA operand read (16 columns, one k) hit 16 distinct bank
//     groups;
//   m-contiguous operand (A of A B): column k holds row pairs; pair c sits at
//     position c ^ (8 ((k >> 2) & 1)), putting the two 16-lane halves of a
//     32-lane read in opposite bank halves.
// MFMA step kq takes k = 4 (lane / 16) + kq, so each lane's four k values are
// one contiguous run (read as 128-bit LDS loads).
//
// gemm_reg_kernel (any alignment, any K): global loads into registers before
// the current stage's MFMAs, written to LDS behind a barrier; LDS element
// (k, x) at k (X + 16) + (x ^ ((k >> 1) & 7)).
//
// MFMA lane layout (measured on gfx950): lane l supplies A(l%16, l/16) and
// B(l/16, l%16) and holds C(l/16 + 4v, l%16) in accumulator element v.  Rows
// of A are fed through the permutation p(i) = 4 (i % 4) + i / 4, so that lane
// l's four accumulator elements are the four consecutive rows 4 (l/16) .. +3
// of its column, stored contiguously.
#include <type_traits>

#include "internal.h"

namespace cqr {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

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
gemm_reg_kernel(int64_t M, int64_t N, int64_t K, double alpha, const double* __restrict__ A, int64_t lda,
                const double* __restrict__ B, int64_t ldb, double beta, double* C, int64_t ldc, int64_t kchunk,
                double* __restrict__ part, const int* __restrict__ gate) {
  if (gate != nullptr && *gate != 0) return;
  if constexpr (TA && ROLE == ROLE_GRAM && MT == NT) {
    // W = Q^T Q is symmetric; its strictly lower tiles are not formed.
    if (M == N && blockIdx.x > blockIdx.y) return;
  }
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
  int64_t kend = (K < kbeg + kchunk) ? K : kbeg + kchunk;
  if constexpr (!TA && (ROLE == ROLE_TRSM || ROLE == ROLE_SMALL)) {
    // B is upper triangular: rows k >= n0 + NT of this tile's columns are zero.
    if (n0 + NT < kend) kend = n0 + NT;
  }
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


// ------------------------------------------------------------------------
// LDS-DMA kernel.
// ------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void;
constexpr int kDmaKT = 16;

// 16-byte global -> LDS copy per lane; lane l lands at lds_base + 16 l.
__device__ __forceinline__ void dma16(const double* g, double* lds_base) {
  __builtin_amdgcn_global_load_lds((const void*)g, (lds_void*)lds_base, 16, 0, 0);
}

// Wait until at most N vector-memory operations of this wave are outstanding.
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Element (k, x) of a k-contiguous stage (X columns of 16 k values).
__device__ __forceinline__ int kc_index(int k, int x) { return x * 16 + 2 * ((k >> 1) ^ ((x >> 1) & 7)) + (k & 1); }
// Element (m, k) of an m-contiguous stage (16 columns of X rows).
template <int X>
__device__ __forceinline__ int mc_index(int m, int k) {
  return k * X + 2 * ((m >> 1) ^ (8 * ((k >> 2) & 1))) + (m & 1);
}

// Same contract as gemm_reg_kernel; requires K and kchunk multiples of 16,
// 16-byte aligned A and B, even lda and ldb, and (for !TA) even M.
// F32C: the operands are rounded to FP32 as they leave LDS and multiplied by
// v_mfma_f32_16x16x4_f32 (twice the FP64 matrix rate) with FP32 accumulation
// over the workgroup's reduction range; the partial sums and the epilogue stay
// FP64.  The operand layout is the FP64 one; the FP32 accumulator holds rows
// 4(l/16) + v of the permuted operand rows, i.e. tile rows l/16 + 4v.
template <int ROLE, bool TA, int MT, int NT, int S, int OCC, int WM = 2, int WN = 2, bool F32C = false>
__global__ void __launch_bounds__(64 * WM * WN, OCC)
gemm_dma_kernel(int64_t M, int64_t N, int64_t K, double alpha, const double* __restrict__ A, int64_t lda,
                const double* __restrict__ B, int64_t ldb, double beta, double* C, int64_t ldc, int64_t kchunk,
                double* __restrict__ part, const int* __restrict__ gate) {
  static_assert(S == 2 || S == 3, "ring depth");
  if (gate != nullptr && *gate != 0) return;
  if constexpr (TA && ROLE == ROLE_GRAM && MT == NT) {
    // W = Q^T Q is symmetric; its strictly lower tiles are not formed.
    if (M == N && blockIdx.x > blockIdx.y) return;
  }
  constexpr int KT = kDmaKT;
  constexpr int NW = WM * WN;
  constexpr int WTM = MT / WM, WTN = NT / WN;
  constexpr int SM = WTM / 16, SN = WTN / 16;
  constexpr int ASTAGE = MT * KT, BSTAGE = NT * KT;                 // doubles per stage
  constexpr int AINS = ASTAGE / 128 / NW, BINS = BSTAGE / 128 / NW; // DMA instructions per wave per stage
  static_assert(AINS >= 1 && BINS >= 1 && SM >= 1 && SN >= 1, "tile shape");
  static_assert(AINS * 128 * NW == ASTAGE && BINS * 128 * NW == BSTAGE, "stage split over waves");
  __shared__ __attribute__((aligned(16))) double sA0[ASTAGE], sA1[ASTAGE], sA2[S > 2 ? ASTAGE : 2];
  __shared__ __attribute__((aligned(16))) double sB0[BSTAGE], sB1[BSTAGE], sB2[S > 2 ? BSTAGE : 2];
  auto slotA = [&](auto c) -> double* {
    if constexpr (c.value == 0) return sA0;
    else if constexpr (c.value == 1) return sA1;
    else return sA2;
  };
  auto slotB = [&](auto c) -> double* {
    if constexpr (c.value == 0) return sB0;
    else if constexpr (c.value == 1) return sB1;
    else return sB2;
  };

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave % WM, wn = wave / WM;
  const int li = lane & 15, lg = lane >> 4;
  const int prow = 4 * (li & 3) + (li >> 2);
  const int64_t m0 = (int64_t)blockIdx.x * MT;
  const int64_t n0 = (int64_t)blockIdx.y * NT;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  int64_t kend = (K < kbeg + kchunk) ? K : kbeg + kchunk;
  if constexpr (!TA && (ROLE == ROLE_TRSM || ROLE == ROLE_SMALL)) {
    // B is upper triangular: rows k >= n0 + NT of this tile's columns are zero
    // (n0 + NT is a multiple of the stage depth).
    if (n0 + NT < kend) kend = n0 + NT;
  }
  const int nst = (kend > kbeg) ? (int)((kend - kbeg) / KT) : 0;

  // Source offsets (elements from the stage origin) of this lane's chunks.
  // Columns past the matrix are clamped to the last one; their values only
  // reach output rows/columns that are never stored.
  int64_t aoff[AINS], boff[BINS];
#pragma unroll
  for (int t = 0; t < AINS; ++t) {
    const int p = (wave * AINS + t) * 64 + lane;  // chunk position in the stage
    if (TA) {
      const int x = p / 8, c = (p % 8) ^ ((x >> 1) & 7);
      const int64_t m = (m0 + x < M) ? m0 + x : M - 1;
      aoff[t] = 2 * c + m * lda;
    } else {
      constexpr int CPC = MT / 2;  // row pairs per column
      const int kk = p / CPC, c = (p % CPC) ^ (8 * ((kk >> 2) & 1));
      const int64_t m = (m0 + 2 * c < M) ? m0 + 2 * c : M - 2;
      aoff[t] = m + (int64_t)kk * lda;
    }
  }
#pragma unroll
  for (int t = 0; t < BINS; ++t) {
    const int p = (wave * BINS + t) * 64 + lane;
    const int x = p / 8, c = (p % 8) ^ ((x >> 1) & 7);
    const int64_t n = (n0 + x < N) ? n0 + x : N - 1;
    boff[t] = 2 * c + n * ldb;
  }

  auto issue = [&](int st, auto slot) {
    const int64_t k0 = kbeg + (int64_t)st * KT;
    const double* ga = A + (TA ? k0 : k0 * lda);
    const double* gb = B + k0;
    double* la = slotA(slot);
    double* lb = slotB(slot);
#pragma unroll
    for (int t = 0; t < AINS; ++t) dma16(ga + aoff[t], la + (wave * AINS + t) * 128);
#pragma unroll
    for (int t = 0; t < BINS; ++t) dma16(gb + boff[t], lb + (wave * BINS + t) * 128);
  };

  using Acc = std::conditional_t<F32C, f4, d4>;
  Acc acc[SM][SN];
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) acc[i][j] = Acc{0, 0, 0, 0};

  auto compute = [&](auto slot) {
    const double* cA = slotA(slot);
    const double* cB = slotB(slot);
#pragma unroll
    for (int kq = 0; kq < 4; ++kq) {
      const int k = 4 * lg + kq;
      double af[SM], bf[SN];
#pragma unroll
      for (int i = 0; i < SM; ++i) {
        const int m = wm * WTM + i * 16 + prow;
        af[i] = TA ? cA[kc_index(k, m)] : cA[mc_index<MT>(m, k)];
      }
#pragma unroll
      for (int j = 0; j < SN; ++j) bf[j] = cB[kc_index(k, wn * WTN + j * 16 + li)];
#pragma unroll
      for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j) {
          if constexpr (F32C)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)af[i], (float)bf[j], acc[i][j], 0, 0, 0);
          else
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
    }
  };

  constexpr int PER_STAGE = AINS + BINS;  // DMA operations per wave per stage
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  // Stage st lives in slot st % S.  Its DMA is complete once at most S - 2
  // later stages are outstanding; the barrier then also guarantees that every
  // wave has finished reading the slot the next DMA overwrites.
  auto step = [&](int st, auto cur, auto nxt) {
    if (st + S - 2 < nst) wait_vmcnt<(S - 2) * PER_STAGE>();
    else wait_vmcnt<0>();
    __syncthreads();
    if (st + S - 1 < nst) issue(st + S - 1, nxt);
    compute(cur);
  };
  if (nst > 0) issue(0, I0{});
  if (S > 2 && nst > 1) issue(1, I1{});
  for (int st = 0; st < nst; st += S) {
    if constexpr (S == 2) {
      step(st, I0{}, I1{});
      if (st + 1 < nst) step(st + 1, I1{}, I0{});
    } else {
      step(st, I0{}, I2{});
      if (st + 1 < nst) step(st + 1, I1{}, I0{});
      if (st + 2 < nst) step(st + 2, I2{}, I1{});
    }
  }

  const int64_t zoff = (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) {
      const int64_t n = n0 + wn * WTN + j * 16 + li;
      const int64_t mb = m0 + wm * WTM + i * 16 + (F32C ? lg : 4 * lg);
      if (n >= N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = mb + (F32C ? 4 * v : v);
        if (m >= M) continue;
        const double val = (double)acc[i][j][v];
        if (part != nullptr) {
          // FP32 sums are stored as FP32: the partial-sum traffic halves.
          if constexpr (F32C) reinterpret_cast<float*>(part)[zoff + m + n * M] = acc[i][j][v];
          else part[zoff + m + n * M] = val;
        } else {
          double c = alpha * val;
          if (beta != 0.0) c += beta * C[m + n * ldc];
          C[m + n * ldc] = c;
        }
      }
    }
}

// C = alpha * sum_z part[z] + beta * C, deterministic: a workgroup covers 64
// consecutive outputs with 4 groups of 64 threads; group g sums its quarter of
// the splits in split order (16 loads in flight), and the 4 group sums are
// added in group order.  P: the partial sums' type (FP64, or FP32 from the
// FP32-arithmetic kernels); the sums are FP64.
template <typename P>
__global__ void __launch_bounds__(256)
splitk_reduce_kernel(int64_t M, int64_t N, int nsplit, const P* __restrict__ part, double alpha, double beta,
                     double* C, int64_t ldc, const int* __restrict__ gate) {
  if (gate != nullptr && *gate != 0) return;
  __shared__ double red[4][64];
  const int64_t total = M * N;
  const int t = threadIdx.x, o = t & 63, g = t >> 6;
  const int zper = (nsplit + 3) / 4;
  const int z0 = g * zper, z1 = (z0 + zper < nsplit) ? z0 + zper : nsplit;
  for (int64_t base = (int64_t)blockIdx.x * 64; base < total; base += (int64_t)gridDim.x * 64) {
    const int64_t idx = base + o;
    double s = 0.0;
    if (idx < total) {
      int z = z0;
      for (; z + 16 <= z1; z += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = (double)part[(int64_t)(z + u) * total + idx];
#pragma unroll
        for (int u = 0; u < 16; ++u) s += v[u];
      }
      for (; z < z1; ++z) s += (double)part[(int64_t)z * total + idx];
    }
    red[g][o] = s;
    __syncthreads();
    if (g == 0 && idx < total) {
      const double sum = ((red[0][o] + red[1][o]) + red[2][o]) + red[3][o];
      const int64_t m = idx % M, n = idx / M;
      double c = alpha * sum;
      if (beta != 0.0) c += beta * C[m + n * ldc];
      C[m + n * ldc] = c;
    }
    __syncthreads();
  }
}

constexpr int kKT = CQR_GEMM_KT;
constexpr int64_t kMaxLd = 4000000;

// The register kernel addresses a thread's elements inside one tile with
// 32-bit byte offsets: 8 * (KT + 128 * ld) must stay below 2^32.
bool ld_ok(int64_t ld) { return ld > 0 && ld <= kMaxLd; }

int64_t tiles_for(int64_t M, int64_t N, int mt, int nt) { return ((M + mt - 1) / mt) * ((N + nt - 1) / nt); }

struct Plan {
  bool dma;
  int mt, nt;
  int nsplit;
  int64_t kchunk;
};

bool dma_eligible(bool ta, int64_t M, int64_t K, const double* A, int64_t lda, const double* B, int64_t ldb) {
  if ((reinterpret_cast<uintptr_t>(A) & 15) || (reinterpret_cast<uintptr_t>(B) & 15)) return false;
  if ((lda & 1) || (ldb & 1)) return false;
  if (K % kDmaKT != 0) return false;
  if (!ta && ((M & 1) || M < 2)) return false;
  return true;
}

// Tile shape: the largest that still occupies every CU (one 128 x 128
// workgroup per CU, two of the 64-wide shapes), else the smallest.  A
// triangular right factor (tri) takes 64-wide column tiles: the reduction of
// column tile n0 stops at n0 + 64, so the exact zeros skipped grow from a
// quarter to three eighths of the product, and twice as many workgroups
// balance the uneven lengths.
void pick_tile(bool ta, int64_t M, int64_t N, int nsplit, int* mt, int* nt, bool tri = false) {
  const bool bigM = M > 64, bigN = N > 64;
  if (tri && !ta && bigM && bigN) { *mt = 128; *nt = 64; return; }
  if (bigM && bigN) {
    const int64_t need = ta ? 512 : 256;
    if (tiles_for(M, N, 128, 128) * nsplit >= need) { *mt = 128; *nt = 128; return; }
    if (ta) { *mt = 128; *nt = 128; return; }
    *mt = 64; *nt = 128;
    return;
  }
  *mt = bigM ? 128 : 64;
  *nt = bigN ? 128 : 64;
}

Plan plan_gemm(bool ta, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B, int64_t ldb,
               bool allow_split, size_t part_cap, bool sym = false, bool tri = false, bool skinny_ta = false) {
  Plan p;
  p.dma = dma_eligible(ta, M, K, A, lda, B, ldb);
  const int kt = p.dma ? kDmaKT : kKT;
  p.nsplit = 1;
  p.mt = p.nt = 0;
  // Skinny shapes (block widths up to 32, as in the tall orthogonalisation):
  // exact-width tiles, and for A^T B enough splits of the long reduction for
  // about 2048 workgroups.  Small products that cannot split their reduction
  // (at most 256 x 256: the block Cholesky composition, R_jj = Lb^T L^T) take
  // 32 x 32 tiles, so that 16-64 workgroups share the work instead of 1-4.
  // The truncated SVD's products A^T X with a block of at most 16 columns
  // (skinny_ta) take a 128 x 16 tile, so that every element of A is read once
  // and no MFMA work is spent on padding columns.
  if (p.dma) {
    if (ta && N <= 16 && M <= 64) { p.mt = 16; p.nt = 16; }
    else if (ta && M <= 32 && N <= 32) { p.mt = 32; p.nt = 32; }
    else if ((!ta || skinny_ta) && N <= 16 && M > 64) { p.mt = 128; p.nt = 16; }
    else if (!(allow_split && ta) && M <= 256 && N <= 256) { p.mt = 32; p.nt = 32; }
  }
  if (p.mt != 0) {
    if (allow_split && ta) {
      int64_t sp = 2048 / tiles_for(M, N, p.mt, p.nt);
      const int64_t by_k = K / (8 * kt);
      const int64_t by_cap = (int64_t)(part_cap / (size_t)(M * N));
      if (sp > by_k) sp = by_k;
      if (sp > by_cap) sp = by_cap;
      p.nsplit = sp > 1 ? (int)sp : 1;
    }
    p.kchunk = K > 0 ? K : 1;
    if (p.nsplit > 1) {
      p.kchunk = (K + p.nsplit - 1) / p.nsplit;
      p.kchunk = (p.kchunk + kt - 1) / kt * kt;
      p.nsplit = (int)((K + p.kchunk - 1) / p.kchunk);
    }
    return p;
  }
  if (allow_split && ta) {
    // Split the reduction so that the workgroups fill whole rounds of the
    // 512 resident slots (two per CU) as closely as possible, each split
    // walking at least 8 stages and fitting the partial-sum buffer; among
    // equally full choices the fewest splits win (less reduction traffic).
    int64_t tiles = tiles_for(M, N, M > 64 ? 128 : 64, N > 64 ? 128 : 64);
    if (sym) {
      // Only the tiles on or above the diagonal are formed (symmetric Gram).
      const int64_t tm = (M + 127) / 128;
      if (M > 64) tiles = tm * (tm + 1) / 2;
    }
    int64_t max_split = K / (8 * kt);
    const int64_t by_cap = (int64_t)(part_cap / (size_t)(M * N));
    if (max_split > by_cap) max_split = by_cap;
    if (max_split > 512) max_split = 512;
    double best_eff = 0.0;
    for (int64_t sp = 1; sp <= (max_split < 1 ? 1 : max_split); ++sp) {
      const int64_t wgs = tiles * sp;
      const int64_t rounds = (wgs + 511) / 512;
      const double eff = (double)wgs / (double)(rounds * 512);
      if (eff > best_eff + 0.02) {
        best_eff = eff;
        p.nsplit = (int)sp;
      }
    }
  }
  p.kchunk = K > 0 ? K : 1;
  if (p.nsplit > 1) {
    p.kchunk = (K + p.nsplit - 1) / p.nsplit;
    p.kchunk = (p.kchunk + kt - 1) / kt * kt;
    p.nsplit = (int)((K + p.kchunk - 1) / p.kchunk);
  }
  if (p.dma) {
    pick_tile(ta, M, N, p.nsplit, &p.mt, &p.nt, tri);
  } else {
    p.mt = M > 64 ? 128 : 64;
    p.nt = N > 64 ? 128 : 64;
    if (p.mt == 128 && p.nt == 128 && tiles_for(M, N, 128, 128) * p.nsplit < 512) p.mt = 64;
  }
  return p;
}

template <int ROLE, bool TA, int MT, int NT, int S, int OCC, int WM = 2, int WN = 2, bool F32C = false>
hipError_t launch_dma(const Plan& p, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                      const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* part, const int* gate,
                      hipStream_t s) {
  const dim3 grid((unsigned)((M + MT - 1) / MT), (unsigned)((N + NT - 1) / NT), (unsigned)p.nsplit);
  hipLaunchKernelGGL((gemm_dma_kernel<ROLE, TA, MT, NT, S, OCC, WM, WN, F32C>), grid, dim3(64 * WM * WN), 0, s, M, N, K,
                     alpha, A, lda, B, ldb, beta, C, ldc, p.kchunk, part, gate);
  return hipGetLastError();
}

template <int ROLE, bool TA, int MT, int NT>
hipError_t launch_reg(const Plan& p, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                      const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* part, const int* gate,
                      hipStream_t s) {
  const dim3 grid((unsigned)((M + MT - 1) / MT), (unsigned)((N + NT - 1) / NT), (unsigned)p.nsplit);
  hipLaunchKernelGGL((gemm_reg_kernel<ROLE, TA, MT, NT, kKT>), grid, dim3(kThreads), 0, s, M, N, K, alpha, A, lda,
                     B, ldb, beta, C, ldc, p.kchunk, part, gate);
  return hipGetLastError();
}

// Ring depth / occupancy / wave grid per DMA tile (measured on gfx950 for the
// q x b update and the s x b projection): 128x128 uses a 2-slot ring and 8
// waves (4 x 2 of 32 x 64 for A^T B, 2 x 4 of 64 x 32 for A B), two waves per
// SIMD; the smaller shapes use 4 waves and a 3-slot ring.  F32C selects the
// FP32-arithmetic form of the DMA kernel (the register kernel has none).
template <int ROLE, bool TA, bool F32C = false>
hipError_t launch(const Plan& p, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                  const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* part, const int* gate,
                  hipStream_t s) {
  if (p.dma) {
    if (p.mt == 16) {
      if constexpr (TA)
        return launch_dma<ROLE, TA, 16, 16, 3, 8, 1, 1, F32C>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, part, gate, s);
    }
    if (p.mt == 32)
      return launch_dma<ROLE, TA, 32, 32, 3, 4, 2, 2, F32C>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, part, gate, s);
    if (p.nt == 16 && p.mt == 128)
      return launch_dma<ROLE, TA, 128, 16, 3, 4, 2, 1, F32C>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, part, gate, s);
    if (p.mt == 128 && p.nt == 128) {
      if (TA)
        return launch_dma<ROLE, TA, 128, 128, 2, 2, 4, 2, F32C>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, part, gate, s);
      return launch_dma<ROLE, TA, 128, 128, 2, 2, 2, 4, F32C>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, part, gate, s);
    }
    if (p.mt == 128) return launch_dma<ROLE, TA, 128, 64, 3, 2, 2, 2, F32C>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, part, gate, s);
    if (p.nt == 128) return launch_dma<ROLE, TA, 64, 128, 3, 2, 2, 2, F32C>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, part, gate, s);
    return launch_dma<ROLE, TA, 64, 64, 3, 3, 2, 2, F32C>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, part, gate, s);
  }
  if (p.mt == 128 && p.nt == 128) return launch_reg<ROLE, TA, 128, 128>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, part, gate, s);
  if (p.mt == 128) return launch_reg<ROLE, TA, 128, 64>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, part, gate, s);
  if (p.nt == 128) return launch_reg<ROLE, TA, 64, 128>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, part, gate, s);
  return launch_reg<ROLE, TA, 64, 64>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, part, gate, s);
}

}  // namespace

hipError_t gemm_tn(Role role, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* part, size_t part_cap,
                   const int* gate, hipStream_t s, double flops, bool f32) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (!ld_ok(lda) || !ld_ok(ldb)) return hipErrorInvalidValue;
  // The FP32-arithmetic Gram splits its reduction at most 64 ways (measured
  // on the q x 256 Gram at q = 32768: 64 splits of 512 rows 14.7 ms per
  // low-precision factorisation, 128 of 256 rows 15.7 ms; 82, 96 and 158
  // splits of 400, 352 and 208 rows 19.4-20.6 ms).
  size_t cap = part_cap;
  if (f32 && role == ROLE_GRAM && (size_t)64 * (size_t)(M * N) < cap) cap = (size_t)64 * (size_t)(M * N);
  const Plan p = plan_gemm(true, M, N, K, A, lda, B, ldb, part != nullptr, cap, role == ROLE_GRAM && M == N,
                           false, role == ROLE_APROD);
  const double bytes = 8.0 * ((double)K * M + (double)K * N + (double)M * N * (beta != 0.0 ? 2.0 : 1.0));
  double* pp = p.nsplit > 1 ? part : nullptr;
  const int slot = prof_begin(s);
  hipError_t e;
  if (role == ROLE_GRAM && f32)
    e = launch<ROLE_GRAM, true, true>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, pp, gate, s);
  else if (role == ROLE_GRAM)
    e = launch<ROLE_GRAM, true>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, pp, gate, s);
  else if (role == ROLE_CHOL && f32)
    e = launch<ROLE_CHOL, true, true>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, pp, gate, s);
  else if (role == ROLE_CHOL)
    e = launch<ROLE_CHOL, true>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, pp, gate, s);
  else if (role == ROLE_APROD)
    e = launch<ROLE_APROD, true>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, pp, gate, s);
  else
    e = launch<ROLE_PROJ, true>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, pp, gate, s);
  prof_end(slot, role, s, flops, bytes);
  if (e != hipSuccess || p.nsplit == 1) return e;
  const int64_t total = M * N;
  int64_t blocks = (total + 63) / 64;
  if (blocks > 8192) blocks = 8192;
  // The FP32-arithmetic DMA instances (ROLE_GRAM, ROLE_CHOL with f32) store
  // FP32 partial sums; the register kernel, which has no FP32 form, FP64.
  const bool f32part = f32 && p.dma && (role == ROLE_GRAM || role == ROLE_CHOL);
  const int slot2 = prof_begin(s);
  if (f32part)
    hipLaunchKernelGGL(splitk_reduce_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, M, N, p.nsplit,
                       reinterpret_cast<const float*>(part), alpha, beta, C, ldc, gate);
  else
    hipLaunchKernelGGL(splitk_reduce_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, M, N, p.nsplit,
                       (const double*)part, alpha, beta, C, ldc, gate);
  e = hipGetLastError();
  prof_end(slot2, ROLE_REDUCE, s, 0.0,
           (double)total * ((f32part ? 4.0 : 8.0) * p.nsplit + 8.0 * (beta != 0.0 ? 2 : 1)));
  return e;
}

hipError_t gemm_nn(Role role, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double beta, double* C, int64_t ldc, const int* gate, hipStream_t s,
                   double flops, bool f32) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (!ld_ok(lda) || !ld_ok(ldb)) return hipErrorInvalidValue;
  const Plan p = plan_gemm(false, M, N, K, A, lda, B, ldb, false, 0, false, role == ROLE_TRSM || role == ROLE_SMALL);
  const double bytes = 8.0 * ((double)K * M + (double)K * N + (double)M * N * (beta != 0.0 ? 2.0 : 1.0));
  const int slot = prof_begin(s);
  hipError_t e;
  switch (role) {
    case ROLE_UPDATE:
      e = launch<ROLE_UPDATE, false>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, nullptr, gate, s);
      break;
    case ROLE_TRSM:
      if (f32)
        e = launch<ROLE_TRSM, false, true>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, nullptr, gate, s);
      else
        e = launch<ROLE_TRSM, false>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, nullptr, gate, s);
      break;
    case ROLE_CHOL:
      if (f32)
        e = launch<ROLE_CHOL, false, true>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, nullptr, gate, s);
      else
        e = launch<ROLE_CHOL, false>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, nullptr, gate, s);
      break;
    case ROLE_APROD:
      e = launch<ROLE_APROD, false>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, nullptr, gate, s);
      break;
    case ROLE_SVD:
      e = launch<ROLE_SVD, false>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, nullptr, gate, s);
      break;
    default:
      if (f32)
        e = launch<ROLE_SMALL, false, true>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, nullptr, gate, s);
      else
        e = launch<ROLE_SMALL, false>(p, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, nullptr, gate, s);
      break;
  }
  prof_end(slot, role, s, flops, bytes);
  return e;
}

}  // namespace cqr
