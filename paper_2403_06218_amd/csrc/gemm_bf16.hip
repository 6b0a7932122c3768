// BF16 GEMM on the CDNA4 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation) for the low-precision form of the factorisation: the
// projections H = P^T Q and the updates Q -= P H of Algorithm 5 (S1/S2,
// S6/S7), which carry almost all of its flops (Table 1).
//
// Both operands are "k-contiguous" BF16 matrices: C (M x N) = alpha * A^T B
// + beta * C with A stored K x M and B stored K x N, column-major.  (For the
// update the caller passes the transposed copy of P.)  The host pads K to a
// multiple of 64 with zeros, aligns every column to 16 bytes and gives the
// leading dimensions in multiples of 8 elements.
//
// Tiling: an MT x NT tile per workgroup of WM x WN wave64s (128 x 256 with
// 2 x 4 waves when N > 128, so that a row panel of A is streamed once for the
// whole width; 128 x 128 with 2 x 4 waves; 64-wide tiles with 2 x 2); K is walked in
// 64-deep stages copied global -> LDS by the LDS-DMA load
// (global_load_lds_dwordx4, 16 bytes = 8 BF16 per lane) into an S-slot ring
// with one barrier per stage.  In LDS a column of a stage is 8 chunks of 8
// consecutive k; chunk c of column x sits at slot c ^ ((x >> 1) & 7), so the
// 16 lanes of a 128-bit operand read (16 columns, one chunk) hit 16 distinct
// 16-byte bank groups.
//
// MFMA lane layout (measured on gfx950): lane l supplies A(l%16, 8(l/16)+e)
// and B(8(l/16)+e, l%16), e = 0..7, and holds C(4(l/16)+v, l%16) in
// accumulator element v.
#include <numeric>
#include <type_traits>

#include "internal.h"

namespace cqr {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void lds_void;
typedef unsigned char fp8_t;  // OCP E4M3 byte

constexpr int kBKT = 64;  // k per stage

__device__ __forceinline__ void dma16(const void* g, void* lds_base) {
  __builtin_amdgcn_global_load_lds(g, (lds_void*)lds_base, 16, 0, 0);
}

// The same with the non-temporal hint (cache-policy bit NT): for an operand
// that is streamed once from HBM, so that it does not displace the shared
// operand from L2 (measured: +15-25% on the 128 x 256 tile).
__device__ __forceinline__ void dma16_stream(const void* g, void* lds_base) {
  __builtin_amdgcn_global_load_lds(g, (lds_void*)lds_base, 16, 0, 2);
}

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Barrier between two stages of a ring.  __syncthreads() carries a
// workgroup-scope release fence, which waits for every outstanding memory
// operation of the wave (vmcnt(0)), the LDS-DMA loads of later stages
// included, and so drains the prefetch ring at every stage.  Here each wave
// has already waited for its own loads of the stage about to be read
// (wait_vmcnt), its LDS reads of the stage just computed are complete
// (lgkmcnt(0), so no load issued after the barrier overwrites a slot that is
// still being read), and compiler-only fences keep LDS accesses on their side
// of the hardware barrier.
__device__ __forceinline__ void stage_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt not waited for
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Tile height of the wide kernel: 256 for projections with at least 12288
// rows of output (measured: 5-15% faster there, slower for fewer rows), and
// for BF16 updates of at least 12288 rows, whose reduction the caller then
// splits in two through FP32 partial sums so that the half as many row tiles
// still occupy every CU (measured at q = 32768: the BF16 updates 83 -> 70 ms
// per factorisation, the extra reduction +9 ms; the FP8 updates 46 -> 38 ms
// with the same +9 ms, so they keep the 128-row tile).
int wide_mt(int role, int64_t M, bool fp8) {
  if (M < 12288) return 128;
  return (role == ROLE_PROJ || !fp8) ? 256 : 128;
}

// Byte offset of chunk c (8 k values) of column x in a stage.
__device__ __forceinline__ int chunk_off(int c, int x) { return x * 128 + 16 * (c ^ ((x >> 1) & 7)); }

// OUT: 0 = FP32 partial sums into part (split-K), 1 = FP32 C, 2 = FP64 C.
template <int ROLE, int OUT, int MT, int NT, int S, int WM, int WN, int OCC>
__global__ void __launch_bounds__(64 * WM * WN, OCC)
gemm_bf16_kernel(int64_t M, int64_t N, int64_t K, float alpha, const __bf16* __restrict__ A, int64_t lda,
                 const __bf16* __restrict__ B, int64_t ldb, float beta, void* C, int64_t ldc, int64_t kchunk,
                 float* __restrict__ part, const int* __restrict__ gate) {
  static_assert(S == 2 || S == 3, "ring depth");
  if (gate != nullptr && *gate != 0) return;
  constexpr int NW = WM * WN;
  constexpr int WTM = MT / WM, WTN = NT / WN;
  constexpr int SM = WTM / 16, SN = WTN / 16;
  constexpr int ASTAGE = MT * kBKT * 2, BSTAGE = NT * kBKT * 2;   // bytes per stage
  constexpr int AINS = ASTAGE / 1024 / NW, BINS = BSTAGE / 1024 / NW;
  static_assert(AINS >= 1 && BINS >= 1 && AINS * 1024 * NW == ASTAGE && BINS * 1024 * NW == BSTAGE, "stage split");
  static_assert(SM >= 1 && SN >= 1, "wave tile");
  __shared__ __attribute__((aligned(16))) char sA0[ASTAGE], sA1[ASTAGE], sA2[S > 2 ? ASTAGE : 16];
  __shared__ __attribute__((aligned(16))) char sB0[BSTAGE], sB1[BSTAGE], sB2[S > 2 ? BSTAGE : 16];
  auto slotA = [&](auto c) -> char* {
    if constexpr (c.value == 0) return sA0;
    else if constexpr (c.value == 1) return sA1;
    else return sA2;
  };
  auto slotB = [&](auto c) -> char* {
    if constexpr (c.value == 0) return sB0;
    else if constexpr (c.value == 1) return sB1;
    else return sB2;
  };

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave % WM, wn = wave / WM;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t m0 = (int64_t)blockIdx.x * MT;
  const int64_t n0 = (int64_t)blockIdx.y * NT;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = (K < kbeg + kchunk) ? K : kbeg + kchunk;
  const int nst = (kend > kbeg) ? (int)((kend - kbeg) / kBKT) : 0;

  // Element offsets of this lane's DMA chunks from the stage origin; columns
  // past the matrix are clamped (their values reach only unstored outputs).
  int64_t aoff[AINS], boff[BINS];
#pragma unroll
  for (int t = 0; t < AINS; ++t) {
    const int p = (wave * AINS + t) * 64 + lane;
    const int x = p / 8, c = (p % 8) ^ ((x >> 1) & 7);
    const int64_t m = (m0 + x < M) ? m0 + x : M - 1;
    aoff[t] = 8 * c + m * lda;
  }
#pragma unroll
  for (int t = 0; t < BINS; ++t) {
    const int p = (wave * BINS + t) * 64 + lane;
    const int x = p / 8, c = (p % 8) ^ ((x >> 1) & 7);
    const int64_t n = (n0 + x < N) ? n0 + x : N - 1;
    boff[t] = 8 * c + n * ldb;
  }

  auto issue = [&](int st, auto slot) {
    const int64_t k0 = kbeg + (int64_t)st * kBKT;
    char* la = slotA(slot);
    char* lb = slotB(slot);
#pragma unroll
    for (int t = 0; t < AINS; ++t) dma16(A + k0 + aoff[t], la + (wave * AINS + t) * 1024);
#pragma unroll
    for (int t = 0; t < BINS; ++t) dma16(B + k0 + boff[t], lb + (wave * BINS + t) * 1024);
  };

  f4 acc[SM][SN];
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  auto compute = [&](auto slot) {
    const char* cA = slotA(slot);
    const char* cB = slotB(slot);
#pragma unroll
    for (int h = 0; h < kBKT / 32; ++h) {
      const int c = 4 * h + lg;  // chunk (8 k values) this lane supplies
      bf16x8 af[SM], bf[SN];
#pragma unroll
      for (int i = 0; i < SM; ++i)
        af[i] = *(const bf16x8*)(cA + chunk_off(c, wm * WTM + i * 16 + li));
#pragma unroll
      for (int j = 0; j < SN; ++j)
        bf[j] = *(const bf16x8*)(cB + chunk_off(c, wn * WTN + j * 16 + li));
#pragma unroll
      for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  };

  constexpr int PER_STAGE = AINS + BINS;
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  auto step = [&](int st, auto cur, auto nxt) {
    if (st + S - 2 < nst) wait_vmcnt<(S - 2) * PER_STAGE>();
    else wait_vmcnt<0>();
    stage_barrier();
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
      const int64_t mb = m0 + wm * WTM + i * 16 + 4 * lg;
      if (n >= N) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = mb + v;
        if (m >= M) continue;
        const float val = acc[i][j][v];
        if constexpr (OUT == 0) {
          part[zoff + m + n * M] = val;
        } else if constexpr (OUT == 1) {
          float* Cf = (float*)C;
          float c = alpha * val;
          if (beta != 0.f) c += beta * Cf[m + n * ldc];
          Cf[m + n * ldc] = c;
        } else {
          double* Cd = (double*)C;
          double c = (double)alpha * (double)val;
          if (beta != 0.f) c += (double)beta * Cd[m + n * ldc];
          Cd[m + n * ldc] = c;
        }
      }
    }
}

// 128 x 256 tile with 2 x 4 waves (64 x 64 per wave; MT_ = 256: 256 x 256
// with 128 x 64 per wave, for the projections of the later blocks, whose
// s x b output needs few splits, and for the BF16 updates, split in two along
// k) and the loads split by wave: waves 0-3 copy A
// (the row panel, unique to the workgroup and streamed from HBM, loaded
// non-temporal), waves 4-7 copy B (shared by all workgroups, served by L2),
// each into a ring of SA / SB slots, so each wave's vmcnt counts only its own
// operand.  Each operand is loaded one stage ahead (two slots each): rings
// that let A run further ahead (3-6 slots, with a barrier that does not drain
// the loads) were measured slower, its prefetches delaying the loads of B
// that the next stage waits for, and a deeper B ring did not help.
//
// E is __bf16 (v_mfma_f32_16x16x32_bf16, 64 k per stage) or fp8 (OCP E4M3
// bytes, v_mfma_scale_f32_16x16x128_f8f6f4, 128 k per stage); both give 128 bytes
// per column per stage, so the LDS layout is the same.  rs / cs (may be
// NULL) multiply accumulator row m / column n before alpha: the inverse
// power-of-two scales of the FP8 operands.
template <typename E, int ROLE, int OUT, int SA = 2, int SB = 2, int MT_ = 128>
__global__ void __launch_bounds__(512, 1)
gemm_lp_wide_kernel(int64_t M, int64_t N, int64_t K, float alpha, const E* __restrict__ A, int64_t lda, int64_t a_blk,
                    const E* __restrict__ B, int64_t ldb, float beta, void* C, int64_t ldc, int64_t kchunk,
                    float* __restrict__ part, const float* __restrict__ rs, const float* __restrict__ cs,
                    const int* __restrict__ gate) {
  static_assert(SA >= 2 && SA <= 8 && SB >= 2 && SB <= 4, "ring depths");
  if (gate != nullptr && *gate != 0) return;
  constexpr bool F8 = sizeof(E) == 1;
  constexpr int KST = F8 ? 128 : kBKT;  // k per stage
  constexpr int EPC = F8 ? 16 : 8;      // elements per 16-byte chunk
  static_assert(MT_ == 128 || MT_ == 256, "tile height");
  constexpr int MT = MT_, NT = 256, WM = 2;
  constexpr int WTM = MT / 2, WTN = 64, SM = WTM / 16, SN = 4;
  constexpr int ASTAGE = MT * 128, BSTAGE = NT * 128;
  static_assert(SA * ASTAGE + SB * BSTAGE <= 160 * 1024, "LDS budget");
  constexpr int AINS = ASTAGE / 1024 / 4, BINS = BSTAGE / 1024 / 4;  // DMA instructions per loading wave
  // One LDS object per ring slot (unused slots take 16 bytes).
  constexpr int AS = ASTAGE, BS = BSTAGE;
  __shared__ __attribute__((aligned(16))) char sA0[AS], sA1[AS], sA2[SA > 2 ? AS : 16], sA3[SA > 3 ? AS : 16],
      sA4[SA > 4 ? AS : 16], sA5[SA > 5 ? AS : 16], sA6[SA > 6 ? AS : 16], sA7[SA > 7 ? AS : 16];
  __shared__ __attribute__((aligned(16))) char sB0[BS], sB1[BS], sB2[SB > 2 ? BS : 16], sB3[SB > 3 ? BS : 16];
  auto slotA = [&](auto c) -> char* {
    if constexpr (c.value == 0) return sA0;
    else if constexpr (c.value == 1) return sA1;
    else if constexpr (c.value == 2) return sA2;
    else if constexpr (c.value == 3) return sA3;
    else if constexpr (c.value == 4) return sA4;
    else if constexpr (c.value == 5) return sA5;
    else if constexpr (c.value == 6) return sA6;
    else return sA7;
  };
  auto slotB = [&](auto c) -> char* {
    if constexpr (c.value == 0) return sB0;
    else if constexpr (c.value == 1) return sB1;
    else if constexpr (c.value == 2) return sB2;
    else return sB3;
  };

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool aloader = wave < 4;
  const int lw = aloader ? wave : wave - 4;  // index among the loading waves of its operand
  const int wm = wave % WM, wn = wave / WM;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t m0 = (int64_t)blockIdx.x * MT;
  const int64_t n0 = (int64_t)blockIdx.y * NT;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = (K < kbeg + kchunk) ? K : kbeg + kchunk;
  const int nst = (kend > kbeg) ? (int)((kend - kbeg) / KST) : 0;

  // Source offsets of this lane's chunks (clamped past the matrix edge).
  constexpr int INS = AINS > BINS ? AINS : BINS;
  int64_t off[INS];
#pragma unroll
  for (int t = 0; t < INS; ++t) {
    const int p = (lw * (aloader ? AINS : BINS) + t) * 64 + lane;
    const int x = p / 8, c = (p % 8) ^ ((x >> 1) & 7);
    if (aloader) {
      const int64_t m = (m0 + x < M) ? m0 + x : M - 1;
      off[t] = EPC * c + (a_blk ? (m >> 7) * a_blk + (m & 127) * KST : m * lda);
    } else {
      const int64_t n = (n0 + x < N) ? n0 + x : N - 1;
      off[t] = EPC * c + n * ldb;
    }
  }
  // A tiled (a_blk > 0): stage k0 of a 128-column block is one contiguous
  // 128 x KST tile, so the stage origin moves by 128 KST per stage.
  const int64_t kmul = a_blk ? 128 : 1;
  auto issueA = [&](int st, auto slot) {
    const int64_t k0 = kbeg + (int64_t)st * KST;
    char* la = slotA(slot);
#pragma unroll
    for (int t = 0; t < AINS; ++t) dma16_stream(A + k0 * kmul + off[t], la + (lw * AINS + t) * 1024);
  };
  auto issueB = [&](int st, auto slot) {
    const int64_t k0 = kbeg + (int64_t)st * KST;
    char* lb = slotB(slot);
#pragma unroll
    for (int t = 0; t < BINS; ++t) dma16(B + k0 + off[t], lb + (lw * BINS + t) * 1024);
  };

  f4 acc[SM][SN];
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  auto compute = [&](auto sa, auto sb) {
    const char* cA = slotA(sa);
    const char* cB = slotB(sb);
    if constexpr (F8) {
      // One v_mfma_scale_f32_16x16x128_f8f6f4 (E4M3 operands, unit scales)
      // per tile and stage, a quarter of the instructions of the 16x16x32
      // form at twice its rate.  The instruction takes 32 k-bytes of its row
      // of A and column of B from each lane group lg; here they are the
      // 16-byte chunks lg and lg + 4 of the stage, read as two 128-bit reads
      // whose addresses follow the BF16 operand reads exactly (lane group lg
      // on chunk c0 + lg of an aligned run of four), the pattern that keeps
      // those reads free of bank conflicts.  A and B share this k order,
      // which is all the product needs.
      typedef int i4v __attribute__((ext_vector_type(4)));
      auto frag = [&](const char* base, int x) {
        const i4v lo = *(const i4v*)(base + chunk_off(lg, x));
        const i4v hi = *(const i4v*)(base + chunk_off(lg + 4, x));
        v8i f;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          f[e] = lo[e];
          f[4 + e] = hi[e];
        }
        return f;
      };
      v8i bf[SN];
#pragma unroll
      for (int j = 0; j < SN; ++j) bf[j] = frag(cB, wn * WTN + j * 16 + li);
#pragma unroll
      for (int i = 0; i < SM; ++i) {
        const v8i af = frag(cA, wm * WTM + i * 16 + li);
#pragma unroll
        for (int j = 0; j < SN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(af, bf[j], acc[i][j], 0, 0, 0, 127, 0, 127);
      }
    } else {
#pragma unroll
      for (int h = 0; h < kBKT / 32; ++h) {
        const int c = 4 * h + lg;
        bf16x8 af[SM], bf[SN];
#pragma unroll
        for (int i = 0; i < SM; ++i) af[i] = *(const bf16x8*)(cA + chunk_off(c, wm * WTM + i * 16 + li));
#pragma unroll
        for (int j = 0; j < SN; ++j) bf[j] = *(const bf16x8*)(cB + chunk_off(c, wn * WTN + j * 16 + li));
#pragma unroll
        for (int i = 0; i < SM; ++i)
#pragma unroll
          for (int j = 0; j < SN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
    }
  };

  // Step st: wait for stage st of this wave's operand, barrier, refill the
  // slots freed by step st-1, compute stage st.  Stage st sits in A slot
  // st % SA and B slot st % SB.
  using std::integral_constant;
  auto step = [&](int st, auto ca, auto na, auto cb, auto nb) {
    if (aloader) {
      if (st + SA - 2 < nst) wait_vmcnt<(SA - 2) * AINS>();
      else wait_vmcnt<0>();
    } else {
      if (st + SB - 2 < nst) wait_vmcnt<(SB - 2) * BINS>();
      else wait_vmcnt<0>();
    }
    stage_barrier();
    if (aloader) {
      if (st + SA - 1 < nst) issueA(st + SA - 1, na);
    } else {
      if (st + SB - 1 < nst) issueB(st + SB - 1, nb);
    }
    compute(ca, cb);
  };
  auto prologue = [&](auto u) {
    if constexpr (u.value < SA - 1) {
      if (aloader && nst > u.value) issueA(u.value, u);
    }
    if constexpr (u.value < SB - 1) {
      if (!aloader && nst > u.value) issueB(u.value, u);
    }
  };
  prologue(integral_constant<int, 0>{});
  prologue(integral_constant<int, 1>{});
  prologue(integral_constant<int, 2>{});
  prologue(integral_constant<int, 3>{});
  prologue(integral_constant<int, 4>{});
  prologue(integral_constant<int, 5>{});
  prologue(integral_constant<int, 6>{});
  // The main loop is unrolled over L = lcm(SA, SB) stages so that every slot
  // index is a compile-time constant.
  constexpr int L = std::lcm(SA, SB);
  auto unit = [&](int st0, auto u) {
    if constexpr (u.value < L) {
      constexpr int ua = u.value % SA, ub = u.value % SB;
      if (st0 + u.value < nst)
        step(st0 + u.value, integral_constant<int, ua>{}, integral_constant<int, (ua + SA - 1) % SA>{},
             integral_constant<int, ub>{}, integral_constant<int, (ub + SB - 1) % SB>{});
    }
  };
  for (int st = 0; st < nst; st += L) {
    static_assert(L <= 24, "unroll length");
    unit(st, integral_constant<int, 0>{}); unit(st, integral_constant<int, 1>{});
    unit(st, integral_constant<int, 2>{}); unit(st, integral_constant<int, 3>{});
    unit(st, integral_constant<int, 4>{}); unit(st, integral_constant<int, 5>{});
    unit(st, integral_constant<int, 6>{}); unit(st, integral_constant<int, 7>{});
    unit(st, integral_constant<int, 8>{}); unit(st, integral_constant<int, 9>{});
    unit(st, integral_constant<int, 10>{}); unit(st, integral_constant<int, 11>{});
    unit(st, integral_constant<int, 12>{}); unit(st, integral_constant<int, 13>{});
    unit(st, integral_constant<int, 14>{}); unit(st, integral_constant<int, 15>{});
    unit(st, integral_constant<int, 16>{}); unit(st, integral_constant<int, 17>{});
    unit(st, integral_constant<int, 18>{}); unit(st, integral_constant<int, 19>{});
    unit(st, integral_constant<int, 20>{}); unit(st, integral_constant<int, 21>{});
    unit(st, integral_constant<int, 22>{}); unit(st, integral_constant<int, 23>{});
  }

  const int64_t zoff = (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) {
      const int64_t n = n0 + wn * WTN + j * 16 + li;
      const int64_t mb = m0 + wm * WTM + i * 16 + 4 * lg;
      if (n >= N) continue;
      const float csn = cs ? cs[n] : 1.f;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = mb + v;
        if (m >= M) continue;
        const float val = acc[i][j][v] * (rs ? rs[m] : 1.f) * csn;
        if constexpr (OUT == 0) {
          part[zoff + m + n * M] = val;
        } else if constexpr (OUT == 1) {
          float* Cf = (float*)C;
          float c = alpha * val;
          if (beta != 0.f) c += beta * Cf[m + n * ldc];
          Cf[m + n * ldc] = c;
        } else {
          double* Cd = (double*)C;
          double c = (double)alpha * (double)val;
          if (beta != 0.f) c += (double)beta * Cd[m + n * ldc];
          Cd[m + n * ldc] = c;
        }
      }
    }
}

// C (FP32 or FP64) = alpha * sum_z part[z] + beta * C, in split order.
template <typename TC>
__global__ void __launch_bounds__(256)
splitk_reduce_f32_kernel(int64_t M, int64_t N, int nsplit, const float* __restrict__ part, float alpha, float beta,
                         TC* C, int64_t ldc, const int* __restrict__ gate) {
  if (gate != nullptr && *gate != 0) return;
  const int64_t total = M * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    TC s = 0;
    for (int z = 0; z < nsplit; ++z) s += (TC)part[(int64_t)z * total + idx];
    const int64_t m = idx % M, n = idx / M;
    TC c = (TC)alpha * s;
    if (beta != 0.f) c += (TC)beta * C[m + n * ldc];
    C[m + n * ldc] = c;
  }
}

template <int ROLE, int OUT, int MT, int NT>
hipError_t launch_bf16(int64_t M, int64_t N, int64_t K, float alpha, const __bf16* A, int64_t lda, const __bf16* B,
                       int64_t ldb, float beta, void* C, int64_t ldc, int64_t kchunk, int nsplit, float* part,
                       const int* gate, hipStream_t s) {
  constexpr bool big = MT == 128 && NT >= 128;
  constexpr int WM = 2;
  constexpr int WN = big ? 4 : 2;
  constexpr int OCC = big ? 1 : 2;
  const dim3 grid((unsigned)((M + MT - 1) / MT), (unsigned)((N + NT - 1) / NT), (unsigned)nsplit);
  hipLaunchKernelGGL((gemm_bf16_kernel<ROLE, OUT, MT, NT, 3, WM, WN, OCC>), grid, dim3(64 * WM * WN), 0, s, M, N, K,
                     alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part, gate);
  return hipGetLastError();
}

template <int ROLE, int OUT>
hipError_t launch_bf16_tile(int64_t M, int64_t N, int64_t K, float alpha, const __bf16* A, int64_t lda,
                            int64_t a_blk, const __bf16* B, int64_t ldb, float beta, void* C, int64_t ldc,
                            int64_t kchunk, int nsplit, float* part, const int* gate, hipStream_t s) {
  // A tiled A is read by the wide kernel only (columns past M or N are
  // clamped and not stored, so any shape fits it).
  if ((M > 64 && N > 128) || a_blk > 0) {
    {
      if (wide_mt(ROLE, M, false) == 256) {
        const dim3 grid((unsigned)((M + 255) / 256), (unsigned)((N + 255) / 256), (unsigned)nsplit);
        hipLaunchKernelGGL((gemm_lp_wide_kernel<__bf16, ROLE, OUT, 2, 2, 256>), grid, dim3(512), 0, s, M, N, K, alpha,
                           A, lda, a_blk, B, ldb, beta, C, ldc, kchunk, part, (const float*)nullptr, (const float*)nullptr,
                           gate);
        return hipGetLastError();
      }
    }
    const dim3 grid((unsigned)((M + 127) / 128), (unsigned)((N + 255) / 256), (unsigned)nsplit);
    hipLaunchKernelGGL((gemm_lp_wide_kernel<__bf16, ROLE, OUT>), grid, dim3(512), 0, s, M, N, K, alpha, A, lda, a_blk,
                       B, ldb, beta, C, ldc, kchunk, part, (const float*)nullptr, (const float*)nullptr, gate);
    return hipGetLastError();
  }
  if (M > 64 && N > 64)
    return launch_bf16<ROLE, OUT, 128, 128>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, nsplit, part, gate,
                                            s);
  if (M > 64)
    return launch_bf16<ROLE, OUT, 128, 64>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, nsplit, part, gate,
                                           s);
  if (N > 64)
    return launch_bf16<ROLE, OUT, 64, 128>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, nsplit, part, gate,
                                           s);
  return launch_bf16<ROLE, OUT, 64, 64>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, nsplit, part, gate, s);
}

int64_t bf16_tiles(int role, int64_t M, int64_t N, bool force_wide) {
  const bool wide = (M > 64 && N > 128) || force_wide;
  const int64_t mt = wide ? wide_mt(role, M, false) : (M > 64 ? 128 : 64), nt = wide ? 256 : (N > 64 ? 128 : 64);
  return ((M + mt - 1) / mt) * ((N + nt - 1) / nt);
}

}  // namespace

bool gemm_bf16_supported(const void* A, int64_t lda, const void* B, int64_t ldb, int64_t K) {
  return !(reinterpret_cast<uintptr_t>(A) & 15) && !(reinterpret_cast<uintptr_t>(B) & 15) && lda % 8 == 0 &&
         ldb % 8 == 0 && K % kBKT == 0;
}

hipError_t gemm_bf16_tn(Role role, int64_t M, int64_t N, int64_t K, float alpha, const __bf16* A, int64_t lda,
                        int64_t a_blk, const __bf16* B, int64_t ldb, float beta, void* C, int64_t ldc, bool c_is_f64,
                        float* part, size_t part_cap, const int* gate, hipStream_t s, double flops) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (!gemm_bf16_supported(A, a_blk ? 8 : lda, B, ldb, K)) return hipErrorInvalidValue;
  if (a_blk < 0 || a_blk % (128 * kBKT) != 0) return hipErrorInvalidValue;
  // Split-K through FP32 partial sums: fill whole rounds of 256 resident
  // workgroups, each walking at least 4 stages, within the partial buffer.
  int nsplit = 1;
  if (part != nullptr) {
    const int64_t tiles = bf16_tiles(role, M, N, a_blk > 0);
    int64_t max_split = K / (4 * kBKT);
    const int64_t by_cap = (int64_t)(part_cap / (size_t)(M * N));
    if (max_split > by_cap) max_split = by_cap;
    if (max_split > 256) max_split = 256;
    double best = 0.0;
    for (int64_t sp = 1; sp <= (max_split < 1 ? 1 : max_split); ++sp) {
      const int64_t wgs = tiles * sp;
      const int64_t rounds = (wgs + 255) / 256;
      const double eff = (double)wgs / (double)(rounds * 256);
      if (eff > best + 0.02) {
        best = eff;
        nsplit = (int)sp;
      }
    }
  }
  int64_t kchunk = K > 0 ? K : kBKT;
  if (nsplit > 1) {
    kchunk = (K + nsplit - 1) / nsplit;
    kchunk = (kchunk + kBKT - 1) / kBKT * kBKT;
    nsplit = (int)((K + kchunk - 1) / kchunk);
  }
  const double bytes = 2.0 * ((double)K * M + (double)K * N) + (c_is_f64 ? 8.0 : 4.0) * (double)M * N *
                                                                  (beta != 0.f ? 2.0 : 1.0);
  const int slot = prof_begin(s);
  hipError_t e;
  if (nsplit > 1)
    e = (role == ROLE_UPDATE)
            ? launch_bf16_tile<ROLE_UPDATE, 0>(M, N, K, alpha, A, lda, a_blk, B, ldb, beta, C, ldc, kchunk, nsplit, part,
                                               gate, s)
            : launch_bf16_tile<ROLE_PROJ, 0>(M, N, K, alpha, A, lda, a_blk, B, ldb, beta, C, ldc, kchunk, nsplit, part, gate,
                                             s);
  else if (c_is_f64)
    e = (role == ROLE_UPDATE)
            ? launch_bf16_tile<ROLE_UPDATE, 2>(M, N, K, alpha, A, lda, a_blk, B, ldb, beta, C, ldc, kchunk, 1, part, gate, s)
            : launch_bf16_tile<ROLE_PROJ, 2>(M, N, K, alpha, A, lda, a_blk, B, ldb, beta, C, ldc, kchunk, 1, part, gate, s);
  else
    e = (role == ROLE_UPDATE)
            ? launch_bf16_tile<ROLE_UPDATE, 1>(M, N, K, alpha, A, lda, a_blk, B, ldb, beta, C, ldc, kchunk, 1, part, gate, s)
            : launch_bf16_tile<ROLE_PROJ, 1>(M, N, K, alpha, A, lda, a_blk, B, ldb, beta, C, ldc, kchunk, 1, part, gate, s);
  prof_end(slot, role, s, flops, bytes);
  if (e != hipSuccess || nsplit == 1) return e;
  const int64_t total = M * N;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  const int slot2 = prof_begin(s);
  if (c_is_f64)
    hipLaunchKernelGGL(splitk_reduce_f32_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, M, N, nsplit, part,
                       alpha, beta, (double*)C, ldc, gate);
  else
    hipLaunchKernelGGL(splitk_reduce_f32_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, M, N, nsplit, part,
                       alpha, beta, (float*)C, ldc, gate);
  e = hipGetLastError();
  prof_end(slot2, ROLE_REDUCE, s, 0.0, 4.0 * (double)total * (nsplit + (beta != 0.f ? 2 : 1)));
  return e;
}

bool gemm_fp8_supported(const void* A, int64_t lda, const void* B, int64_t ldb, int64_t K) {
  return !(reinterpret_cast<uintptr_t>(A) & 15) && !(reinterpret_cast<uintptr_t>(B) & 15) && lda % 16 == 0 &&
         ldb % 16 == 0 && K % 128 == 0;
}

hipError_t gemm_fp8_tn(Role role, int64_t M, int64_t N, int64_t K, float alpha, const uint8_t* A, int64_t lda,
                       int64_t a_blk, const uint8_t* B, int64_t ldb, float beta, void* C, int64_t ldc, bool c_is_f64,
                       const float* rs, const float* cs, float* part, size_t part_cap, const int* gate, hipStream_t s,
                       double flops) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (!gemm_fp8_supported(A, a_blk ? 16 : lda, B, ldb, K)) return hipErrorInvalidValue;
  if (a_blk < 0 || a_blk % (128 * 128) != 0) return hipErrorInvalidValue;
  // The wide tile (columns past N are clamped and not stored), 128 or 256 rows.
  const int mt = wide_mt(role, M, true);
  int nsplit = 1;
  if (part != nullptr) {
    const int64_t tiles = ((M + mt - 1) / mt) * ((N + 255) / 256);
    int64_t max_split = K / (4 * 128);
    const int64_t by_cap = (int64_t)(part_cap / (size_t)(M * N));
    if (max_split > by_cap) max_split = by_cap;
    if (max_split > 256) max_split = 256;
    double best = 0.0;
    for (int64_t sp = 1; sp <= (max_split < 1 ? 1 : max_split); ++sp) {
      const int64_t wgs = tiles * sp;
      const int64_t rounds = (wgs + 255) / 256;
      const double eff = (double)wgs / (double)(rounds * 256);
      if (eff > best + 0.02) {
        best = eff;
        nsplit = (int)sp;
      }
    }
  }
  int64_t kchunk = K > 0 ? K : 128;
  if (nsplit > 1) {
    kchunk = (K + nsplit - 1) / nsplit;
    kchunk = (kchunk + 127) / 128 * 128;
    nsplit = (int)((K + kchunk - 1) / kchunk);
  }
  const double bytes = ((double)K * M + (double)K * N) + (c_is_f64 ? 8.0 : 4.0) * (double)M * N *
                                                          (beta != 0.f ? 2.0 : 1.0);
  const dim3 grid((unsigned)((M + mt - 1) / mt), (unsigned)((N + 255) / 256), (unsigned)nsplit);
  const fp8_t* a8 = (const fp8_t*)A;
  const fp8_t* b8 = (const fp8_t*)B;
  const int slot = prof_begin(s);
  if (mt == 256) {
    if (nsplit > 1)
      hipLaunchKernelGGL((gemm_lp_wide_kernel<fp8_t, ROLE_PROJ, 0, 2, 2, 256>), grid, dim3(512), 0, s, M, N, K, alpha,
                         a8, lda, a_blk, b8, ldb, beta, C, ldc, kchunk, part, rs, cs, gate);
    else if (c_is_f64)
      hipLaunchKernelGGL((gemm_lp_wide_kernel<fp8_t, ROLE_PROJ, 2, 2, 2, 256>), grid, dim3(512), 0, s, M, N, K, alpha,
                         a8, lda, a_blk, b8, ldb, beta, C, ldc, kchunk, part, rs, cs, gate);
    else
      return hipErrorInvalidValue;
  } else if (nsplit > 1) {
    if (role == ROLE_UPDATE)
      hipLaunchKernelGGL((gemm_lp_wide_kernel<fp8_t, ROLE_UPDATE, 0>), grid, dim3(512), 0, s, M, N, K, alpha, a8, lda, a_blk,
                         b8, ldb, beta, C, ldc, kchunk, part, rs, cs, gate);
    else
      hipLaunchKernelGGL((gemm_lp_wide_kernel<fp8_t, ROLE_PROJ, 0>), grid, dim3(512), 0, s, M, N, K, alpha, a8, lda, a_blk,
                         b8, ldb, beta, C, ldc, kchunk, part, rs, cs, gate);
  } else if (c_is_f64) {
    if (role == ROLE_UPDATE)
      hipLaunchKernelGGL((gemm_lp_wide_kernel<fp8_t, ROLE_UPDATE, 2>), grid, dim3(512), 0, s, M, N, K, alpha, a8, lda, a_blk,
                         b8, ldb, beta, C, ldc, kchunk, part, rs, cs, gate);
    else
      hipLaunchKernelGGL((gemm_lp_wide_kernel<fp8_t, ROLE_PROJ, 2>), grid, dim3(512), 0, s, M, N, K, alpha, a8, lda, a_blk,
                         b8, ldb, beta, C, ldc, kchunk, part, rs, cs, gate);
  } else {
    return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  prof_end(slot, role, s, flops, bytes);
  if (e != hipSuccess || nsplit == 1) return e;
  const int64_t total = M * N;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  const int slot2 = prof_begin(s);
  hipLaunchKernelGGL(splitk_reduce_f32_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, M, N, nsplit, part,
                     alpha, beta, (double*)C, ldc, gate);
  e = hipGetLastError();
  prof_end(slot2, ROLE_REDUCE, s, 0.0, 4.0 * (double)total * (nsplit + (beta != 0.f ? 2 : 1)));
  return e;
}

}  // namespace cqr
