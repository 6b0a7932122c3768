// Batched form: CGS-QR (Algorithms 3-5) and the solve x = R^{-1} Q^T b for
// many independent square systems of uneven size (n <= 512), FP64 or FP32.
//
// One workgroup owns one matrix from start to finish.  A persistent grid
// pulls matrix indices from a device counter over an order sorted by
// decreasing n, so the largest matrices start first and the tail is short.
// Sizes are grouped into buckets; each bucket runs the kernel instance
// (block width, waves per workgroup) chosen for it, one persistent launch per
// bucket in use.
//
// Per column block (width w <= BW, padded to wp = 16 or 32 with identity in
// the Gram):
//   * the block lives in LDS (swizzled so that both row- and column-wise MFMA
//     operand reads are free of bank conflicts);
//   * projection H = P^T Q_j (Alg. 5 S1/S6) and update Q_j -= P H (S2/S7)
//     run on MFMA in chunks of 64 finished columns, P read from global memory
//     (L2), the update accumulated in registers and applied at the end of the
//     pass (classical Gram-Schmidt: all projections of a pass use the same
//     Q_j);
//   * Gram W = Q_j^T Q_j on MFMA, Cholesky in one wave (registers, readlane),
//     TRSM Q_j := Q_j L^{-T} one row per thread (Alg. 4 S1-S3, Alg. 5 S3-S5);
//   * R_jj = Lbar^T L^T and H := H + Hbar L^T (corrected S11/S12);
//   * a Cholesky breakdown redoes the block column by column by CGS2
//     (Alg. 5 with b = 1), in the kernel.
// The solve keeps y = Q^T b in LDS, filled block by block, and back
// substitutes with R block by block at the end.
#include <cstring>
#include <mutex>

#include "internal.h"
#include "wave_chol.h"
#include "../../include/cqr.h"

namespace cqr {
namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T>
struct Mf;
template <>
struct Mf<double> {
  using V = d4v;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // Row of accumulator element v in lane group g = lane / 16 (column lane % 16).
  static __device__ __forceinline__ int crow(int g, int v) { return g + 4 * v; }
  static __device__ __forceinline__ double rl(double x, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
  }
};
template <>
struct Mf<float> {
  using V = f4v;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int crow(int g, int v) { return 4 * g + v; }
  static __device__ __forceinline__ float rl(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
  }
};

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Swizzled LDS index of (row, col) in a row-major array with ld columns
// (ld a multiple of 16).
__device__ __forceinline__ int sw(int row, int col, int ld) { return row * ld + (col ^ (row & 15)); }

constexpr int kMaxBuckets = 8;
constexpr int kBatchNMax = 512;

struct BatchArgs {
  const int32_t* n;
  void* const* A;
  const int32_t* lda;
  void* const* R;
  const int32_t* ldr;
  void* const* B;
  int32_t* info;
  int32_t* flags;
  const int32_t* order;
  const int32_t* range;   // [2 * bucket]: start, end in `order`
  int32_t* counter;       // one per bucket
  int bucket;
  int bw;                 // block width, 16 or 32 (<= BW)
};

// Cholesky W = L L^T of the leading WP x WP part of sW (row-major, ld BW+1),
// by wave 0 (lane i holds row i; see wave_chol).  Writes L (row-major, ld
// BW+1, zero above the diagonal) and 1/L_kk.  Returns false on a pivot that is
// not > 0 (NaN too).
template <typename T, int WP, int BW>
__device__ bool chol_wave(const T* sW, T* sL, T* sDinv, int lane) {
  constexpr int LDW = BW + 1;
  T a[WP];
  const bool own = lane < WP;
#pragma unroll
  for (int j = 0; j < WP; ++j) a[j] = own ? sW[lane * LDW + j] : T(0);
  T lii, linv;
  const bool ok = wave_chol<T, WP>(a, lii, linv, lane);
  if (own) {
#pragma unroll
    for (int j = 0; j < WP; ++j) sL[lane * LDW + j] = (j < lane) ? a[j] : ((j == lane) ? lii : T(0));
    sDinv[lane] = linv;
  }
  return ok;
}

// Q_j := Q_j L^{-T} row by row (forward substitution x L^T = q).
template <typename T, int WP, int BW>
__device__ void trsm_rows(T* sQ, const T* sL, const T* sDinv, int n, int tid, int nt) {
  constexpr int LDW = BW + 1;
  for (int r = tid; r < n; r += nt) {
    // Keeps the compiler from hoisting all WP^2/2 loads of L out of the loop.
    asm volatile("" ::: "memory");
    T x[WP];
#pragma unroll
    for (int c = 0; c < WP; ++c) x[c] = sQ[sw(r, c, BW)];
#pragma unroll
    for (int c = 0; c < WP; ++c) {
      T t = x[c];
#pragma unroll
      for (int p = 0; p < c; ++p) t -= x[p] * sL[c * LDW + p];
      x[c] = t * sDinv[c];
    }
#pragma unroll
    for (int c = 0; c < WP; ++c) sQ[sw(r, c, BW)] = x[c];
  }
}

template <typename T, int NMAX, int BW, int NW, int OCC = (NW == 4 && NMAX <= 128) ? 2 : 1, int PBF = 0>
__global__ __launch_bounds__(NW * 64, OCC) void batch_kernel(BatchArgs ar) {
  static_assert(BW == 16 || BW == 32, "block width");
  constexpr int NT = NW * 64;
  constexpr int LDW = BW + 1;
  constexpr int MAXRT = (NMAX / 16 + NW - 1) / NW;  // update row tiles per wave
  constexpr int MAXCT = BW / 16;
  constexpr int RSZ = (NW * 256 > NMAX ? NW * 256 : NMAX);
  // Two chunk buffers when they fit beside the block, else one.
  constexpr int PB = PBF ? PBF : (((2 * NMAX * 16 + NMAX * BW) * (int)sizeof(T) <= 100 * 1024) ? 2 : 1);
  constexpr int TPC = NT / 16;                   // loader threads per chunk column
  constexpr int PRE = (NMAX + TPC - 1) / TPC;    // chunk elements per loader thread
  using V = typename Mf<T>::V;

  __shared__ T sQ[NMAX * BW];
  __shared__ T sP[PB][NMAX * 16];  // 16 finished columns of P (swizzled, ld 16)
  // The projection of one chunk (chunk loop) and the Gram (after it) share storage.
  __shared__ T sHW[(16 * BW > BW * LDW) ? 16 * BW : BW * LDW];
  T* const sH = sHW;
  T* const sW = sHW;
  __shared__ T sR2[RSZ];           // projection / Gram partial tiles; fallback projections
  __shared__ T sL[2][BW * LDW];
  __shared__ T sDinv[2][BW];
  // y = Q^T b waits in the subdiagonal of R (R(c + 1, c) holds y_c; the last
  // entry here) until the back substitution, which restores the zeros.
  __shared__ T sYlast;
  __shared__ T sRed[NW];
  __shared__ int sInt[2];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int r0 = ar.range[2 * ar.bucket], r1 = ar.range[2 * ar.bucket + 1];

  for (;;) {
    if (tid == 0) sInt[0] = atomicAdd(ar.counter + ar.bucket, 1);
    __syncthreads();
    const int kidx = sInt[0];
    __syncthreads();
    if (kidx >= r1 - r0) break;
    const int m = ar.order[r0 + kidx];
    const int n = ar.n[m];
    const int lda = ar.lda[m], ldr = ar.ldr[m];
    T* A = (T*)ar.A[m];
    T* R = (T*)ar.R[m];
    T* Bv = ar.B ? (T*)ar.B[m] : nullptr;
    const int np = (n + 15) & ~15;
    const int bw = ar.bw;
    const int nblk = (n + bw - 1) / bw;
    int info = 0, flags = 0;

    for (int j = 0; j < nblk; ++j) {
      const int s = j * bw;
      const int w = min(bw, n - s);
      const int wp = (w + 15) & ~15;
      const int nct = wp >> 4;
      // Load the block (zero rows >= n and columns >= w).
      for (int e = tid; e < np * wp; e += NT) {
        const int r = e % np, c = e / np;
        sQ[sw(r, c, BW)] = (r < n && c < w) ? A[(size_t)r + (size_t)(s + c) * lda] : T(0);
      }
      __syncthreads();

      bool ok = true;
      for (int pass = 0; pass < 2 && ok; ++pass) {
        if (s > 0) {
          V acc[MAXRT][MAXCT];
#pragma unroll
          for (int t = 0; t < MAXRT; ++t)
#pragma unroll
            for (int c = 0; c < MAXCT; ++c) acc[t][c] = V{};
          // Chunks of 16 finished columns: staged in LDS (loads of chunk ch+1 in
          // flight in registers while chunk ch is used), projection split
          // over rows across waves with partial tiles summed in a fixed order,
          // update accumulated in registers.
          const int nch = s >> 4;
          const int lc = tid / TPC, lr = tid - lc * TPC;
          const int ks = NW / nct;  // waves per projection tile
          // Two chunks of loads in flight: ring slot q holds chunk ch (q = ch % 2)
          // and is refilled with chunk ch + 2 once stored to LDS.
          T ring0[PRE], ring1[PRE];
          auto gload = [&](int ch, T (&pre)[PRE]) {
            const T* pc = A + (size_t)(16 * ch + lc) * lda;
#pragma unroll
            for (int u = 0; u < PRE; ++u) {
              const int r = lr + TPC * u;
              pre[u] = (r < n) ? pc[r] : T(0);
            }
          };
          auto body = [&](int ch, T (&pre)[PRE]) {
            T* buf = sP[(PB == 2) ? (ch & 1) : 0];
#pragma unroll
            for (int u = 0; u < PRE; ++u) {
              const int r = lr + TPC * u;
              if (r < np) buf[sw(r, lc, 16)] = pre[u];
            }
            // The second pass adds to the R entries the first pass wrote: fetch
            // this thread's ones now (16 w <= 16 BW entries per chunk).
            T rprev[(16 * BW + NT - 1) / NT];
            if (pass == 1) {
#pragma unroll
              for (int u = 0; u < (16 * BW + NT - 1) / NT; ++u) {
                const int e = tid + u * NT;
                rprev[u] = (e < 16 * w) ? R[(size_t)(16 * ch + (e & 15)) + (size_t)(s + (e >> 4)) * ldr] : T(0);
              }
            }
            __syncthreads();
            if (ch + 2 < nch) gload(ch + 2, pre);
            {
              const int ct = wave / ks, kp = wave - ct * ks;
              V h = V{};
              for (int m16 = 16 * kp; m16 < np; m16 += 16 * ks) {
                const int rb = m16 + 4 * lg;
#pragma unroll
                for (int t = 0; t < 4; ++t)
                  h = Mf<T>::mma(buf[sw(rb + t, li, 16)], sQ[sw(rb + t, 16 * ct + li, BW)], h);
              }
#pragma unroll
              for (int v = 0; v < 4; ++v) sR2[wave * 256 + Mf<T>::crow(lg, v) * 16 + li] = h[v];
            }
            __syncthreads();
            for (int e = tid; e < 16 * wp; e += NT) {
              const int k = e & 15, c = e >> 4, ct = c >> 4;
              T v = T(0);
              for (int q = 0; q < ks; ++q) v += sR2[(ct * ks + q) * 256 + k * 16 + (c & 15)];
              sH[sw(k, c, BW)] = v;
              if (pass == 0 && c < w) R[(size_t)(16 * ch + k) + (size_t)(s + c) * ldr] = v;
            }
            __syncthreads();
            if (pass == 1) {
              // H := H + Hbar L^T for this chunk's rows (L of the first pass).
#pragma unroll
              for (int u = 0; u < (16 * BW + NT - 1) / NT; ++u) {
                const int e = tid + u * NT;
                if (e < 16 * w) {
                  const int k = e & 15, c = e >> 4;
                  T add = T(0);
                  for (int p = 0; p <= c; ++p) add += sH[sw(k, p, BW)] * sL[0][c * LDW + p];
                  R[(size_t)(16 * ch + k) + (size_t)(s + c) * ldr] = rprev[u] + add;
                }
              }
            }
#pragma unroll
            for (int kk = 0; kk < 16; kk += 4) {
              T bv[MAXCT];
#pragma unroll
              for (int c = 0; c < MAXCT; ++c) bv[c] = (c < nct) ? sH[sw(kk + lg, 16 * c + li, BW)] : T(0);
#pragma unroll
              for (int t = 0; t < MAXRT; ++t) {
                const int rt = wave + t * NW;
                if (16 * rt < np) {
                  const T av = buf[sw(16 * rt + li, kk + lg, 16)];
#pragma unroll
                  for (int c = 0; c < MAXCT; ++c)
                    if (c < nct) acc[t][c] = Mf<T>::mma(av, bv[c], acc[t][c]);
                }
              }
            }
            if (PB == 1) __syncthreads();  // the single buffer is refilled next
          };
          gload(0, ring0);
          if (nch > 1) gload(1, ring1);
          for (int ch = 0; ch < nch; ch += 2) {
            body(ch, ring0);
            if (ch + 1 < nch) body(ch + 1, ring1);
          }
          // Apply the update (each wave owns its row tiles).
#pragma unroll
          for (int t = 0; t < MAXRT; ++t) {
            const int rt = wave + t * NW;
            if (16 * rt < np) {
#pragma unroll
              for (int c = 0; c < MAXCT; ++c)
                if (c < nct) {
#pragma unroll
                  for (int v = 0; v < 4; ++v) {
                    const int r = 16 * rt + Mf<T>::crow(lg, v);
                    sQ[sw(r, 16 * c + li, BW)] -= acc[t][c][v];
                  }
                }
            }
          }
          __syncthreads();
        }
        // Gram W = Q_j^T Q_j: tiles x row-splits = NW units.
        {
          const int tiles = nct * nct;
          const int ks = NW / tiles;
          const int tile = wave / ks, kp = wave - tile * ks;
          const int ta = tile / nct, tb = tile - ta * nct;
          V g = V{};
          for (int m16 = 16 * kp; m16 < np; m16 += 16 * ks) {
            const int rb = m16 + 4 * lg;
#pragma unroll
            for (int t = 0; t < 4; ++t)
              g = Mf<T>::mma(sQ[sw(rb + t, 16 * ta + li, BW)], sQ[sw(rb + t, 16 * tb + li, BW)], g);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) sR2[wave * 256 + Mf<T>::crow(lg, v) * 16 + li] = g[v];
          __syncthreads();
          for (int e = tid; e < wp * wp; e += NT) {
            const int i = e / wp, jj = e - i * wp;
            const int t = (i >> 4) * nct + (jj >> 4);
            T val = T(0);
            for (int q = 0; q < ks; ++q) val += sR2[(t * ks + q) * 256 + (i & 15) * 16 + (jj & 15)];
            if (i == jj && i >= w) val = T(1);
            sW[i * LDW + jj] = val;
          }
          __syncthreads();
        }
        if (wave == 0) {
          const bool good = (wp == 16) ? chol_wave<T, 16, BW>(sW, sL[pass], sDinv[pass], lane)
                                       : chol_wave<T, (BW == 32 ? 32 : 16), BW>(sW, sL[pass], sDinv[pass], lane);
          if (lane == 0) sInt[1] = good ? 0 : 1;
        }
        __syncthreads();
        if (sInt[1]) {
          ok = false;
        } else {
          if (wp == 16)
            trsm_rows<T, 16, BW>(sQ, sL[pass], sDinv[pass], n, tid, NT);
          else
            trsm_rows<T, (BW == 32 ? 32 : 16), BW>(sQ, sL[pass], sDinv[pass], n, tid, NT);
          __syncthreads();
        }
      }

      if (ok) {
        // R_jj = Lbar^T L^T; zeros below the diagonal down to row n-1.
        const int rows = n - s;
        for (int e = tid; e < rows * w; e += NT) {
          const int rr = e % rows, c = e / rows;
          if (rr == c + 1) continue;  // y_{s+c} goes there
          T v = T(0);
          if (rr <= c)
            for (int p = rr; p <= c; ++p) v += sL[1][p * LDW + rr] * sL[0][c * LDW + p];
          R[(size_t)(s + rr) + (size_t)(s + c) * ldr] = v;
        }
        for (int c = wave; c < w; c += NW) {
          T d = T(0);
          if (Bv)
            for (int r = lane; r < n; r += 64) d += sQ[sw(r, c, BW)] * Bv[r];
          d = wave_sum(d);
          if (lane == 0) {
            if (s + c + 1 < n) R[(size_t)(s + c + 1) + (size_t)(s + c) * ldr] = d;
            else sYlast = d;
          }
        }
        for (int e = tid; e < n * w; e += NT) {
          const int r = e % n, c = e / n;
          A[(size_t)r + (size_t)(s + c) * lda] = sQ[sw(r, c, BW)];
        }
        __syncthreads();
      } else {
        // CGS2 fallback, column by column against everything before it.
        flags |= CQR_FLAG_FALLBACK;
        if (info == 0) info = j + 1;
        T* sV = sQ;
        T* sHv = sR2;
        for (int c = 0; c < w; ++c) {
          const int col = s + c;
          for (int r = tid; r < n; r += NT) sV[r] = A[(size_t)r + (size_t)col * lda];
          __syncthreads();
          T lp0 = T(0), lp1 = T(0);
          bool fail = false;
          for (int pass = 0; pass < 2 && !fail; ++pass) {
            if (col > 0) {
              for (int p = wave; p < col; p += NW) {
                const T* pc = A + (size_t)p * lda;
                T d = T(0);
                for (int r = lane; r < n; r += 64) d += pc[r] * sV[r];
                d = wave_sum(d);
                if (lane == 0) sHv[p] = d;
              }
              __syncthreads();
              if (pass == 0)
                for (int p = tid; p < col; p += NT) R[(size_t)p + (size_t)col * ldr] = sHv[p];
              for (int r = tid; r < n; r += NT) {
                T d = T(0);
                for (int p = 0; p < col; ++p) d += A[(size_t)r + (size_t)p * lda] * sHv[p];
                sV[r] -= d;
              }
              __syncthreads();
            }
            T part = T(0);
            for (int r = tid; r < n; r += NT) part += sV[r] * sV[r];
            part = wave_sum(part);
            if (lane == 0) sRed[wave] = part;
            __syncthreads();
            T nrm2 = T(0);
            for (int q = 0; q < NW; ++q) nrm2 += sRed[q];
            if (!(nrm2 > T(0))) {
              fail = true;
            } else {
              const T l = sqrt(nrm2);
              if (pass == 0) lp0 = l; else lp1 = l;
              const T inv = T(1) / l;
              for (int r = tid; r < n; r += NT) sV[r] *= inv;
              if (pass == 1)
                for (int p = tid; p < col; p += NT) R[(size_t)p + (size_t)col * ldr] += sHv[p] * lp0;
            }
            __syncthreads();
          }
          if (fail) flags |= CQR_FLAG_ZERO_COL;
          for (int r = tid; r < n; r += NT) {
            A[(size_t)r + (size_t)col * lda] = fail ? T(0) : sV[r];
            if (r > col + 1) R[(size_t)r + (size_t)col * ldr] = T(0);
          }
          if (tid == 0) R[(size_t)col + (size_t)col * ldr] = fail ? T(0) : lp1 * lp0;
          if (wave == 0) {
            T d = T(0);
            if (!fail)
              for (int r = lane; r < n; r += 64) d += sV[r] * (Bv ? Bv[r] : T(0));
            d = wave_sum(d);
            if (lane == 0) {
              if (col + 1 < n) R[(size_t)(col + 1) + (size_t)col * ldr] = d;
              else sYlast = d;
            }
          }
          __syncthreads();
        }
      }
    }

    // Back substitution R x = y, block by block from the last, with y gathered
    // from the subdiagonal of R into the (now free) block buffer.
    if (Bv) {
      T* const sY = sQ;
      __syncthreads();
      for (int r = tid; r < n; r += NT) {
        if (r + 1 < n) {
          sY[r] = R[(size_t)(r + 1) + (size_t)r * ldr];
          R[(size_t)(r + 1) + (size_t)r * ldr] = T(0);
        } else {
          sY[r] = sYlast;
        }
      }
      __syncthreads();
      for (int J = nblk - 1; J >= 0; --J) {
        const int s = J * bw, w = min(bw, n - s);
        if (wave == 0) {
          T rrow[BW];
#pragma unroll
          for (int c = 0; c < BW; ++c)
            rrow[c] = (lane < w && c < w) ? R[(size_t)(s + lane) + (size_t)(s + c) * ldr] : T(0);
          T yi = (lane < w) ? sY[s + lane] : T(0);
#pragma unroll
          for (int c = BW - 1; c >= 0; --c) {
            if (c < w) {
              const T xc = Mf<T>::rl(yi, c) / Mf<T>::rl(rrow[c], c);
              if (lane == c) yi = xc;
              else if (lane < c) yi -= rrow[c] * xc;
            }
          }
          if (lane < w) sY[s + lane] = yi;
        }
        __syncthreads();
        for (int r = tid; r < s; r += NT) {
          T d = T(0);
          for (int c = 0; c < w; ++c) d += R[(size_t)r + (size_t)(s + c) * ldr] * sY[s + c];
          sY[r] -= d;
        }
        __syncthreads();
      }
      for (int r = tid; r < n; r += NT) Bv[r] = sY[r];
    }
    if (tid == 0) {
      ar.info[m] = info;
      if (ar.flags) ar.flags[m] = flags;
    }
    __syncthreads();
  }
}

// Sort by decreasing n (counting sort in one workgroup), bucket ranges,
// counters; invalid entries get info = -1 and are not scheduled.
struct SetupArgs {
  int count;
  const int32_t* n;
  void* const* A;
  const int32_t* lda;
  void* const* R;
  const int32_t* ldr;
  int32_t* info;
  int32_t* flags;
  int32_t* order;
  int32_t* range;
  int32_t* counter;
  int nbuckets;
  int hi[kMaxBuckets];
};

__global__ __launch_bounds__(1024) void batch_setup_kernel(SetupArgs a) {
  __shared__ int hist[kBatchNMax + 2];
  const int tid = threadIdx.x;
  for (int v = tid; v < kBatchNMax + 2; v += 1024) hist[v] = 0;
  __syncthreads();
  const int nmax = a.hi[a.nbuckets - 1];
  for (int i = tid; i < a.count; i += 1024) {
    const int ni = a.n[i];
    const bool valid = ni >= 1 && ni <= nmax && a.lda[i] >= ni && a.ldr[i] >= ni && a.A[i] && a.R[i];
    if (valid) {
      atomicAdd(&hist[ni], 1);
    } else {
      a.info[i] = -1;
      if (a.flags) a.flags[i] = 0;
    }
  }
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int v = kBatchNMax; v >= 1; --v) {
      const int h = hist[v];
      hist[v] = acc;  // first position of size v in decreasing order
      acc += h;
    }
    hist[0] = acc;  // number of valid entries
    for (int b = 0; b < a.nbuckets; ++b) {
      a.range[2 * b] = hist[a.hi[b]];
      a.range[2 * b + 1] = (b == 0) ? acc : hist[a.hi[b - 1]];
      a.counter[b] = 0;
    }
  }
  __syncthreads();
  for (int i = tid; i < a.count; i += 1024) {
    const int ni = a.n[i];
    const bool valid = ni >= 1 && ni <= nmax && a.lda[i] >= ni && a.ldr[i] >= ni && a.A[i] && a.R[i];
    if (valid) a.order[atomicAdd(&hist[ni], 1)] = i;
  }
}

// ------------------------------------------------------------ instances
typedef void (*BatchFn)(BatchArgs);

struct Instance {
  int dtype, nmax, bw, waves;
  BatchFn fn;
};

const Instance kInstances[] = {
    {CQR_F64, 256, 16, 4, batch_kernel<double, 256, 16, 4>},
    {CQR_F64, 256, 32, 4, batch_kernel<double, 256, 32, 4>},
    {CQR_F64, 256, 16, 8, batch_kernel<double, 256, 16, 8>},
    {CQR_F64, 256, 32, 8, batch_kernel<double, 256, 32, 8>},
    {CQR_F64, 512, 16, 4, batch_kernel<double, 512, 16, 4>},
    {CQR_F64, 512, 16, 8, batch_kernel<double, 512, 16, 8>},
    {CQR_F32, 256, 16, 4, batch_kernel<float, 256, 16, 4>},
    {CQR_F32, 256, 32, 4, batch_kernel<float, 256, 32, 4>},
    {CQR_F32, 256, 16, 8, batch_kernel<float, 256, 16, 8>},
    {CQR_F32, 256, 32, 8, batch_kernel<float, 256, 32, 8>},
    {CQR_F32, 512, 16, 4, batch_kernel<float, 512, 16, 4>},
    {CQR_F32, 512, 32, 8, batch_kernel<float, 512, 32, 8>},
    // Small-size instances: less LDS and fewer registers, so that several
    // matrices share a CU and hide each other's latency.
    {CQR_F64, 64, 16, 4, batch_kernel<double, 64, 16, 4>},
    {CQR_F64, 128, 16, 4, batch_kernel<double, 128, 16, 4>},
    {CQR_F64, 128, 16, 8, batch_kernel<double, 128, 16, 8>},
    {CQR_F32, 64, 16, 4, batch_kernel<float, 64, 16, 4>},
    {CQR_F32, 128, 16, 4, batch_kernel<float, 128, 16, 4>},
    {CQR_F32, 128, 16, 8, batch_kernel<float, 128, 16, 8>},
    {CQR_F32, 256, 16, 4, batch_kernel<float, 256, 16, 4, 2>},  // two per CU
    {CQR_F64, 256, 16, 4, batch_kernel<double, 256, 16, 4, 2, 1>},  // two per CU: single chunk buffer
};
constexpr int kNumInstances = (int)(sizeof(kInstances) / sizeof(kInstances[0]));

struct Plan {
  int nbuckets;
  int hi[kMaxBuckets];
  int inst[kMaxBuckets];
};

std::mutex g_plan_mu;
// Default plans (the fastest instance per bucket as measured by the autotuner
// on MI355X for n uniform in [8, 256] and n = 512); the autotuner in the
// Python package replaces them.
Plan g_plan[2] = {
    {4, {64, 128, 256, 512}, {12, 13, 19, 5}},
    {4, {64, 128, 256, 512}, {15, 17, 18, 11}},
};

int grid_for(const Instance& in) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)in.fn, in.waves * 64, 0) != hipSuccess)
    return 0;
  if (per < 1) per = 1;
  return cus * per;
}

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t batch_layout(int64_t count, char* base, int32_t** order, int32_t** range, int32_t** counter) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += a256(bytes);
    return p;
  };
  int32_t* o = (int32_t*)take((size_t)(count > 0 ? count : 1) * 4);
  int32_t* r = (int32_t*)take(2 * kMaxBuckets * 4);
  int32_t* c = (int32_t*)take(kMaxBuckets * 4);
  if (order) *order = o;
  if (range) *range = r;
  if (counter) *counter = c;
  return off;
}

// Enqueue the setup kernel and one persistent launch per bucket, with the
// sort order, bucket ranges and work counters laid out at `work` (device
// memory of at least batch_layout(count) bytes).  Arguments already checked.
int batched_launch(int64_t count, int dtype, const int32_t* n, void* const* A, const int32_t* lda, void* const* R,
                   const int32_t* ldr, void* const* B, int32_t* info, int32_t* flags, char* work, hipStream_t st) {
  Plan plan;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    plan = g_plan[dtype];
  }
  SetupArgs sa;
  memset(&sa, 0, sizeof(sa));
  sa.count = (int)count;
  sa.n = n;
  sa.A = A;
  sa.lda = lda;
  sa.R = R;
  sa.ldr = ldr;
  sa.info = info;
  sa.flags = flags;
  batch_layout(count, work, &sa.order, &sa.range, &sa.counter);
  sa.nbuckets = plan.nbuckets;
  for (int b = 0; b < plan.nbuckets; ++b) sa.hi[b] = plan.hi[b];
  int slot = prof_begin(st);
  hipLaunchKernelGGL(batch_setup_kernel, dim3(1), dim3(1024), 0, st, sa);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return CQR_ERR_HIP_BASE - (int)e;
  prof_end(slot, ROLE_BATCH_SETUP, st, 0.0, (double)count * 24);
  // Largest sizes first: buckets from the top down.
  for (int b = plan.nbuckets - 1; b >= 0; --b) {
    const Instance& in = kInstances[plan.inst[b]];
    const int grid = grid_for(in);
    if (grid <= 0) return CQR_ERR_HIP_BASE - (int)hipErrorInvalidConfiguration;
    BatchArgs ba;
    ba.n = n;
    ba.A = A;
    ba.lda = lda;
    ba.R = R;
    ba.ldr = ldr;
    ba.B = B;
    ba.info = info;
    ba.flags = flags;
    ba.order = sa.order;
    ba.range = sa.range;
    ba.counter = sa.counter;
    ba.bucket = b;
    ba.bw = in.bw;
    slot = prof_begin(st);
    hipLaunchKernelGGL(in.fn, dim3(grid), dim3(in.waves * 64), 0, st, ba);
    e = hipGetLastError();
    if (e != hipSuccess) return CQR_ERR_HIP_BASE - (int)e;
    prof_end(slot, ROLE_BATCH, st, 0.0, 0.0);
  }
  return CQR_OK;
}

// Argument checks shared by both entry points (the same return codes).
int batched_check(int64_t count, int dtype, const int32_t* n, void* const* A, const int32_t* lda, void* const* R,
                  const int32_t* ldr, const int32_t* info) {
  if (count < 0 || count > INT32_MAX) return -1;
  if (dtype != CQR_F64 && dtype != CQR_F32) return -2;
  if (count == 0) return CQR_OK;
  if (!n) return -3;
  if (!A) return -4;
  if (!lda) return -5;
  if (!R) return -6;
  if (!ldr) return -7;
  if (!info) return -9;
  return CQR_OK;
}

}  // namespace
}  // namespace cqr

using namespace cqr;

extern "C" {

int cqr_batched_instance(int32_t id, int32_t* dtype, int32_t* nmax, int32_t* bw, int32_t* waves) {
  if (id < 0 || id >= kNumInstances) return CQR_ERR_UNSUPPORTED;
  const Instance& in = kInstances[id];
  if (dtype) *dtype = in.dtype;
  if (nmax) *nmax = in.nmax;
  if (bw) *bw = in.bw;
  if (waves) *waves = in.waves;
  return CQR_OK;
}

int cqr_batched_plan_get(int dtype, int32_t* nbuckets, int32_t* hi, int32_t* inst) {
  if (dtype != CQR_F64 && dtype != CQR_F32) return -1;
  if (!nbuckets || !hi || !inst) return -2;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  const Plan& p = g_plan[dtype];
  *nbuckets = p.nbuckets;
  for (int b = 0; b < p.nbuckets; ++b) {
    hi[b] = p.hi[b];
    inst[b] = p.inst[b];
  }
  return CQR_OK;
}

int cqr_batched_plan_set(int dtype, int32_t nbuckets, const int32_t* hi, const int32_t* inst) {
  if (dtype != CQR_F64 && dtype != CQR_F32) return -1;
  if (nbuckets < 1 || nbuckets > kMaxBuckets) return -2;
  if (!hi) return -3;
  if (!inst) return -4;
  for (int b = 0; b < nbuckets; ++b) {
    if (hi[b] < 1 || hi[b] > kBatchNMax || (b > 0 && hi[b] <= hi[b - 1])) return -3;
    if (inst[b] < 0 || inst[b] >= kNumInstances) return -4;
    const Instance& in = kInstances[inst[b]];
    if (in.dtype != dtype || in.nmax < hi[b]) return -4;
  }
  std::lock_guard<std::mutex> lk(g_plan_mu);
  Plan& p = g_plan[dtype];
  p.nbuckets = nbuckets;
  for (int b = 0; b < nbuckets; ++b) {
    p.hi[b] = hi[b];
    p.inst[b] = inst[b];
  }
  return CQR_OK;
}

int cqr_batched_workspace_size(int64_t count, size_t* bytes) {
  if (count < 0 || count > INT32_MAX) return -1;
  if (!bytes) return -2;
  *bytes = batch_layout(count, nullptr, nullptr, nullptr, nullptr);
  return CQR_OK;
}

int cqr_batched_factor_solve(int64_t count, int dtype, const int32_t* n, void* const* A, const int32_t* lda,
                             void* const* R, const int32_t* ldr, void* const* B, int32_t* info, int32_t* flags,
                             void* work, size_t work_bytes, void* stream) {
  int rc = batched_check(count, dtype, n, A, lda, R, ldr, info);
  if (rc != CQR_OK || count == 0) return rc;
  const size_t need = batch_layout(count, nullptr, nullptr, nullptr, nullptr);
  if (!work || work_bytes < need) return CQR_ERR_WORKSPACE;
  return batched_launch(count, dtype, n, A, lda, R, ldr, B, info, flags, (char*)work, (hipStream_t)stream);
}

}  // extern "C"
