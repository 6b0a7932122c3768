// Low-precision form of the factorisation and the FP64 iterative refinement.
//
// cqr_factor_mixed runs CGS-QR (Algorithms 3-5) with the projections
// (Alg. 5 S1/S6) and updates (S2/S7) on BF16 or FP8 (OCP E4M3) MFMA with FP32
// accumulation, while the working block, its Gram matrices, Cholesky factors
// and TRSMs stay in FP64.  Finished columns are kept in the low precision
// twice (column-major for the projections' A^T, transposed for the updates'
// A) and returned as FP32 Q; R is returned in FP32.  FP8 operands carry one
// power-of-two scale per column, undone exactly in the GEMM epilogue.  Y itself is read, never written, so that the
// refinement can compute residuals against it.
//
// cqr_solve_ir: x_0 = 0, then repeatedly d = R^{-1} Q^T r (FP32 factors, FP64
// arithmetic), x += d, r = rhs - Y x (FP64), until the HPL scaled residual
// ||r||_inf / (||Y||_inf ||x||_inf n eps) is below the tolerance.
#include <cstring>

#include "internal.h"
#include "../../include/cqr.h"

namespace cqr {
namespace {

#define MX_TRY(expr)                                          \
  do {                                                        \
    hipError_t e_ = (expr);                                   \
    if (e_ != hipSuccess) return CQR_ERR_HIP_BASE - (int)e_;  \
  } while (0)

#define MX_RC(expr)             \
  do {                          \
    const int rc_ = (expr);     \
    if (rc_ != CQR_OK) return rc_; \
  } while (0)

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
int64_t up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

bool g_tiled = true;  // tiled storage of the finished columns (cqr_set_mixed_layout)

// Element (k, m) of a tiled K x M operand with 128-column blocks of a_blk
// elements and k-stages of kst elements (128 bytes per column).
__device__ __forceinline__ int64_t tiled_index(int64_t k, int64_t m, int64_t a_blk, int kst) {
  return (m >> 7) * a_blk + (k / kst) * (128 * (int64_t)kst) + (m & 127) * kst + (k % kst);
}

// Buffers of the column block being orthogonalised.
struct Slot {
  double* Qj;       // q x b working block (FP64)
  double* H;        // rp x b first-pass projection (FP64)
  __bf16* B16;      // qp x b: BF16 copy of the block being projected (ld qp)
  __bf16* H16;      // rp x b: BF16 copy of a projection (ld rp)
  uint8_t* B8;      // qp x b: FP8 copy of the block
  uint8_t* H8;      // rp x b: FP8 copy of a projection
  float* binv;      // b: inverse scales of the block's columns (FP8)
};

struct MixedWork {
  int* status;
  double *W, *LT1, *XT1, *LT2, *XT2, *Rjj;  // b x b
  double* T;        // q x b after the first pass
  double* Hb;       // rp x b projections, second pass
  Slot slot;
  // BF16 form
  __bf16* P16;      // qp x rp: finished columns, column-major (ld qp)
  __bf16* P16T;     // rp x qp: finished columns transposed (ld rp)
  // FP8 form (OCP E4M3 bytes, each column with a power-of-two scale)
  uint8_t* P8;      // qp x rp
  uint8_t* P8T;     // rp x qp
  float* pinv;      // rp: inverse scale of each finished column
  float* hinv;      // b: inverse scales of a projection's columns (FP8)
  double* cmax;     // b: column maxima
  float* part;      // split-K partial sums
  size_t part_cap;
  void* fb;         // breakdown fallback workspace (counters first; zero at the start of a call)
  int64_t qp, rp;
  int64_t b;        // the block width of the call (every block but a ragged last one)
  // Tiled storage of the finished columns (see gemm_bf16_tn): a_blk of P
  // (K = qp rows, 128-column blocks) and of P^T (K = rp, 128-row blocks);
  // 0 = column-major.
  int64_t blk_p, blk_pt;
};

size_t mixed_layout(int64_t q, int64_t r, int64_t b, int prec, char* base, MixedWork* w) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += a256(bytes);
    return p;
  };
  MixedWork tmp;
  MixedWork* o = w ? w : &tmp;
  memset(o, 0, sizeof(*o));
  // Rows and columns of the low-precision copies padded to 128 (the tiled
  // layout's column blocks; a multiple of the BF16 and FP8 k-stages).
  o->qp = up(q > 0 ? q : 1, 128);
  o->rp = up(r > 0 ? r : 1, 128);
  o->b = b;
  const bool tiled = g_tiled;
  o->blk_p = tiled ? o->qp * 128 : 0;
  o->blk_pt = tiled ? o->rp * 128 : 0;
  const size_t bb = (size_t)b * b * 8, qb = (size_t)q * b * 8;
  o->status = (int*)take(64);
  o->W = (double*)take(bb);
  o->LT1 = (double*)take(bb);
  o->XT1 = (double*)take(bb);
  o->LT2 = (double*)take(bb);
  o->XT2 = (double*)take(bb);
  o->Rjj = (double*)take(bb);
  o->T = (double*)take(qb);
  o->Hb = (double*)take((size_t)o->rp * b * 8);
  {
    Slot& sl = o->slot;
    sl.Qj = (double*)take(qb);
    sl.H = (double*)take((size_t)o->rp * b * 8);
    if (prec == CQR_PREC_FP8) {
      sl.B8 = (uint8_t*)take((size_t)o->qp * b);
      sl.H8 = (uint8_t*)take((size_t)o->rp * b);
      sl.binv = (float*)take((size_t)b * 4);
    } else {
      sl.B16 = (__bf16*)take((size_t)o->qp * b * 2);
      sl.H16 = (__bf16*)take((size_t)o->rp * b * 2);
    }
  }
  if (prec == CQR_PREC_FP8) {
    o->P8 = (uint8_t*)take((size_t)o->qp * o->rp);
    o->P8T = (uint8_t*)take((size_t)o->rp * o->qp);
    o->pinv = (float*)take((size_t)o->rp * 4);
    o->hinv = (float*)take((size_t)b * 4);
  } else {
    o->P16 = (__bf16*)take((size_t)o->qp * o->rp * 2);
    o->P16T = (__bf16*)take((size_t)o->rp * o->qp * 2);
  }
  o->cmax = (double*)take((size_t)b * 8);
  o->part_cap = (size_t)16 << 20;
  o->part = (float*)take(o->part_cap * 4);
  o->fb = take(fallback_workspace_bytes(r > b ? r : b));
  return off;
}

// dst (bf16, rows_pad x cols, ld ldd) = bf16(src (rows x cols, lds)); rows
// rows..rows_pad-1 are zero.  Column j = blockIdx.y; each thread converts 4
// consecutive rows and stores them as one 8-byte word (rows_pad and ldd are
// multiples of 4, dst 8-byte aligned).
constexpr int kCvtRows = 4 * 256;  // rows per workgroup of the conversion kernels
__global__ void __launch_bounds__(256)
to_bf16_kernel(int64_t rows, int64_t rows_pad, int64_t cols, const double* __restrict__ src, int64_t lds,
               __bf16* __restrict__ dst, int64_t ldd, const int* __restrict__ gate) {
  if (gate != nullptr && *gate != 0) return;
  const int64_t j = blockIdx.y;
  const int64_t i0 = (int64_t)blockIdx.x * kCvtRows + 4 * threadIdx.x;
  if (j >= cols || i0 >= rows_pad) return;
  const double* sc = src + j * lds;
  typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
  bf4 o;
#pragma unroll
  for (int u = 0; u < 4; ++u) o[u] = (i0 + u < rows) ? (__bf16)sc[i0 + u] : (__bf16)0.0f;
  *(bf4*)(dst + i0 + j * ldd) = o;
}

// ---------------------------------------------------------------- FP8 operands
// OCP E4M3 (the gfx950 FP8 format: largest finite 448, no saturation in the
// conversion instruction, so values are clamped first).  Every operand column
// is scaled by a power of two s = 2^(8 - e), with max |column| = f 2^e,
// f in [0.5, 1), which maps the column maximum into [128, 256); the GEMM
// epilogue multiplies by 1/s exactly.

__device__ __forceinline__ uint8_t to_e4m3(float v) {
  v = fminf(fmaxf(v, -448.f), 448.f);
  return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(v, 0.f, 0, false) & 0xff);
}

__device__ __forceinline__ float pow2_scale(double m) {
  if (!(m > 0.0) || !(m < 1e300)) return 1.f;
  int e;
  frexp(m, &e);
  e = e < -110 ? -110 : (e > 120 ? 120 : e);  // keeps s and 1/s normal floats
  return ldexpf(1.f, 8 - e);
}

// cmax[j] = max_i |src(i, j) * rowscale[i]| (rowscale may be NULL); one
// 1024-thread workgroup per column, 8 loads in flight per thread.  Maxima are
// exact, so the order of the reduction does not matter.
constexpr int kColmaxThreads = 1024;
__global__ void __launch_bounds__(kColmaxThreads)
colmax_kernel(int64_t rows, const double* __restrict__ src, int64_t lds, const float* __restrict__ rowscale,
              double* __restrict__ cmax, const int* __restrict__ gate) {
  if (gate != nullptr && *gate != 0) return;
  constexpr int T = kColmaxThreads;
  __shared__ double red[T];
  const int j = blockIdx.x, t = threadIdx.x;
  const double* col = src + (int64_t)j * lds;
  double m = 0.0;
  int64_t i0 = t;
  for (; i0 + 7 * T < rows; i0 += 8 * T) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = col[i0 + u * T] * (rowscale ? (double)rowscale[i0 + u * T] : 1.0);
#pragma unroll
    for (int u = 0; u < 8; ++u) m = fmax(m, fabs(v[u]));
  }
  for (; i0 < rows; i0 += T) m = fmax(m, fabs(col[i0] * (rowscale ? (double)rowscale[i0] : 1.0)));
  red[t] = m;
  __syncthreads();
  for (int h = T / 2; h > 0; h >>= 1) {
    if (t < h) red[t] = red[t + h] > red[t] ? red[t + h] : red[t];
    __syncthreads();
  }
  if (t == 0) cmax[j] = red[0];
}

// dst (FP8, rows_pad x cols, ld ldd) = e4m3(src(i, j) * rowscale[i] * s_j)
// with s_j from cmax[j]; colinv[j] = 1 / s_j; rows >= rows are zero.
// Column j = blockIdx.y; each thread converts 4 consecutive rows and stores
// them as one 4-byte word (rows_pad and ldd are multiples of 4).
__global__ void __launch_bounds__(256)
to_fp8_kernel(int64_t rows, int64_t rows_pad, int64_t cols, const double* __restrict__ src, int64_t lds,
              const float* __restrict__ rowscale, const double* __restrict__ cmax, uint8_t* __restrict__ dst,
              int64_t ldd, float* __restrict__ colinv, const int* __restrict__ gate) {
  if (gate != nullptr && *gate != 0) return;
  const int64_t j = blockIdx.y;
  const int64_t i0 = (int64_t)blockIdx.x * kCvtRows + 4 * threadIdx.x;
  if (j >= cols || i0 >= rows_pad) return;
  const float sc = pow2_scale(cmax[j]);
  const double* scol = src + j * lds;
  uint32_t word = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t i = i0 + u;
    uint32_t v = 0;
    if (i < rows) v = to_e4m3((float)(scol[i] * (rowscale ? (double)rowscale[i] : 1.0) * (double)sc));
    word |= v << (8 * u);
  }
  *(uint32_t*)(dst + i0 + j * ldd) = word;
  if (i0 == 0) colinv[j] = 1.f / sc;
}

// A finished block Qj (q x w, FP64): Q32[:, c0:c0+w] = float(Qj),
// P8[:, c0 + j] = e4m3(Qj[:, j] s_j) and P8T[c0 + j, :] its transpose, with
// s_j from cmax[j]; pinv[c0 + j] = 1 / s_j.
__global__ void __launch_bounds__(256)
finish_block_fp8_kernel(int64_t q, int w, const double* __restrict__ Qj, int64_t ldj, float* __restrict__ Q32,
                        int64_t ldq, uint8_t* __restrict__ P8, int64_t ldp, uint8_t* __restrict__ P8T, int64_t ldpt,
                        int64_t blk_p, int64_t blk_pt, const double* __restrict__ cmax, float* __restrict__ pinv,
                        int64_t c0, const int* __restrict__ gate) {
  if (gate != nullptr && *gate != 0) return;
  __shared__ uint8_t tile[64][65];
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int j0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
  for (int jj = ty; jj < 64; jj += 4) {
    const int64_t i = i0 + tx;
    const int j = j0 + jj;
    if (i < q && j < w) {
      const double v = Qj[i + (int64_t)j * ldj];
      const float sc = pow2_scale(cmax[j]);
      Q32[i + (c0 + j) * ldq] = (float)v;
      const uint8_t h = to_e4m3((float)(v * (double)sc));
      P8[blk_p ? tiled_index(i, c0 + j, blk_p, 128) : i + (c0 + j) * ldp] = h;
      tile[jj][tx] = h;
      if (i == 0) pinv[c0 + j] = 1.f / sc;
    }
  }
  __syncthreads();
  for (int ii = ty; ii < 64; ii += 4) {
    const int64_t i = i0 + ii;
    const int j = j0 + tx;
    if (i < q && j < w) P8T[blk_pt ? tiled_index(c0 + j, i, blk_pt, 128) : (c0 + j) + i * ldpt] = tile[tx][ii];
  }
}

// A finished block Qj (q x w, FP64): Q32[:, c0:c0+w] = float(Qj),
// P16[:, c0:c0+w] = bf16(Qj), P16T[c0:c0+w, :] = bf16(Qj)^T (through an LDS
// tile so that both the column-major and the transposed writes coalesce).
__global__ void __launch_bounds__(256)
finish_block_kernel(int64_t q, int w, const double* __restrict__ Qj, int64_t ldj, float* __restrict__ Q32,
                    int64_t ldq, __bf16* __restrict__ P16, int64_t ldp, __bf16* __restrict__ P16T, int64_t ldpt,
                    int64_t blk_p, int64_t blk_pt, int64_t c0, const int* __restrict__ gate) {
  if (gate != nullptr && *gate != 0) return;
  __shared__ __bf16 tile[64][65];
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int j0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
  for (int jj = ty; jj < 64; jj += 4) {
    const int64_t i = i0 + tx;
    const int j = j0 + jj;
    if (i < q && j < w) {
      const double v = Qj[i + (int64_t)j * ldj];
      Q32[i + (c0 + j) * ldq] = (float)v;
      const __bf16 h = (__bf16)v;
      P16[blk_p ? tiled_index(i, c0 + j, blk_p, 64) : i + (c0 + j) * ldp] = h;
      tile[jj][tx] = h;
    }
  }
  __syncthreads();
  for (int ii = ty; ii < 64; ii += 4) {
    const int64_t i = i0 + ii;
    const int j = j0 + tx;
    if (i < q && j < w) P16T[blk_pt ? tiled_index(c0 + j, i, blk_pt, 64) : (c0 + j) + i * ldpt] = tile[tx][ii];
  }
}

// R32[0:rows, cols] = float(src) for a rows x cols FP64 block.
__global__ void __launch_bounds__(256)
to_f32_kernel(int64_t rows, int64_t cols, const double* __restrict__ src, int64_t lds, float* __restrict__ dst,
              int64_t ldd, const int* __restrict__ gate) {
  if (gate != nullptr && *gate != 0) return;
  const int64_t total = rows * cols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx % rows, j = idx / rows;
    dst[i + j * ldd] = (float)src[i + j * lds];
  }
}

__global__ void __launch_bounds__(256) fill_kernel(int64_t n, char* __restrict__ p) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void __launch_bounds__(256) zero_f32_kernel(int64_t rows, int64_t cols, float* __restrict__ X, int64_t ldx) {
  const int64_t total = rows * cols;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x)
    X[idx % rows + (idx / rows) * ldx] = 0.f;
}

// Grid of the conversion kernels: kCvtRows rows by one column per workgroup.
dim3 cvt_grid(int64_t rows_pad, int64_t cols) {
  return dim3((unsigned)((rows_pad + kCvtRows - 1) / kCvtRows), (unsigned)cols);
}

unsigned grid_of(int64_t total) {
  int64_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  return (unsigned)blocks;
}

// ---------------------------------------------------------------- refinement

// part[c][i] = sum over columns j in chunk c of Y(i, j) x_j; with ABS also
// pabs[c][i] = the same sum of |Y(i, j)| (the row sums of ||Y||_inf, taken
// in the same pass over Y).
template <bool ABS>
__global__ void __launch_bounds__(256)
gemv_n_part_kernel(int64_t n, const double* __restrict__ Y, int64_t ldy, const double* __restrict__ x, int64_t chunk,
                   double* __restrict__ part, double* __restrict__ pabs) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (i >= n) return;
  const int64_t j0 = c * chunk, j1 = (j0 + chunk < n) ? j0 + chunk : n;
  double acc = 0.0, aab = 0.0;
  for (int64_t j = j0; j < j1; ++j) {
    const double y = Y[i + j * ldy];
    acc += y * x[j];
    if (ABS) aab += fabs(y);
  }
  part[c * n + i] = acc;
  if (ABS) pabs[c * n + i] = aab;
}

// r = rhs - sum_c part[c] (or the row sums themselves when rhs == nullptr);
// out[0] = max |r_i|, computed by one workgroup per 256 rows into blockmax.
__global__ void __launch_bounds__(256)
residual_kernel(int64_t n, int nchunk, const double* __restrict__ part, const double* __restrict__ rhs,
                double* __restrict__ r, double* __restrict__ blockmax) {
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * n + i];
    v = rhs ? rhs[i] - s : s;
    if (r) r[i] = v;
  }
  red[threadIdx.x] = fabs(v);
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) blockmax[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) max_kernel(int64_t n, const double* __restrict__ v, double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) m = fmax(m, fabs(v[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// y = Q^T v with FP32 Q, FP64 v and accumulation: one wave per column; with
// VEC (16-byte aligned columns) each lane reads 4 consecutive entries at a
// time into four accumulators, added in a fixed order at the end.
template <bool VEC>
__global__ void __launch_bounds__(256)
gemv_t_f32_kernel(int64_t n, const float* __restrict__ Q, int64_t ldq, const double* __restrict__ v,
                  double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  const float* qc = Q + j * ldq;
  double acc = 0.0;
  if constexpr (VEC) {
    double a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t i = 4 * lane;
    for (; i + 3 < n; i += 256) {
      const float4 q4 = *(const float4*)(qc + i);
      acc += (double)q4.x * v[i];
      a1 += (double)q4.y * v[i + 1];
      a2 += (double)q4.z * v[i + 2];
      a3 += (double)q4.w * v[i + 3];
    }
    for (int64_t t = i; t < n && t < i + 4; ++t) acc += (double)qc[t] * v[t];
    acc = (acc + a1) + (a2 + a3);
  } else {
    for (int64_t i = lane; i < n; i += 64) acc += (double)qc[i] * v[i];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) y[j] = acc;
}

// info = 0 and the k block flags = 0 (device outputs; NULL skips them).
__global__ void init_info_kernel(int32_t* info, int32_t* flags, int64_t k) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && info) info[0] = 0;
  if (flags && i < k) flags[i] = 0;
}

__global__ void __launch_bounds__(256) axpy_kernel(int64_t n, const double* __restrict__ d, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] += d[i];
}

// ---------------------------------------------------------------- factor

// Breakdown fallback of one block (Section 3): when a Cholesky factorisation
// of the block broke down (or the block's breakdown is forced), the block is
// restored from Y and redone column by column by CGS2 in FP64 arithmetic
// against the FP32 finished columns, writing the slot's Qj, its projections H
// and the triangle ws.Rjj; info and flags record it and the status word is
// cleared, so the block's remaining steps run.  An empty launch otherwise.
hipError_t block_fallback(int64_t q, int64_t w, int64_t s, const double* Yj, int64_t ldy, const float* Q32,
                          int64_t ldq, const MixedWork& ws, const Slot& sl, int blk, int32_t* info, int32_t* flags,
                          hipStream_t st) {
  if (blk == forced_breakdown_block()) {
    hipError_t e = force_breakdown(ws.status, blk, st);
    if (e != hipSuccess) return e;
  }
  return cgs2_fallback_f32basis(q, s, w, Q32, ldq, sl.Qj, q, sl.H, ws.rp, ws.Rjj, w, Yj, ldy, ws.status, info, flags,
                                blk, ws.fb, st);
}

// The low-precision copy of a block X (q x w, FP64) as the projection's B
// operand: BF16, or FP8 with its column scales (binv) from the column maxima.
int stage_operand(int prec, int64_t q, int64_t w, const double* X, const MixedWork& ws, const Slot& sl, double* cmax,
                  const int* gate, hipStream_t st) {
  if (prec == CQR_PREC_FP8) {
    hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)w), dim3(kColmaxThreads), 0, st, q, X, q, (const float*)nullptr,
                       cmax, gate);
    MX_TRY(hipGetLastError());
    hipLaunchKernelGGL(to_fp8_kernel, cvt_grid(ws.qp, w), dim3(256), 0, st, q, ws.qp, w, X, q, (const float*)nullptr,
                       cmax, sl.B8, ws.qp, sl.binv, gate);
  } else {
    hipLaunchKernelGGL(to_bf16_kernel, cvt_grid(ws.qp, w), dim3(256), 0, st, q, ws.qp, w, X, q, sl.B16, ws.qp, gate);
  }
  MX_TRY(hipGetLastError());
  return CQR_OK;
}

// Classical Gram-Schmidt step of Algorithm 5 (S1/S2 or S6/S7) against the
// finished columns c0 .. c1-1, from the low-precision copy of X staged in the
// slot: Hd[c0:c1] = P[:, c0:c1]^T X (FP32 accumulation into FP64), then
// X -= P[:, c0:c1] Hd[c0:c1] with the projection rounded to the low precision
// (hinv: its column scales in the FP8 form).  c0 is a multiple of the K
// granule (64 BF16, 128 FP8); rows c1 .. up(c1) - 1 of the copy are zero.
int project_update(int prec, int64_t q, int64_t w, int64_t c0, int64_t c1, double* X, double* Hd,
                   const MixedWork& ws, const Slot& sl, float* hinv, double* cmax, float* part, const int* gate,
                   hipStream_t st) {
  const int64_t m = c1 - c0;
  if (m <= 0) return CQR_OK;
  const double flops = 2.0 * (double)w * (double)q * (double)m;
  if (prec == CQR_PREC_FP8) {
    const int64_t kp = up(c1, 128) - c0;
    const uint8_t* pa = ws.blk_p ? ws.P8 + (c0 >> 7) * ws.blk_p : ws.P8 + c0 * ws.qp;
    MX_TRY(gemm_fp8_tn(ROLE_PROJ, m, w, ws.qp, 1.0f, pa, ws.qp, ws.blk_p, sl.B8, ws.qp, 0.0f, Hd + c0, ws.rp, true,
                       ws.pinv + c0, sl.binv, part, ws.part_cap, gate, st, flops));
    // H' = diag(1/s_P) H, then per-column scales for its FP8 copy.
    hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)w), dim3(kColmaxThreads), 0, st, m, Hd + c0, ws.rp,
                       ws.pinv + c0, cmax, gate);
    MX_TRY(hipGetLastError());
    hipLaunchKernelGGL(to_fp8_kernel, cvt_grid(kp, w), dim3(256), 0, st, m, kp, w, Hd + c0, ws.rp, ws.pinv + c0,
                       cmax, sl.H8 + c0, ws.rp, hinv, gate);
    MX_TRY(hipGetLastError());
    // X -= (P diag(s_P)) (diag(1/s_P) H), columns undone by 1/s_H.
    const uint8_t* pt = ws.blk_pt ? ws.P8T + c0 * 128 : ws.P8T + c0;
    MX_TRY(gemm_fp8_tn(ROLE_UPDATE, q, w, kp, -1.0f, pt, ws.rp, ws.blk_pt, sl.H8 + c0, ws.rp, 1.0f, X, q, true,
                       nullptr, hinv, nullptr, 0, gate, st, flops));
  } else {
    const int64_t kp = up(c1, 64) - c0;
    const __bf16* pa = ws.blk_p ? ws.P16 + (c0 >> 7) * ws.blk_p : ws.P16 + c0 * ws.qp;
    MX_TRY(gemm_bf16_tn(ROLE_PROJ, m, w, ws.qp, 1.0f, pa, ws.qp, ws.blk_p, sl.B16, ws.qp, 0.0f, Hd + c0, ws.rp, true,
                        part, ws.part_cap, gate, st, flops));
    hipLaunchKernelGGL(to_bf16_kernel, cvt_grid(kp, w), dim3(256), 0, st, m, kp, w, Hd + c0, ws.rp, sl.H16 + c0,
                       ws.rp, gate);
    MX_TRY(hipGetLastError());
    // X -= P H  (A = P^T stored k-contiguous); for at least 12288 rows the
    // 256-row tile with the reduction split in two through FP32 partial sums.
    const __bf16* pt = ws.blk_pt ? ws.P16T + c0 * 128 : ws.P16T + c0;
    MX_TRY(gemm_bf16_tn(ROLE_UPDATE, q, w, kp, -1.0f, pt, ws.rp, ws.blk_pt, sl.H16 + c0, ws.rp, 1.0f, X, q, true,
                        part, ws.part_cap, gate, st, flops));
  }
  return CQR_OK;
}

// Block j from the end of its first-pass update: S3-S5, the second pass
// S6-S10 against all s finished columns, S11/S12, the fallback, then R (FP32)
// and the finished columns in FP32 and the low precision.  Main stream,
// gated on the status word.
int block_rest(int prec, int64_t q, int64_t w, int64_t s, const double* Yj, int64_t ldy, float* Q32, int64_t ldq,
               float* R32, int64_t ldr, const MixedWork& ws, const Slot& sl, int blk, int32_t* info, int32_t* flags,
               hipStream_t st) {
  const int* gate = ws.status;
  const double dq = (double)q, dw = (double)w, ds = (double)s;
  for (int pass = 0; pass < 2; ++pass) {
    double* X = pass == 0 ? sl.Qj : ws.T;  // block being orthogonalised
    if (pass == 1 && s > 0) {
      MX_RC(stage_operand(prec, q, w, ws.T, ws, sl, ws.cmax, gate, st));
      MX_RC(project_update(prec, q, w, 0, s, ws.T, ws.Hb, ws, sl, ws.hinv, ws.cmax, ws.part, gate, st));
    }
    // S3/S8 (Gram) and S5/S10 (TRSM) on the FP64 block in FP32 arithmetic
    // (FP32 products and sums over each workgroup's reduction range, FP64
    // split sums and results); S4/S9 the Cholesky factorisation in FP32
    // arithmetic.  Their rounding is far below the projections' BF16/FP8
    // rounding that the factors carry anyway, and the FP32 Cholesky already
    // rounds the Gram to FP32.  The
    // strictly lower blocks of the factors' buffers are never written, so
    // they keep the zeros of the cleared workspace for every block of the
    // call's width (a ragged last block lays the buffers out with another
    // leading dimension and clears them).
    MX_TRY(gemm_tn(ROLE_GRAM, w, w, q, 1.0, X, q, X, q, 0.0, ws.W, w, (double*)ws.part, ws.part_cap / 2, gate, st,
                   (s > 0 ? 2.0 : 1.0) * dw * dw * dq, /*f32=*/true));
    MX_TRY(chol_inv_wide((int)w, ws.W, w, pass == 0 ? ws.LT1 : ws.LT2, pass == 0 ? ws.XT1 : ws.XT2, ws.Rjj, ws.status,
                         pass + 1, blk, st, /*f32=*/true, /*lower_zero=*/w == ws.b));
    MX_TRY(gemm_nn(ROLE_TRSM, q, w, w, 1.0, X, q, pass == 0 ? ws.XT1 : ws.XT2, w, 0.0, pass == 0 ? ws.T : sl.Qj, q,
                   gate, st, dw * dw * dq, /*f32=*/true));
  }
  // S11 R_jj = Lb^T L^T in FP64, S12 H = H + Hb L^T in FP32 arithmetic on
  // FP64 data (R is returned in FP32); then the fallback (a breakdown redoes
  // the block by CGS2), R (FP32) and the finished columns.
  MX_TRY(gemm_nn(ROLE_SMALL, w, w, w, 1.0, ws.LT2, w, ws.LT1, w, 0.0, ws.Rjj, w, gate, st, dw * dw * dw));
  if (s > 0)
    MX_TRY(gemm_nn(ROLE_SMALL, s, w, w, 1.0, ws.Hb, ws.rp, ws.LT1, w, 1.0, sl.H, ws.rp, gate, st, dw * ds,
                   /*f32=*/true));
  MX_TRY(block_fallback(q, w, s, Yj, ldy, Q32, ldq, ws, sl, blk, info, flags, st));
  if (s > 0) {
    hipLaunchKernelGGL(to_f32_kernel, dim3(grid_of(s * w)), dim3(256), 0, st, s, w, sl.H, ws.rp, R32 + s * ldr, ldr,
                       gate);
    MX_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(to_f32_kernel, dim3(grid_of(w * w)), dim3(256), 0, st, w, w, ws.Rjj, w, R32 + s + s * ldr, ldr,
                     gate);
  MX_TRY(hipGetLastError());
  const dim3 fgrid((unsigned)((q + 63) / 64), (unsigned)((w + 63) / 64));
  if (prec == CQR_PREC_FP8) {
    hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)w), dim3(kColmaxThreads), 0, st, q, sl.Qj, q,
                       (const float*)nullptr, ws.cmax, gate);
    MX_TRY(hipGetLastError());
    hipLaunchKernelGGL(finish_block_fp8_kernel, fgrid, dim3(256), 0, st, q, (int)w, sl.Qj, q, Q32, ldq, ws.P8, ws.qp,
                       ws.P8T, ws.rp, ws.blk_p, ws.blk_pt, ws.cmax, ws.pinv, s, gate);
  } else {
    hipLaunchKernelGGL(finish_block_kernel, fgrid, dim3(256), 0, st, q, (int)w, sl.Qj, q, Q32, ldq, ws.P16, ws.qp,
                       ws.P16T, ws.rp, ws.blk_p, ws.blk_pt, s, gate);
  }
  MX_TRY(hipGetLastError());
  return CQR_OK;
}

// Block j: its copy of Y, the first pass against all s finished columns,
// then the rest.
int block_plain(int prec, int64_t q, int64_t w, int64_t s, const double* Yj, int64_t ldy, float* Q32, int64_t ldq,
                float* R32, int64_t ldr, const MixedWork& ws, int blk, int32_t* info, int32_t* flags,
                hipStream_t st) {
  const Slot& sl = ws.slot;
  MX_TRY(copy_matrix(q, w, Yj, ldy, sl.Qj, q, ws.status, st));
  if (s > 0) {
    MX_RC(stage_operand(prec, q, w, sl.Qj, ws, sl, ws.cmax, ws.status, st));
    MX_RC(project_update(prec, q, w, 0, s, sl.Qj, sl.H, ws, sl, ws.hinv, ws.cmax, ws.part, ws.status, st));
  }
  return block_rest(prec, q, w, s, Yj, ldy, Q32, ldq, R32, ldr, ws, sl, blk, info, flags, st);
}

}  // namespace
}  // namespace cqr

using namespace cqr;

extern "C" {

int cqr_workspace_size_mixed(int64_t q, int64_t r, int64_t b, int prec, size_t* bytes) {
  if (q < 0) return -1;
  if (r < 0 || r > q) return -2;
  if (b < 1) return -3;
  if (b > 256 || b % 16 != 0) return CQR_ERR_UNSUPPORTED;
  if (prec != CQR_PREC_BF16 && prec != CQR_PREC_FP8) return CQR_ERR_UNSUPPORTED;
  if (!bytes) return -5;
  *bytes = mixed_layout(q, r, b, prec, nullptr, nullptr);
  return CQR_OK;
}

int cqr_factor_mixed(int64_t q, int64_t r, int64_t b, int prec, const double* Y, int64_t ldy, float* Q, int64_t ldq,
                     float* R, int64_t ldr, void* work, size_t work_bytes, int32_t* info, int32_t* block_flags,
                     void* stream) {
  if (q < 0) return -1;
  if (r < 0 || r > q) return -2;
  if (b < 1) return -3;
  if (b > 256 || b % 16 != 0) return CQR_ERR_UNSUPPORTED;
  if (prec != CQR_PREC_BF16 && prec != CQR_PREC_FP8) return CQR_ERR_UNSUPPORTED;
  if (!Y && q * r > 0) return -5;
  if (ldy < (q > 1 ? q : 1) || (ldy & 1)) return ldy < q ? -6 : CQR_ERR_UNSUPPORTED;
  if (!Q && q * r > 0) return -7;
  if (ldq < (q > 1 ? q : 1)) return -8;
  if (!R && r > 0) return -9;
  if (ldr < (r > 1 ? r : 1)) return -10;
  if (reinterpret_cast<uintptr_t>(Y) & 15) return CQR_ERR_UNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  const int64_t k = (r + b - 1) / b;
  if (info || block_flags) {
    const int64_t nk = k > 1 ? k : 1;
    hipLaunchKernelGGL(init_info_kernel, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, st, info, block_flags, k);
    MX_TRY(hipGetLastError());
  }
  if (r == 0) return CQR_OK;
  const size_t need = mixed_layout(q, r, b, prec, nullptr, nullptr);
  if (!work || work_bytes < need) return CQR_ERR_WORKSPACE;
  MixedWork ws;
  mixed_layout(q, r, b, prec, (char*)work, &ws);
  // Zero the whole workspace: the BF16 buffers rely on zero padding and on
  // not-yet-finished columns reading as zero.
  hipLaunchKernelGGL(fill_kernel, dim3(grid_of((int64_t)need)), dim3(256), 0, st, (int64_t)need, (char*)work);
  MX_TRY(hipGetLastError());
  hipLaunchKernelGGL(zero_f32_kernel, dim3(grid_of(r * r)), dim3(256), 0, st, r, r, R, ldr);
  MX_TRY(hipGetLastError());
  for (int64_t blk = 0; blk < k; ++blk) {
    const int64_t s = blk * b;
    const int64_t w = (r - s < b) ? r - s : b;
    const int rc = block_plain(prec, q, w, s, Y + s * ldy, ldy, Q, ldq, R, ldr, ws, (int)blk, info, block_flags, st);
    if (rc) return rc;
  }
  return CQR_OK;
}

// Testing aid: storage order of the finished low-precision columns.
int cqr_set_mixed_layout(int tiled) {
  if (tiled != 0 && tiled != 1) return -1;
  g_tiled = tiled != 0;
  return CQR_OK;
}

int cqr_solve_ir_workspace_size(int64_t n, size_t* bytes) {
  if (n < 0) return -1;
  if (!bytes) return -2;
  const int64_t nchunk = 16;
  *bytes = a256((size_t)(2 * nchunk + 4) * (size_t)(n > 0 ? n : 1) * 8) + a256((size_t)((n + 255) / 256 + 8) * 8) +
           trsv_workspace_bytes(n);
  return CQR_OK;
}

int cqr_solve_ir(int64_t n, const double* Y, int64_t ldy, const float* Q, int64_t ldq, const float* R, int64_t ldr,
                 const double* rhs, double* x, int32_t maxiter, double tol, int32_t* iters, double* scaled_resid,
                 void* work, size_t work_bytes, void* stream) {
  if (n < 0) return -1;
  if (!Y && n > 0) return -2;
  if (ldy < (n > 1 ? n : 1)) return -3;
  if (!Q && n > 0) return -4;
  if (ldq < (n > 1 ? n : 1)) return -5;
  if (!R && n > 0) return -6;
  if (ldr < (n > 1 ? n : 1)) return -7;
  if (!rhs && n > 0) return -8;
  if (!x && n > 0) return -9;
  if (maxiter < 1) return -10;
  if (!(tol > 0.0)) return -11;
  if (iters) *iters = 0;
  if (scaled_resid) *scaled_resid = 0.0;
  if (n == 0) return CQR_OK;
  size_t need = 0;
  cqr_solve_ir_workspace_size(n, &need);
  if (!work || work_bytes < need) return CQR_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  const int nchunk = 16;
  const int64_t chunk = (n + nchunk - 1) / nchunk;
  double* part = (double*)work;                 // nchunk x n
  double* pabs = part + (int64_t)nchunk * n;    // nchunk x n (row sums of |Y|)
  double* r = pabs + (int64_t)nchunk * n;       // residual
  double* c = r + n;                            // Q^T r, then d
  double* bm = (double*)((char*)work + a256((size_t)(2 * nchunk + 4) * n * 8));  // block maxima, then scalars
  const int64_t nblk = (n + 255) / 256;
  double* scal = bm + nblk;                     // [0] |Y|_inf [1] |r|_inf [2] |x|_inf
  void* tw = (char*)work + a256((size_t)(2 * nchunk + 4) * n * 8) + a256((size_t)(nblk + 8) * 8);
  const bool vec = (ldq % 4 == 0) && !(reinterpret_cast<uintptr_t>(Q) & 15);
  const unsigned* terr = trsv_error_word(n, tw);
  MX_TRY(trsv_prepare(n, true, R, ldr, tw, st));
  const dim3 gpart((unsigned)nblk, (unsigned)nchunk);
  // x = 0, r = rhs.
  MX_TRY(zero_matrix(n, 1, x, n, st));
  MX_TRY(copy_matrix(n, 1, rhs, n, r, n, nullptr, st));
  const double eps = 2.220446049250313e-16;
  for (int it = 1; it <= maxiter; ++it) {
    // d = R^{-1} Q^T r
    if (vec)
      hipLaunchKernelGGL(gemv_t_f32_kernel<true>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, n, Q, ldq, r, c);
    else
      hipLaunchKernelGGL(gemv_t_f32_kernel<false>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, n, Q, ldq, r, c);
    MX_TRY(hipGetLastError());
    MX_TRY(trsv_solve(n, true, R, ldr, tw, c, it - 1, st));
    hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)nblk), dim3(256), 0, st, n, c, x);
    MX_TRY(hipGetLastError());
    // r = rhs - Y x, ||r||_inf, ||x||_inf; in the first step also ||Y||_inf
    // from the same pass over Y.
    if (it == 1) {
      hipLaunchKernelGGL(gemv_n_part_kernel<true>, gpart, dim3(256), 0, st, n, Y, ldy, x, chunk, part, pabs);
      MX_TRY(hipGetLastError());
      hipLaunchKernelGGL(residual_kernel, dim3((unsigned)nblk), dim3(256), 0, st, n, nchunk, pabs,
                         (const double*)nullptr, (double*)nullptr, bm);
      MX_TRY(hipGetLastError());
      hipLaunchKernelGGL(max_kernel, dim3(1), dim3(256), 0, st, nblk, bm, scal + 0);
      MX_TRY(hipGetLastError());
    } else {
      hipLaunchKernelGGL(gemv_n_part_kernel<false>, gpart, dim3(256), 0, st, n, Y, ldy, x, chunk, part,
                         (double*)nullptr);
      MX_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(residual_kernel, dim3((unsigned)nblk), dim3(256), 0, st, n, nchunk, part, rhs, r, bm);
    MX_TRY(hipGetLastError());
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(256), 0, st, nblk, bm, scal + 1);
    MX_TRY(hipGetLastError());
    hipLaunchKernelGGL(max_kernel, dim3(1), dim3(256), 0, st, n, x, scal + 2);
    MX_TRY(hipGetLastError());
    double h[3];
    unsigned herr = 0;
    MX_TRY(hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, st));
    MX_TRY(hipMemcpyAsync(&herr, terr, sizeof(herr), hipMemcpyDeviceToHost, st));
    MX_TRY(hipStreamSynchronize(st));
    if (herr != 0) return CQR_ERR_HIP_BASE - (int)hipErrorLaunchTimeOut;
    const double res = h[1] / (h[0] * h[2] * (double)n * eps);
    if (iters) *iters = it;
    if (scaled_resid) *scaled_resid = res;
    if (res < tol) break;
  }
  return CQR_OK;
}

}  // extern "C"
