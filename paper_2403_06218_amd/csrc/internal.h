// Internal declarations shared by the HIP sources of libcqr.so.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace cqr {

// Kernel roles: each role is a distinct kernel symbol, so a profiler's
// per-kernel statistics separate them, and the library's own launch timing
// (cqr_prof_*) accumulates per role.
enum Role : int {
  ROLE_PROJ = 0,    // H = P^T Q        (Alg. 5 S1/S6)          TN GEMM, split-K
  ROLE_UPDATE,      // Q = Q - P H      (Alg. 5 S2/S7)          NN GEMM
  ROLE_GRAM,        // W = Q^T Q        (Alg. 4 S1/S4, 5 S3/S8) TN GEMM, split-K; for M == N the
                    //                  strictly lower tiles (tile height) of W are left unwritten
  ROLE_TRSM,        // Q = Q L^{-T}     (Alg. 4 S3/S6, 5 S5/S10) NN GEMM by (L^{-1})^T; B upper triangular
  ROLE_SMALL,       // R = Lb^T L^T, H += Hbar L^T (Alg. 5 S11/S12); B upper triangular
  ROLE_REDUCE,      // split-K partial sums -> C
  ROLE_CHOL,        // W = L L^T and L^{-1}  (Alg. 4 S2/S5, 5 S4/S9)
  ROLE_COPY,        // block save / restore for the breakdown fallback
  ROLE_GEMV,        // solve: c = Q^T rhs
  ROLE_TRSV_INV,    // solve: inverses of the 64 x 64 diagonal blocks of R
  ROLE_TRSV,        // solve: back substitution R x = c, one launch
  ROLE_BATCH,       // batched form: whole factorisation + solve, one workgroup per matrix
  ROLE_BATCH_SETUP, // batched form: size sort and bucket boundaries
  ROLE_ADJOINT,     // adjoint of the solve
  ROLE_FALLBACK,    // breakdown fallback: the failed block redone by CGS2 (gated, one launch per block)
  ROLE_APROD,       // truncated SVD: products with the input matrix, A X (NN) and A^T X (TN)
  ROLE_SVD,         // truncated SVD: small dense SVD (one-sided Jacobi), B_k assembly, residuals
  ROLE_SPMM,        // truncated SVD: sparse products A X and A^T X (CSR)
  ROLE_COUNT
};

const char* role_name(int role);

// Launch timing hooks (no-ops unless cqr_prof_enable(1)).
int prof_begin(hipStream_t s);
void prof_end(int slot, int role, hipStream_t s, double flops, double bytes);

// C = alpha * A^T B + beta * C;  A: K x M (lda), B: K x N (ldb), C: M x N (ldc).
// Split over K through `part` (capacity part_cap doubles) when it pays.
// f32 (ROLE_GRAM and ROLE_CHOL only): FP32 products and per-split sums (stored
// as FP32 in `part`), FP64 data and split reduction.
hipError_t gemm_tn(Role role, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* part,
                   size_t part_cap, const int* gate, hipStream_t s, double flops, bool f32 = false);

// C = alpha * A B + beta * C;  A: M x K (lda), B: K x N (ldb), C: M x N (ldc).
// C may alias neither A nor B except element-wise (C(m,n) read only by its own update).
// f32 (ROLE_TRSM, ROLE_SMALL and ROLE_CHOL only): FP32 products and sums,
// FP64 data.
hipError_t gemm_nn(Role role, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double beta, double* C, int64_t ldc, const int* gate,
                   hipStream_t s, double flops, bool f32 = false);

// BF16 GEMM with FP32 accumulation: C (M x N) = alpha * A^T B + beta * C with
// A (K x M) and B (K x N) BF16, k-contiguous.  C is FP64 when c_is_f64, else
// FP32.  With `part` non-null the reduction over K may be split through FP32
// partial sums in `part` (capacity part_cap floats), added into C in split
// order by a second launch.
// Requires 16-byte aligned A and B, lda and ldb multiples of 8, K a multiple of 64.
// A is column-major (lda) when a_blk == 0, else tiled: columns in blocks of
// 128, each block a_blk elements holding its k-stages (64 k, 128 bytes per
// column) one after the other, each stage 128 columns x 64 k contiguous:
// element (k, m) at (m / 128) a_blk + (k / 64) 8192 + (m % 128) 64 + k % 64.
bool gemm_bf16_supported(const void* A, int64_t lda, const void* B, int64_t ldb, int64_t K);
hipError_t gemm_bf16_tn(Role role, int64_t M, int64_t N, int64_t K, float alpha, const __bf16* A, int64_t lda,
                        int64_t a_blk, const __bf16* B, int64_t ldb, float beta, void* C, int64_t ldc, bool c_is_f64,
                        float* part, size_t part_cap, const int* gate, hipStream_t s, double flops);

// FP8 (OCP E4M3 bytes) GEMM with FP32 accumulation, same contract as
// gemm_bf16_tn (C FP64 only, or FP32 split-K partials reduced into FP64 C),
// with optional per-row rs[m] and per-column cs[n] multipliers of A^T B (the
// inverse power-of-two scales of the operands).  Requires 16-byte aligned A
// and B, lda and ldb multiples of 16, K a multiple of 128.
bool gemm_fp8_supported(const void* A, int64_t lda, const void* B, int64_t ldb, int64_t K);
// A tiled as for BF16 with 128-k stages (128 bytes per column): element
// (k, m) at (m / 128) a_blk + (k / 128) 16384 + (m % 128) 128 + k % 128.
hipError_t gemm_fp8_tn(Role role, int64_t M, int64_t N, int64_t K, float alpha, const uint8_t* A, int64_t lda,
                       int64_t a_blk, const uint8_t* B, int64_t ldb, float beta, void* C, int64_t ldc, bool c_is_f64,
                       const float* rs, const float* cs, float* part, size_t part_cap, const int* gate, hipStream_t s,
                       double flops);

// Lower Cholesky W = L L^T of a b x b SPD matrix (b <= 128) and the inverse of
// L, in one workgroup.  Writes LT = L^T and XT = (L^{-1})^T (both b x b,
// leading dimension b, upper triangular with zero strictly-lower part).  On a
// pivot that is not > 0 sets status[0] = code, status[1] = blk.  With f32 the
// factorisation runs in FP32 arithmetic (FP64 input and outputs; b > 16).
hipError_t chol_inv(int b, const double* W, int64_t ldw, double* LT, double* XT, int* status, int code, int blk,
                    hipStream_t s, bool f32 = false);
// The same for b <= 256 through a 2 x 2 block split at 128 (MFMA GEMMs for the
// off-diagonal blocks and the Schur complement, in FP64).  W's trailing block
// is overwritten; tmp holds 128 x (b - 128) doubles.  lower_zero: the strictly
// lower (b-128) x 128 blocks of LT and XT already hold zeros (they are never
// written), so they are not cleared.
hipError_t chol_inv_wide(int b, double* W, int64_t ldw, double* LT, double* XT, double* tmp, int* status, int code,
                         int blk, hipStream_t s, bool f32 = false, bool lower_zero = false);

// Row-streaming steps of CGS-CQR2 for a narrow block (w <= 16 columns, s <= 128
// basis columns, q >= 16384 rows): tall_eligible tells whether they apply.
// The block is written only by the last step, so a breakdown leaves it intact.
// tall_proj:        H (s x w, ldh) = P^T X.
// tall_update_gram: Y = X - P H (no update when s == 0; Y may be X), then
//                   W (w x w, ld w) = Y^T Y.
// tall_trsm_proj:   T = X XT (XT w x w, ld w); if s > 0 and Hb != NULL also
//                   Hb (s x w, ldhb) = P^T T.
// Partial sums go through `part` (capacity part_cap doubles); every kernel is
// gated on *gate == 0.
bool tall_eligible(int64_t q, int64_t w, int64_t s);
hipError_t tall_proj(int64_t q, int s, int w, const double* P, int64_t ldp, const double* X, int64_t ldx, double* H,
                     int64_t ldh, double* part, size_t part_cap, const int* gate, hipStream_t st);
hipError_t tall_update_gram(int64_t q, int s, int w, const double* P, int64_t ldp, const double* H, int64_t ldh,
                            const double* X, int64_t ldx, double* Y, int64_t ldy, double* W, double* part,
                            size_t part_cap, const int* gate, hipStream_t st);
hipError_t tall_trsm_proj(int64_t q, int s, int w, const double* X, int64_t ldx, const double* XT, double* T,
                          int64_t ldt, const double* P, int64_t ldp, double* Hb, int64_t ldhb, double* part,
                          size_t part_cap, const int* gate, hipStream_t st);

// dst (rows x cols, ldd) = src (rows x cols, lds); gated on *gate == 0 when gate != NULL.
hipError_t copy_matrix(int64_t rows, int64_t cols, const double* src, int64_t lds, double* dst, int64_t ldd,
                       const int* gate, hipStream_t s);
// X (rows x cols) = 0.
hipError_t zero_matrix(int64_t rows, int64_t cols, double* X, int64_t ldx, hipStream_t s);

// Breakdown fallback (Section 3): redo the block Q (q x w, ldq) column by
// column by CGS2 against P (q x s, ldp) and its own earlier columns, in one
// launch gated on status[0] != 0 (an empty launch otherwise).  Restores the
// block from `save` (q x w, ldsave) first when save != NULL.  Writes H (s x w,
// ldh) and R (w x w, ldr); sets flags[blk] and info (first block, 1-based) when
// those are not NULL, then clears status.  `fbwork` holds
// fallback_workspace_bytes(s + w) bytes whose first 256 bytes (the counters)
// are zero before the first call; the kernel leaves them zero.  The _f32basis
// form takes the FP32 finished columns of the low-precision form as P (FP64
// arithmetic).
size_t fallback_workspace_bytes(int64_t sw);
hipError_t cgs2_fallback(int64_t q, int64_t s, int64_t w, const double* P, int64_t ldp, double* Q, int64_t ldq,
                         double* H, int64_t ldh, double* R, int64_t ldr, const double* save, int64_t ldsave,
                         int* status, int32_t* info, int32_t* flags, int blk, void* fbwork, hipStream_t st);
hipError_t cgs2_fallback_f32basis(int64_t q, int64_t s, int64_t w, const float* P, int64_t ldp, double* Q,
                                  int64_t ldq, double* H, int64_t ldh, double* R, int64_t ldr, const double* save,
                                  int64_t ldsave, int* status, int32_t* info, int32_t* flags, int blk, void* fbwork,
                                  hipStream_t st);
// Sets status = {1, blk} when no breakdown is recorded (the forced breakdown
// of cqr_set_forced_breakdown); forced_breakdown_block() is that block, or -1.
hipError_t force_breakdown(int* status, int blk, hipStream_t st);
int64_t forced_breakdown_block();

// Sparse matrix in CSR form with its transpose (also CSR), for the products
// A X and A^T X of the truncated SVD.  Row pointers and column indices are
// int32 (nnz < 2^31).  xrm: scratch of max(m, n) * 64 doubles holding the
// dense operand in row-major order.
struct SparseCsr {
  int64_t m, n, nnz;
  const int32_t* rowptr;   // m + 1
  const int32_t* col;      // nnz
  const double* val;       // nnz
  const int32_t* trowptr;  // n + 1 (CSR of A^T)
  const int32_t* tcol;
  const double* tval;
  double* xrm;
};
// C (m x w, ldc) = A X (X n x w, ldx), or with trans C (n x w) = A^T X (X m x w).
hipError_t spmm(const SparseCsr& S, bool trans, int64_t w, const double* X, int64_t ldx, double* C, int64_t ldc,
                hipStream_t st);
size_t spmm_scratch_doubles(int64_t m, int64_t n);

// Bound of one wait of a bounded wait loop (grid barrier, look-back), in
// ticks of the device's constant-rate clock (wall_clock64).
uint64_t wait_limit_ticks();

// Solve kernels.
hipError_t gemv_t(int64_t n, const double* Q, int64_t ldq, const double* x, double* y, hipStream_t s);

// Back substitution R x = c (R n x n upper triangular, FP64 or FP32 entries;
// c and x FP64, in place in y).  trsv_prepare forms the inverses of R's
// 64 x 64 diagonal blocks in `work` (trsv_workspace_bytes(n)) and clears its
// counters; then trsv_solve calls number seq = 0, 1, 2, ... of that sequence
// each solve one right-hand side with the same R.  *trsv_error_word(n, work)
// is nonzero if a wait was abandoned (the x block published after it is NaN).
// trsv_status copies that word into status[0] (device, int32: 0 or 1).
size_t trsv_workspace_bytes(int64_t n);
hipError_t trsv_prepare(int64_t n, bool f32, const void* R, int64_t ldr, void* work, hipStream_t s);
hipError_t trsv_solve(int64_t n, bool f32, const void* R, int64_t ldr, void* work, double* y, int64_t seq,
                      hipStream_t s);
const unsigned* trsv_error_word(int64_t n, const void* work);
hipError_t trsv_status(int64_t n, const void* work, int32_t* status, hipStream_t s);

}  // namespace cqr
