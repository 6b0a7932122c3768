/*
 * cqr.h -- C ABI of libcqr.so: QR factorisation by block classical
 * Gram-Schmidt with CholeskyQR2 re-orthogonalisation, on one AMD MI355X
 * (gfx950), in IEEE double precision, and the linear solve from its factors.
 *
 * The operations follow Tomas, Quintana-Orti, Anzt, "Fast Truncated SVD of
 * Sparse and Dense Matrices on Graphics Processors" (arXiv 2403.06218),
 * Section 3 (Algorithms 3, 4 and 5 and Table 1).
 *
 * Conventions shared by every entry point
 *   - Matrices are column-major: element (i, j) of X with leading dimension
 *     ldx is X[i + j * ldx].  Dimensions and leading dimensions are int64_t.
 *   - Every matrix and vector pointer is a DEVICE pointer (hipMalloc'd or a
 *     torch CUDA tensor), unless the parameter says "host".
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     All device work is enqueued on that stream, in stream order.
 *   - The caller owns every buffer.  The library never allocates device
 *     memory; scratch space is the caller's `work` buffer of at least the size
 *     the matching *_workspace_size function returns (256-byte aligned).
 *   - Leading dimensions are at most 4,000,000 (CQR_ERR_UNSUPPORTED beyond).
 *   - Return value: CQR_OK (0); -i if argument i (1-based position in the
 *     C signature) is invalid; CQR_ERR_* below otherwise.  On an argument error
 *     nothing is enqueued.
 *   - Outputs of type int32_t* marked "host" are written by the host after the
 *     call has synchronised the stream; those marked "device" are written by
 *     the call's kernels, in stream order.
 */
#ifndef CQR_H
#define CQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CQR_OK 0
#define CQR_ERR_UNSUPPORTED (-100) /* valid request this build does not support (b > 256, ld > 4e6) */
#define CQR_ERR_WORKSPACE (-101)   /* work == NULL or work_bytes below the required size     */
#define CQR_ERR_TOO_LARGE (-102)   /* size above the fixed scratch of cqr_solve_noalloc       */
#define CQR_ERR_HIP_BASE (-1000)   /* -1000 - hipError_t: a HIP launch or runtime call failed */

/* Precision forms of cqr_factor_mixed. */
#define CQR_PREC_BF16 1 /* projections and updates on BF16 MFMA with FP32 accumulation */
#define CQR_PREC_FP8 2  /* ... on FP8 (OCP E4M3) MFMA, per-column power-of-two scales, FP32 accumulation */

/* info of cqr_factor / cqr_orth / cqr_orth_against when a bounded wait inside
 * the breakdown fallback was abandoned (its workgroups were not all resident
 * within cqr_set_wait_limit_us); Q, R and H are then not valid. */
#define CQR_INFO_WAIT_ABANDONED (-2)

/* Bits of the per-block flags written by cqr_factor. */
#define CQR_FLAG_FALLBACK 1 /* the block's Cholesky factorisation broke down; redone by CGS2 */
#define CQR_FLAG_ZERO_COL 2 /* the block holds a column with no component outside the earlier ones */

/* Human-readable text for a return code (static storage, never NULL). */
const char* cqr_status_string(int code);

/* Library version string (static storage). */
const char* cqr_version(void);

/*
 * Bytes of device workspace cqr_factor needs for Y (q x r) and block width b;
 * also valid for cqr_orth (r = b) and cqr_orth_against (r = s + b).
 * Returns -1..-3 for q < 0, r < 0 or r > q, b < 1; CQR_ERR_UNSUPPORTED for
 * b > 256.
 */
int cqr_workspace_size(int64_t q, int64_t r, int64_t b, size_t* bytes);

/*
 * CGS-QR (Algorithm 3): Y (q x r, q >= r) = Q R with Q^T Q = I and R upper
 * triangular with positive diagonal.  Q overwrites Y in place.
 *   Y, ldy   in: Y; out: Q.  ldy >= max(1, q).
 *   R, ldr   out: r x r upper triangular (strictly lower part set to 0).
 *   b        block width, 1 <= b <= 256; the last block has width r - (k-1) b
 *            with k = ceil(r / b).  Block 1 is orthogonalised by CholeskyQR2
 *            (Algorithm 4); block j >= 2 by CGS-CQR2 (Algorithm 5) against the
 *            s = (j-1) b columns before it, its projection written to
 *            R[0:s, block j] and its triangular factor to the diagonal block.
 *            Blocks wider than 128 factor their Gram matrix as a 2 x 2 block.
 *   work     device workspace of work_bytes >= cqr_workspace_size(q, r, b).
 *   info     device int32, may be NULL: 0, or the 1-based index of the first
 *            block whose Cholesky factorisation broke down (a pivot that is not
 *            > 0, NaN included).  Such a block is restored and redone column by
 *            column by classical Gram-Schmidt with re-orthogonalisation (CGS2),
 *            which the paper's Section 3 prescribes as the fallback; the
 *            result is still a QR factorisation.  CQR_INFO_WAIT_ABANDONED if a
 *            bounded wait of that fallback was abandoned (results not valid).
 *   block_flags  device int32, may be NULL, length k: CQR_FLAG_* bits per
 *            block.  A column whose remainder after projection has zero norm
 *            gets a zero Q column and R_jj = 0 (CQR_FLAG_ZERO_COL).
 * Asynchronous: every step, the fallback decision included, runs in kernels
 * enqueued on `stream`; nothing is read back to the host, so the call can be
 * captured in a hipGraph.  info and block_flags are valid once the stream
 * has reached the end of the call.  Calls sharing a workspace must not
 * overlap.
 */
int cqr_factor(int64_t q, int64_t r, int64_t b, double* Y, int64_t ldy, double* R, int64_t ldr, void* work,
               size_t work_bytes, int32_t* info, int32_t* block_flags, void* stream);

/*
 * CholeskyQR2 (Algorithm 4): Q (q x b, q >= b, b <= 256) in place ->
 * orthonormal Q and R (b x b upper triangular) with Q_in = Q_out R.  info
 * (device int32, may be NULL): 0, 1 if the fallback to CGS2 was taken, or
 * CQR_INFO_WAIT_ABANDONED.  Asynchronous like cqr_factor.
 */
int cqr_orth(int64_t q, int64_t b, double* Q, int64_t ldq, double* R, int64_t ldr, void* work, size_t work_bytes,
             int32_t* info, void* stream);

/*
 * CGS-CQR2 (Algorithm 5): orthogonalise Q (q x b, b <= 256) against P (q x s,
 * whose columns are assumed orthonormal) ->  Q_in = P H + Q_out R,
 * P^T Q_out = 0, Q_out^T Q_out = I.  H (s x b, ldh >= max(1, s)) and R (b x b)
 * are outputs.  Q and P must not overlap.  q >= s + b.  info as for cqr_orth
 * (device); asynchronous like cqr_factor.
 */
int cqr_orth_against(int64_t q, int64_t b, int64_t s, double* Q, int64_t ldq, const double* P, int64_t ldp,
                     double* H, int64_t ldh, double* R, int64_t ldr, void* work, size_t work_bytes, int32_t* info,
                     void* stream);

/*
 * Bound of every bounded wait inside the library's kernels (the grid barriers
 * of the breakdown fallback, the look-back of the back substitution), in
 * microseconds of device time; default 10 s.  Past it a kernel stops waiting,
 * finishes without hanging and reports the abandoned wait (info
 * CQR_INFO_WAIT_ABANDONED, or the status of cqr_solve).  Applies to launches
 * made after the call.  Returns -1 for us < 0.
 */
int cqr_set_wait_limit_us(int64_t us);

/*
 * Testing aid for the breakdown fallback of Section 3: from the next call on,
 * cqr_factor and cqr_factor_mixed treat block blk (0-based) as if its
 * Cholesky factorisation had broken down -- the block is redone by the CGS2
 * fallback and info / block_flags report it -- so the fallback can be checked
 * on inputs whose exact QR is known and well conditioned.  blk = -1 (the
 * default) turns it off.  Returns -1 for blk < -1.  Process-wide.
 */
int cqr_set_forced_breakdown(int64_t blk);

/* Bytes of device workspace cqr_solve needs for order n (returns -1 for n < 0). */
int cqr_solve_workspace_size(int64_t n, size_t* bytes);

/*
 * Solve Y x = rhs from the factors of cqr_factor for square Y (n x n):
 * x = R^{-1} (Q^T rhs) -- a matrix-vector product then back substitution.
 * (The paper does not solve systems; this is the factorisation's use.)
 *   x        in: rhs (length n); out: the solution.
 *   work     device, cqr_solve_workspace_size(n) bytes: Q^T rhs, the FP64
 *            inverses of R's 64 x 64 diagonal blocks and the counters of the
 *            one-launch substitution (cleared by the call itself).  Calls that
 *            share a workspace must not overlap.
 *   status   device int32, may be NULL (not written when n == 0): 0, or 1 if
 *            the back substitution abandoned a bounded wait for a finished
 *            row block (see cqr_set_wait_limit_us); x is then not valid, and
 *            the blocks from the abandoned one upwards are NaN.
 * A zero diagonal entry of R (a dependent column) yields Inf/NaN entries.
 * Asynchronous: enqueues the work on `stream` and returns (capturable in a
 * hipGraph: kernels only).
 */
int cqr_solve(int64_t n, const double* Q, int64_t ldq, const double* R, int64_t ldr, double* x, void* work,
              size_t work_bytes, int32_t* status, void* stream);

/*
 * cqr_solve for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same results, with the workspace in a fixed array of
 * 33 MiB that the library holds on each GPU it runs on, from the first call
 * on that GPU until the process ends.  No allocation, no workspace argument.
 *   n        0 <= n <= CQR_NOALLOC_MAX_N (65536); above it the call returns
 *            CQR_ERR_TOO_LARGE and enqueues nothing.
 *   Q, R, x, status   as for cqr_solve.
 * All calls on one GPU share that GPU's array, which keeps the last call's
 * contents; calls that overlap on one GPU (other streams or threads) race and
 * must not be made.  Asynchronous, kernels only (capturable).
 */
#define CQR_NOALLOC_MAX_N 65536
int cqr_solve_noalloc(int64_t n, const double* Q, int64_t ldq, const double* R, int64_t ldr, double* x,
                      int32_t* status, void* stream);

/*
 * Low-precision form of cqr_factor (not in the paper, which computes in IEEE
 * double): CGS-QR (Algorithm 3) with the projections H = P^T Q and the updates
 * Q -= P H of Algorithm 5 (S1/S2, S6/S7) on BF16 matrix cores with FP32
 * accumulation (prec = CQR_PREC_BF16) or on FP8 E4M3 matrix cores with one
 * power-of-two scale per operand column (prec = CQR_PREC_FP8); the working
 * block, its Gram matrices, Cholesky factors and triangular solves stay in
 * FP64.
 *   Y, ldy   in (device, FP64, 16-byte aligned, even ldy): q x r; not modified.
 *   Q, ldq   out (FP32): q x r with Q^T Q ~ I to BF16 (FP8) accuracy.
 *   R, ldr   out (FP32): r x r upper triangular.
 *   b        block width: a multiple of 16, at most 256 (a width above 128
 *            factors its Gram matrix as a 2 x 2 block).
 *   info     device int32, may be NULL: 0, or the 1-based index of the first
 *            block whose Cholesky factorisation broke down.  As in cqr_factor
 *            (Section 3's fallback), such a block is redone column by column
 *            by CGS2, here in FP64 arithmetic against the FP32 finished
 *            columns, and the result is still a QR factorisation.
 *            CQR_INFO_WAIT_ABANDONED as for cqr_factor.
 *   block_flags  device int32, may be NULL, length ceil(r / b): CQR_FLAG_* bits.
 * Asynchronous and kernels only, like cqr_factor (capturable).
 */
int cqr_workspace_size_mixed(int64_t q, int64_t r, int64_t b, int prec, size_t* bytes);

/*
 * Testing aid for cqr_factor_mixed: the storage of the finished columns in
 * the low precision, tiled (1, the default: 128-column blocks of contiguous
 * 128-byte k-stages, so that every stage of a product reads one contiguous
 * tile) or column-major (0).  Only where the products read their operand
 * changes, so the results are the same bits.  Returns -1 for tiled not 0/1.
 * Process-wide; applies to calls made after it.
 */
int cqr_set_mixed_layout(int tiled);
int cqr_factor_mixed(int64_t q, int64_t r, int64_t b, int prec, const double* Y, int64_t ldy, float* Q, int64_t ldq,
                     float* R, int64_t ldr, void* work, size_t work_bytes, int32_t* info, int32_t* block_flags,
                     void* stream);

/*
 * FP64 iterative refinement of Y x = rhs (square, n x n) with the factors of
 * cqr_factor_mixed: x_0 = 0; d = R^{-1} Q^T r (FP32 factors, FP64
 * arithmetic); x += d; r = rhs - Y x in FP64; stop when the HPL scaled residual
 * ||r||_inf / (||Y||_inf ||x||_inf n eps) < tol or after maxiter updates.
 *   x        out (device, FP64, length n).
 *   iters, scaled_resid   host, may be NULL: updates done, final residual.
 * Synchronises the stream once per iteration.  Returns
 * -1000 - hipErrorLaunchTimeOut if the back substitution ever abandoned a
 * wait for a finished block (a bounded wait; x is then not valid).
 */
int cqr_solve_ir_workspace_size(int64_t n, size_t* bytes);
int cqr_solve_ir(int64_t n, const double* Y, int64_t ldy, const float* Q, int64_t ldq, const float* R, int64_t ldr,
                 const double* rhs, double* x, int32_t maxiter, double tol, int32_t* iters, double* scaled_resid,
                 void* work, size_t work_bytes, void* stream);

/*
 * Batched form: CGS-QR (Algorithms 3-5) and the solve x = R^{-1} Q^T b of
 * `count` independent square systems A_i x_i = b_i of uneven size
 * 1 <= n_i <= 512, in FP64 or FP32, one workgroup per matrix in persistent
 * launches (one per size bucket of the plan; see cqr_batched_plan_*).  Every
 * array below is in device memory and indexed by i; every call is
 * stream-ordered and asynchronous (capturable in a hipGraph: no host
 * synchronisation, no memset, no allocation).
 *   dtype    CQR_F64 (double) or CQR_F32 (float): the element type of every
 *            A_i, R_i, B_i, and the arithmetic of the whole path.
 *   n        n_i.
 *   A, lda   column-major n_i x n_i, lda_i >= n_i.  In: A_i; out: Q_i (in place).
 *   R, ldr   out: n_i x n_i upper triangular R_i (strictly lower part zero).
 *   B        may be NULL (factor only).  In: b_i (length n_i); out: x_i.
 *   info     out: 0, the 1-based first block whose Cholesky broke down and was
 *            redone by CGS2, or -1 for an entry with an invalid size, leading
 *            dimension or NULL pointer (that entry is left untouched).
 *   flags    may be NULL; out: CQR_FLAG_FALLBACK | CQR_FLAG_ZERO_COL bits.
 *   work     device workspace of cqr_batched_workspace_size(count) bytes.
 * Block width and kernel instance come from the plan for n_i's bucket.  An
 * exactly dependent column gives a zero Q column and R_jj = 0, and then x_i
 * holds infinities or NaNs.
 * Returns 0, -1..-9 for an invalid argument, CQR_ERR_WORKSPACE, or
 * -1000 - hipError_t.
 */
#define CQR_F64 0
#define CQR_F32 1
int cqr_batched_workspace_size(int64_t count, size_t* bytes);
int cqr_batched_factor_solve(int64_t count, int dtype, const int32_t* n, void* const* A, const int32_t* lda,
                             void* const* R, const int32_t* ldr, void* const* B, int32_t* info, int32_t* flags,
                             void* work, size_t work_bytes, void* stream);

/*
 * Kernel instances of the batched form: id -> element type, largest n,
 * block width and waves per workgroup.  CQR_ERR_UNSUPPORTED past the last id.
 */
int cqr_batched_instance(int32_t id, int32_t* dtype, int32_t* nmax, int32_t* bw, int32_t* waves);

/*
 * Plan of the batched form for one element type: nbuckets (<= 8) size buckets
 * with ascending upper bounds hi[b] (bucket b holds hi[b-1] < n <= hi[b]; the
 * last bound is the largest n accepted) and the instance inst[b] that serves
 * each (its nmax >= hi[b]).  The library starts with a default plan; the
 * package's autotuner measures the instances and sets a new one.  Host arrays.
 */
int cqr_batched_plan_get(int dtype, int32_t* nbuckets, int32_t* hi, int32_t* inst);
int cqr_batched_plan_set(int dtype, int32_t nbuckets, const int32_t* hi, const int32_t* inst);

/*
 * Adjoint of the batched solve (reverse mode): with A_i = Q_i R_i the stored
 * factors and x_i = A_i^{-1} b_i from cqr_batched_factor_solve, and g_i the
 * upstream gradient dL/dx_i,
 *   lambda_i = A_i^{-T} g_i = Q_i (R_i^{-T} g_i),  dA_i = -lambda_i x_i^T,
 *   db_i = lambda_i.
 * Device arrays indexed by i, as in cqr_batched_factor_solve: n, Q/ldq, R/ldr
 * (inputs), x, g (inputs, length n_i), dA/ldda (output, column-major n_i x n_i),
 * db (output, length n_i).  dtype CQR_F64 or CQR_F32 for every array.
 * Entries with n_i outside [1, 512], a leading dimension below n_i or a NULL
 * pointer are skipped.  No workspace; asynchronous on `stream`.  A zero R_ii
 * gives infinities or NaNs in that entry's outputs.
 * Returns 0, -1..-12 for an invalid argument, or -1000 - hipError_t.
 */
int cqr_batched_solve_backward(int64_t count, int dtype, const int32_t* n, void* const* Q, const int32_t* ldq,
                               void* const* R, const int32_t* ldr, void* const* x, void* const* g, void* const* dA,
                               const int32_t* ldda, void* const* db, void* stream);

/* ------------------------------------------------------------------------
 * Truncated SVD (Section 2): RandSVD (Algorithm 1) and LancSVD (Algorithm 2)
 * of an m x n matrix A, on the factorisations above.  A is dense (column-major
 * FP64) or sparse (CSR, with its transpose as a second CSR).  Every step runs
 * in the library's kernels on `stream` (asynchronous, no host round trip):
 * the products with A, the orthogonalisations (Algorithms 3-5 with the
 * device-side CGS2 fallback) and the small SVD (one-sided Jacobi, one
 * workgroup).  The random start blocks are inputs.  r <= 256, r a multiple of
 * b, b <= 256; LancSVD also needs m >= r + b (it forms Qbar_{k+1}).
 * ------------------------------------------------------------------------ */
#define CQR_SVD_LANCZOS 0
#define CQR_SVD_RANDOMIZED 1
#define CQR_SVD_SPARSE 2 /* OR'ed into `method`: workspace of the CSR entry points */

/* Bytes of device workspace of cqr_lancsvd / cqr_randsvd (method
 * CQR_SVD_LANCZOS or CQR_SVD_RANDOMIZED, | CQR_SVD_SPARSE for the _csr forms). */
int cqr_svd_workspace_size(int method, int64_t m, int64_t n, int64_t r, int64_t b, size_t* bytes);

/*
 * LancSVD (Algorithm 2): block Golub-Kahan-Lanczos with full orthogonalisation
 * of both bases and the basic restart, p restart cycles of k = r / b blocks.
 *   A, lda   m x n, column-major.
 *   Q1, ldq  m x b start block (S1 orthonormalises it by Algorithm 4).
 *   U, ldu   out: m x r left singular vectors (U = Pbar_k Ubar, S9).
 *   sigma    out: r singular values of B_k, decreasing.
 *   V, ldv   out: n x r right singular vectors (V = P_k Vbar, S8).
 *   info     device int32, may be NULL: the number of orthogonalisations that
 *            took the CGS2 fallback, or CQR_INFO_WAIT_ABANDONED.
 * B_k carries L_i = (R factor of S3)^T on its diagonal blocks and the R factor
 * of S5 below them.
 */
int cqr_lancsvd(int64_t m, int64_t n, const double* A, int64_t lda, int64_t r, int64_t b, int p, const double* Q1,
                int64_t ldq, double* U, int64_t ldu, double* sigma, double* V, int64_t ldv, int32_t* info,
                void* work, size_t work_bytes, void* stream);

/*
 * RandSVD (Algorithm 1): p steps of randomized subspace iteration from the
 * n x r start block Q0 (ldq >= n), CGS-QR (Algorithm 3, block width b) of
 * A Q (m x r) and of A^T Qbar (n x r), the SVD of R_p, U = Qbar_p Vbar,
 * V = Q_p Ubar.  Outputs and info as for cqr_lancsvd.
 */
int cqr_randsvd(int64_t m, int64_t n, const double* A, int64_t lda, int64_t r, int64_t b, int p, const double* Q0,
                int64_t ldq, double* U, int64_t ldu, double* sigma, double* V, int64_t ldv, int32_t* info,
                void* work, size_t work_bytes, void* stream);

/*
 * The same two drivers for a sparse A (m x n, nnz nonzeros, CSR with int32
 * row pointers and column indices; rows need not be sorted) together with its
 * transpose (trowptr, tcol, tval: the n x m CSR of A^T, e.g. from
 * cqr_csr_transpose).  Workspace: cqr_svd_workspace_size(method |
 * CQR_SVD_SPARSE, ...).
 */
int cqr_lancsvd_csr(int64_t m, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col, const double* val,
                    const int32_t* trowptr, const int32_t* tcol, const double* tval, int64_t r, int64_t b, int p,
                    const double* Q1, int64_t ldq, double* U, int64_t ldu, double* sigma, double* V, int64_t ldv,
                    int32_t* info, void* work, size_t work_bytes, void* stream);
int cqr_randsvd_csr(int64_t m, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col, const double* val,
                    const int32_t* trowptr, const int32_t* tcol, const double* tval, int64_t r, int64_t b, int p,
                    const double* Q0, int64_t ldq, double* U, int64_t ldu, double* sigma, double* V, int64_t ldv,
                    int32_t* info, void* work, size_t work_bytes, void* stream);

/*
 * Small dense SVD B = U diag(sigma) V^T of an r x r matrix (r <= 256) by
 * one-sided Jacobi in one workgroup (the GESVD step of Algorithms 1 and 2,
 * which the paper runs on the CPU).  sigma decreasing; columns of U with
 * sigma = 0 are zero.  sweeps (device int32, may be NULL): sweeps used, or
 * minus the sweep limit (60) if it was reached before convergence.
 */
int cqr_small_svd_workspace_size(int64_t r, size_t* bytes);
int cqr_small_svd(int64_t r, const double* B, int64_t ldb, double* U, int64_t ldu, double* sigma, double* V,
                  int64_t ldv, int32_t* sweeps, void* work, size_t work_bytes, void* stream);

/*
 * Products with A of the truncated SVD on the FP64 MFMA GEMM kernels:
 * C = alpha A^T B + beta C (trans_a = 1, A: K x M) or alpha A B + beta C
 * (trans_a = 0, A: M x K); B: K x N, C: M x N.  `work` (may be NULL) holds the
 * split-K partial sums of the transposed form (cqr_gemm_workspace_size bytes).
 */
int cqr_gemm_workspace_size(size_t* bytes);
int cqr_gemm(int trans_a, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
             const double* B, int64_t ldb, double beta, double* C, int64_t ldc, void* work, size_t work_bytes,
             void* stream);

/*
 * Residuals of computed triplets: res[j] = ||A v_j - sigma_j u_j||_2 / sigma_j
 * for j < count (dense A).  work: m * count doubles.
 */
int cqr_svd_residuals(int64_t m, int64_t n, const double* A, int64_t lda, int64_t count, const double* U,
                      int64_t ldu, const double* sigma, const double* V, int64_t ldv, double* res, void* work,
                      size_t work_bytes, void* stream);

/*
 * Sparse products (Table 1, SpMM rows): C = A X (trans = 0; rowptr/col/val
 * the m x n CSR of A, X n x w, C m x w) or C = A^T X (trans = 1; rowptr/col/
 * val the n x m CSR of A^T, X m x w, C n x w).  m, n are the dimensions of A
 * in both cases.  work: cqr_spmm_workspace_size(m, n) bytes (X in row-major
 * order).  Each row of C sums its nonzeros in storage order (reproducible).
 */
int cqr_spmm_workspace_size(int64_t m, int64_t n, size_t* bytes);
int cqr_spmm(int trans, int64_t m, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
             const double* val, int64_t w, const double* X, int64_t ldx, double* C, int64_t ldc, void* work,
             size_t work_bytes, void* stream);

/*
 * CSR of A^T from the CSR of A (m x n, nnz nonzeros), on the device: column
 * counts, a prefix sum, a scatter and a sort of every row of A^T by column, so
 * the result is unique (rows of A^T in increasing order).  trowptr: n + 1
 * entries; tcol, tval: nnz.  work: cqr_csr_transpose_workspace_size(n) bytes.
 */
int cqr_csr_transpose_workspace_size(int64_t n, size_t* bytes);
int cqr_csr_transpose(int64_t m, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col, const double* val,
                      int32_t* trowptr, int32_t* tcol, double* tval, void* work, size_t work_bytes, void* stream);

/*
 * Launch timing.  While enabled, every kernel launch the library makes is
 * bracketed by a pair of hipEvents on its stream.  cqr_prof_query synchronises
 * those events and returns, for the kernel role `name` (see cqr_prof_name),
 * the number of launches, their summed duration in ms, and the summed
 * algorithmic flop and byte counts of those launches (Table 1 cost model).
 */
int cqr_prof_enable(int on);
int cqr_prof_reset(void);
int cqr_prof_query(const char* name, int64_t* launches, double* total_ms, double* flops, double* bytes);
/* Name of kernel role i (0-based), or NULL past the last one. */
const char* cqr_prof_name(int i);

#ifdef __cplusplus
}
#endif

#endif /* CQR_H */
