/*
 * CPU FP64 oracle for the block Gram-Schmidt QR factorization of
 * Tomas, Quintana-Orti, Anzt, "Fast Truncated SVD of Sparse and Dense
 * Matrices on Graphics Processors" (arXiv 2403.06218), Section 3.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code with the HIP library.
 *
 * Two independent oracles:
 *   O-def  the result by definition: thin QR Y = QR with Q^T Q = I and R upper
 *          triangular with positive diagonal (unique for full column rank),
 *          computed by textbook unblocked Householder QR [GVL3 Sec. 5.2]
 *          followed by a sign normalisation of the diagonal of R.
 *   O-alg  the paper's algorithm, step by step: CGS-QR (Algorithm 3) built from
 *          CholeskyQR2 (Algorithm 4) for the first column block and CGS-CQR2
 *          (Algorithm 5) for the later ones, with the Cholesky-breakdown
 *          fallback to classical Gram-Schmidt with re-orthogonalisation that
 *          Section 3 ("Orthogonalization via CholeskyQR2") describes.
 *
 * Readings of the paper taken here (each is argued where it is used):
 *   R1  Algorithm 4 step S7 and Algorithm 5 step S11 print R = L^T Lbar^T; the
 *       algebra of steps S3/S6 (resp. S5/S10) gives R = Lbar^T L^T.  The
 *       corrected order is the default; the printed order is kept as a variant.
 *   R2  Algorithm 5 step S12 prints H := H + Hbar; the algebra gives
 *       H := H + Hbar L^T.  Corrected by default; printed kept as a variant.
 *   R3  Algorithm 4 step S5 factors the Gram matrix of step S4 (Wbar).
 *   R4  A Cholesky breakdown is a pivot that is not > 0 (this includes NaN).
 *   R5  The fallback re-does only the failed column block, column by column,
 *       as Algorithm 5 with b = 1 (that is, CGS2) against all earlier columns,
 *       starting from the block's original contents.
 *   R6  r need not be a multiple of b: the last block has width r - (k-1) b.
 *   R7  Storage is column-major with a leading dimension; Q overwrites Y.
 *   R8  A column whose projected remainder has zero norm in the fallback is an
 *       exactly dependent column: its Q column is set to zero and R_jj = 0.
 *
 * All matrices are column-major: element (i, j) of X with leading dimension ld
 * is X[i + j*ld].  All arithmetic is IEEE double with round-to-nearest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define AT(X, i, j, ld) ((X)[(size_t)(i) + (size_t)(j) * (size_t)(ld)])

/* ------------------------------------------------------------------------ */
/* Basic building blocks (Table 1: GEMM, POTRF, TRSM, TRMM, ADD).            */
/* ------------------------------------------------------------------------ */

/* C (m x n) = A^T B, A is k x m, B is k x n.  Plain triple loop. */
static void mat_tn(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double* C, int64_t ldc) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < m; ++i) {
      double acc = 0.0;
      for (int64_t p = 0; p < k; ++p) acc += AT(A, p, i, lda) * AT(B, p, j, ldb);
      AT(C, i, j, ldc) = acc;
    }
}

/* C (m x n) -= A B, A is m x k, B is k x n. */
static void mat_sub_nn(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                       const double* B, int64_t ldb, double* C, int64_t ldc) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j)
    for (int64_t p = 0; p < k; ++p) {
      const double bpj = AT(B, p, j, ldb);
      for (int64_t i = 0; i < m; ++i) AT(C, i, j, ldc) -= AT(A, i, p, lda) * bpj;
    }
}

/*
 * W = L L^T, lower Cholesky in place (Table 1 POTRF), j-k-i ordering:
 * column j is finished from the already finished columns 0..j-1.
 * Returns 0, or j+1 if the j-th pivot is not > 0 (reading R4).  The strictly
 * upper part of W is set to zero on success.
 */
int ora_chol(int64_t b, double* W, int64_t ldw) {
  for (int64_t j = 0; j < b; ++j) {
    double d = AT(W, j, j, ldw);
    for (int64_t p = 0; p < j; ++p) d -= AT(W, j, p, ldw) * AT(W, j, p, ldw);
    if (!(d > 0.0)) return (int)(j + 1);
    const double ljj = sqrt(d);
    AT(W, j, j, ldw) = ljj;
    for (int64_t i = j + 1; i < b; ++i) {
      double v = AT(W, i, j, ldw);
      for (int64_t p = 0; p < j; ++p) v -= AT(W, i, p, ldw) * AT(W, j, p, ldw);
      AT(W, i, j, ldw) = v / ljj;
    }
  }
  for (int64_t j = 1; j < b; ++j)
    for (int64_t i = 0; i < j; ++i) AT(W, i, j, ldw) = 0.0;
  return 0;
}

/*
 * Q (q x b) := Q L^{-T}, L lower b x b (Table 1 TRSM, right side, transposed).
 * Row by row: x L^T = y  <=>  L x^T = y^T, solved by forward substitution.
 */
void ora_trsm_rlt(int64_t q, int64_t b, double* Q, int64_t ldq, const double* L, int64_t ldl) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < q; ++i)
    for (int64_t c = 0; c < b; ++c) {
      double v = AT(Q, i, c, ldq);
      for (int64_t p = 0; p < c; ++p) v -= AT(L, c, p, ldl) * AT(Q, i, p, ldq);
      AT(Q, i, c, ldq) = v / AT(L, c, c, ldl);
    }
}

/* R (b x b) = U1 U2 with U1, U2 upper triangular (Table 1 TRMM). */
static void upper_times_upper(int64_t b, const double* U1, int64_t ld1, const double* U2, int64_t ld2,
                              double* R, int64_t ldr) {
  for (int64_t j = 0; j < b; ++j)
    for (int64_t i = 0; i < b; ++i) {
      double acc = 0.0;
      if (i <= j)
        for (int64_t p = i; p <= j; ++p) acc += AT(U1, i, p, ld1) * AT(U2, p, j, ld2);
      AT(R, i, j, ldr) = acc;
    }
}

/* Upper triangular transpose of a lower triangular L: U = L^T. */
static void transpose_lower(int64_t b, const double* L, int64_t ldl, double* U, int64_t ldu) {
  for (int64_t j = 0; j < b; ++j)
    for (int64_t i = 0; i < b; ++i) AT(U, i, j, ldu) = (i <= j) ? AT(L, j, i, ldl) : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 4: CholeskyQR2.                                                 */
/* ------------------------------------------------------------------------ */

#define ORA_VARIANT_PRINTED_R 1  /* R = L^T Lbar^T as printed (R1 not applied)  */
#define ORA_VARIANT_PRINTED_H 2  /* H = H + Hbar as printed (R2 not applied)     */

/*
 * Q (q x b) in place -> orthonormal Q and upper triangular R (b x b), with
 * Q_in = Q_out R.  Returns 0, or 1 / 2 if the Cholesky factorisation of step
 * S2 / S5 broke down (then Q and R are left partially updated).
 */
int ora_cholqr2(int64_t q, int64_t b, double* Q, int64_t ldq, double* R, int64_t ldr, int variant) {
  double* L = (double*)calloc((size_t)(b * b), sizeof(double));
  double* Lb = (double*)calloc((size_t)(b * b), sizeof(double));
  double* LT = (double*)calloc((size_t)(b * b), sizeof(double));
  double* LbT = (double*)calloc((size_t)(b * b), sizeof(double));
  int rc = 0;
  mat_tn(b, b, q, Q, ldq, Q, ldq, L, b);                 /* S1  W = Q^T Q          */
  if (ora_chol(b, L, b)) { rc = 1; goto done; }          /* S2  W = L L^T          */
  ora_trsm_rlt(q, b, Q, ldq, L, b);                      /* S3  Q = Q L^{-T}       */
  mat_tn(b, b, q, Q, ldq, Q, ldq, Lb, b);                /* S4  Wbar = Q^T Q       */
  if (ora_chol(b, Lb, b)) { rc = 2; goto done; }         /* S5  Wbar = Lb Lb^T (R3) */
  ora_trsm_rlt(q, b, Q, ldq, Lb, b);                     /* S6  Q = Q Lb^{-T}      */
  transpose_lower(b, L, b, LT, b);
  transpose_lower(b, Lb, b, LbT, b);
  if (variant & ORA_VARIANT_PRINTED_R)
    upper_times_upper(b, LT, b, LbT, b, R, ldr);         /* S7 as printed          */
  else
    upper_times_upper(b, LbT, b, LT, b, R, ldr);         /* S7  R = Lb^T L^T (R1)  */
done:
  free(L); free(Lb); free(LT); free(LbT);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 5: CGS-CQR2, orthogonalise Q (q x b) against P (q x s).          */
/* ------------------------------------------------------------------------ */

/*
 * Outputs Q (in place), H (s x b) and R (b x b) with
 *   Q_in = P H + Q_out R,  P^T Q_out = 0,  Q_out^T Q_out = I  (to rounding).
 * Returns 0, or 1 / 2 if the Cholesky factorisation of step S4 / S9 broke down.
 */
int ora_cgs_cqr2(int64_t q, int64_t b, int64_t s, double* Q, int64_t ldq, const double* P, int64_t ldp,
                 double* H, int64_t ldh, double* R, int64_t ldr, int variant) {
  double* Hb = (double*)calloc((size_t)((s > 0 ? s : 1) * b), sizeof(double));
  double* L = (double*)calloc((size_t)(b * b), sizeof(double));
  double* Lb = (double*)calloc((size_t)(b * b), sizeof(double));
  double* LT = (double*)calloc((size_t)(b * b), sizeof(double));
  double* LbT = (double*)calloc((size_t)(b * b), sizeof(double));
  int rc = 0;
  mat_tn(s, b, q, P, ldp, Q, ldq, H, ldh);               /* S1  H = P^T Q          */
  mat_sub_nn(q, b, s, P, ldp, H, ldh, Q, ldq);           /* S2  Q = Q - P H        */
  mat_tn(b, b, q, Q, ldq, Q, ldq, L, b);                 /* S3  W = Q^T Q          */
  if (ora_chol(b, L, b)) { rc = 1; goto done; }          /* S4  W = L L^T          */
  ora_trsm_rlt(q, b, Q, ldq, L, b);                      /* S5  Q = Q L^{-T}       */
  mat_tn(s, b, q, P, ldp, Q, ldq, Hb, s > 0 ? s : 1);    /* S6  Hbar = P^T Q       */
  mat_sub_nn(q, b, s, P, ldp, Hb, s > 0 ? s : 1, Q, ldq);/* S7  Q = Q - P Hbar     */
  mat_tn(b, b, q, Q, ldq, Q, ldq, Lb, b);                /* S8  W = Q^T Q          */
  if (ora_chol(b, Lb, b)) { rc = 2; goto done; }         /* S9  W = Lb Lb^T        */
  ora_trsm_rlt(q, b, Q, ldq, Lb, b);                     /* S10 Q = Q Lb^{-T}      */
  transpose_lower(b, L, b, LT, b);
  transpose_lower(b, Lb, b, LbT, b);
  if (variant & ORA_VARIANT_PRINTED_R)
    upper_times_upper(b, LT, b, LbT, b, R, ldr);         /* S11 as printed         */
  else
    upper_times_upper(b, LbT, b, LT, b, R, ldr);         /* S11 R = Lb^T L^T (R1)  */
  /* S12: H = H + Hbar L^T (R2), or H = H + Hbar as printed. */
  for (int64_t j = 0; j < b; ++j)
    for (int64_t i = 0; i < s; ++i) {
      double add;
      if (variant & ORA_VARIANT_PRINTED_H) {
        add = AT(Hb, i, j, s);
      } else {
        add = 0.0;
        for (int64_t p = j; p < b; ++p) add += AT(Hb, i, p, s) * AT(LT, p, j, b);
      }
      AT(H, i, j, ldh) += add;
    }
done:
  free(Hb); free(L); free(Lb); free(LT); free(LbT);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Fallback: classical Gram-Schmidt with re-orthogonalisation (CGS2).        */
/* ------------------------------------------------------------------------ */

/*
 * Re-does columns c0 .. c0+w-1 of Q one at a time as Algorithm 5 with b = 1
 * (reading R5): column c is orthogonalised against Q[:, 0:c].  The columns
 * must hold the block's original contents on entry.  Writes R[0:c+1, c].
 * Returns the number of exactly dependent columns found (reading R8).
 */
static int cgs2_columns(int64_t q, int64_t c0, int64_t w, double* Q, int64_t ldq, double* R, int64_t ldr) {
  int nzero = 0;
  for (int64_t c = c0; c < c0 + w; ++c) {
    double* v = &AT(Q, 0, c, ldq);
    double* h = &AT(R, 0, c, ldr);
    double rcc = 0.0;
    int rc;
    if (c == 0) {
      rc = ora_cholqr2(q, 1, v, ldq, &rcc, 1, 0);       /* Algorithm 4, b = 1 */
    } else {
      rc = ora_cgs_cqr2(q, 1, c, v, ldq, Q, ldq, h, ldr, &rcc, 1, 0);
    }
    if (rc != 0) {
      /* The remainder after projection has zero (or NaN) norm. */
      for (int64_t i = 0; i < q; ++i) v[i] = 0.0;
      rcc = 0.0;
      ++nzero;
    }
    AT(R, c, c, ldr) = rcc;
  }
  return nzero;
}

/*
 * Algorithm 5 with the Section 3 breakdown fallback, for callers that keep
 * the basis and the block side by side: X holds [P | Q] with P = X[:, 0:s]
 * (orthonormal columns) and the block Q = X[:, s:s+w].  Q is orthogonalised
 * against P (H = s x w coefficients, R = w x w triangle, Q_in = P H + Q_out R).
 * If either Cholesky factorisation breaks down, Q is restored and redone
 * column by column by CGS2 against P and its own earlier columns (reading R5,
 * R8 for an exactly dependent column).  s = 0 is Algorithm 4 with the same
 * fallback.  Returns 0, 1 (fallback taken) or 3 (fallback with a zero column).
 */
int ora_orth_against_fb(int64_t q, int64_t s, int64_t w, double* X, int64_t ldx, double* H, int64_t ldh, double* R,
                        int64_t ldr) {
  double* save = (double*)malloc((size_t)(q * w + 1) * sizeof(double));
  for (int64_t c = 0; c < w; ++c) memcpy(&save[c * q], &AT(X, 0, s + c, ldx), (size_t)q * sizeof(double));
  int rc = ora_cgs_cqr2(q, w, s, &AT(X, 0, s, ldx), ldx, X, ldx, H, ldh, R, ldr, 0);
  if (rc == 0) {
    free(save);
    return 0;
  }
  for (int64_t c = 0; c < w; ++c) memcpy(&AT(X, 0, s + c, ldx), &save[c * q], (size_t)q * sizeof(double));
  const int64_t t = s + w;
  double* Rt = (double*)calloc((size_t)(t * t), sizeof(double));
  const int nz = cgs2_columns(q, s, w, X, ldx, Rt, t);
  for (int64_t c = 0; c < w; ++c) {
    for (int64_t i = 0; i < s; ++i) AT(H, i, c, ldh) = AT(Rt, i, s + c, t);
    for (int64_t i = 0; i < w; ++i) AT(R, i, c, ldr) = AT(Rt, s + i, s + c, t);
  }
  free(Rt);
  free(save);
  return nz > 0 ? 3 : 1;
}

/* ------------------------------------------------------------------------ */
/* Loop invariants of Algorithm 3 after a finished column block.             */
/* ------------------------------------------------------------------------ */

/*
 * With J finished columns (Q0 = copy of the input Y):
 *   I1  ||Q[:, :J]^T Q[:, :J] - I||_F / (q eps)
 *   I2  ||Y[:, :J] - Q[:, :J] R[:J, :J]||_F / (q eps ||Y[:, :J]||_F)
 *   I3  R[:J, :J] upper triangular with exact zeros below the diagonal and
 *       a diagonal > 0 (or == 0 exactly for a dependent column)      -> 0 / 1
 *   I4  Q[:, J:] bit-identical to Y[:, J:]                             -> 0 / 1
 * Y0 is the input with leading dimension ldy0 (>= q).  out[0..3] receives the
 * running maxima of I1, I2 and the violation flags (the caller zeroes it
 * before the first call).  Exported so that tests can feed it factorizations
 * with planted violations.
 */
void ora_check_invariants(int64_t q, int64_t r, int64_t J, const double* Y0, int64_t ldy0, const double* Q,
                          int64_t ldq, const double* R, int64_t ldr, double* out) {
  const double eps = 0x1p-52;
  double orth = 0.0, rec = 0.0, ynorm = 0.0;
  for (int64_t j = 0; j < J; ++j)
    for (int64_t i = 0; i < J; ++i) {
      double acc = 0.0;
      for (int64_t p = 0; p < q; ++p) acc += AT(Q, p, i, ldq) * AT(Q, p, j, ldq);
      double d = acc - (i == j ? 1.0 : 0.0);
      orth += d * d;
    }
  for (int64_t j = 0; j < J; ++j)
    for (int64_t i = 0; i < q; ++i) {
      double acc = 0.0;
      for (int64_t p = 0; p <= j; ++p) acc += AT(Q, i, p, ldq) * AT(R, p, j, ldr);
      double d = AT(Y0, i, j, ldy0) - acc;
      rec += d * d;
      ynorm += AT(Y0, i, j, ldy0) * AT(Y0, i, j, ldy0);
    }
  double i1 = sqrt(orth) / ((double)q * eps);
  double i2 = (ynorm > 0.0) ? sqrt(rec) / ((double)q * eps * sqrt(ynorm)) : 0.0;
  int bad3 = 0, bad4 = 0;
  for (int64_t j = 0; j < J; ++j) {
    for (int64_t i = j + 1; i < J; ++i)
      if (AT(R, i, j, ldr) != 0.0) bad3 = 1;
    if (!(AT(R, j, j, ldr) >= 0.0)) bad3 = 1;
  }
  for (int64_t j = J; j < r; ++j)
    for (int64_t i = 0; i < q; ++i)
      if (memcmp(&AT(Q, i, j, ldq), &AT(Y0, i, j, ldy0), sizeof(double)) != 0) bad4 = 1;
  if (i1 > out[0]) out[0] = i1;
  if (i2 > out[1]) out[1] = i2;
  if (bad3) out[2] = 1.0;
  if (bad4) out[3] = 1.0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 3: CGS-QR.                                                       */
/* ------------------------------------------------------------------------ */

/*
 * Y (q x r, q >= r) is overwritten by Q; R (r x r) receives the upper
 * triangular factor.  Block width b >= 1; k = ceil(r / b) blocks (R6).
 * block_flags (length k, may be NULL): bit 0 = the block fell back to CGS2,
 * bit 1 = the block holds an exactly dependent column.
 * info (may be NULL): 0, or the 1-based index of the first fallback block.
 * inv (length 4, may be NULL): if non-NULL the loop invariants I1..I4 are
 * checked after every block and their worst values stored there.
 * Returns 0, or a negative argument index.
 */
int ora_cgs_qr(int64_t q, int64_t r, int64_t b, double* Y, int64_t ldy, double* R, int64_t ldr, int variant,
               int32_t* block_flags, int32_t* info, double* inv) {
  if (q < 0) return -1;
  if (r < 0 || r > q) return -2;
  if (b < 1) return -3;
  if (ldy < (q > 1 ? q : 1)) return -5;
  if (ldr < (r > 1 ? r : 1)) return -7;
  const int64_t k = (r + b - 1) / b;
  double* Y0 = NULL;
  double* save = (double*)malloc((size_t)(q * b + 1) * sizeof(double));
  if (inv) {
    Y0 = (double*)malloc((size_t)(q * r + 1) * sizeof(double));
    for (int64_t j = 0; j < r; ++j) memcpy(&Y0[j * q], &AT(Y, 0, j, ldy), (size_t)q * sizeof(double));
    inv[0] = inv[1] = inv[2] = inv[3] = 0.0;
  }
  if (info) *info = 0;
  for (int64_t j = 0; j < r; ++j)
    for (int64_t i = 0; i < r; ++i) AT(R, i, j, ldr) = 0.0;

  for (int64_t blk = 0; blk < k; ++blk) {
    const int64_t s = blk * b;                      /* columns already finished */
    const int64_t w = (r - s < b) ? (r - s) : b;    /* this block's width (R6)  */
    double* Qj = &AT(Y, 0, s, ldy);
    double* Rjj = &AT(R, s, s, ldr);
    double* Hj = &AT(R, 0, s, ldr);
    int32_t flags = 0;
    for (int64_t c = 0; c < w; ++c) memcpy(&save[c * q], &AT(Qj, 0, c, ldy), (size_t)q * sizeof(double));
    int rc;
    if (blk == 0)
      rc = ora_cholqr2(q, w, Qj, ldy, Rjj, ldr, variant);                 /* Alg. 3 S1 */
    else
      rc = ora_cgs_cqr2(q, w, s, Qj, ldy, Y, ldy, Hj, ldr, Rjj, ldr, variant); /* Alg. 3 S2 */
    if (rc != 0) {
      /* Cholesky breakdown: restore the block and redo it by CGS2 (R5). */
      for (int64_t c = 0; c < w; ++c) memcpy(&AT(Qj, 0, c, ldy), &save[c * q], (size_t)q * sizeof(double));
      for (int64_t c = s; c < s + w; ++c)
        for (int64_t i = 0; i < r; ++i) AT(R, i, c, ldr) = 0.0;
      flags |= 1;
      if (cgs2_columns(q, s, w, Y, ldy, R, ldr) > 0) flags |= 2;
      if (info && *info == 0) *info = (int32_t)(blk + 1);
    }
    if (block_flags) block_flags[blk] = flags;
    if (inv) ora_check_invariants(q, r, s + w, Y0, q, Y, ldy, R, ldr, inv);
  }
  free(save);
  free(Y0);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* O-def: Householder QR with positive diag(R).                              */
/* ------------------------------------------------------------------------ */

/*
 * Thin QR of Y (q x r, q >= r) by unblocked Householder reflections
 * [GVL3 Alg. 5.2.1], Q formed explicitly by applying the reflectors to the
 * first r columns of the identity, then every i with R_ii < 0 has row i of R
 * and column i of Q negated, so that diag(R) >= 0 and the factorisation is
 * the unique one for full column rank.  Y is not modified.
 */
int ora_householder_qr(int64_t q, int64_t r, const double* Y, int64_t ldy, double* Q, int64_t ldq, double* R,
                       int64_t ldr) {
  if (q < 0) return -1;
  if (r < 0 || r > q) return -2;
  double* A = (double*)malloc((size_t)(q * r + 1) * sizeof(double));
  double* V = (double*)calloc((size_t)(q * r + 1), sizeof(double)); /* reflector vectors */
  double* beta = (double*)calloc((size_t)(r + 1), sizeof(double));  /* H = I - beta v v^T */
  for (int64_t j = 0; j < r; ++j)
    for (int64_t i = 0; i < q; ++i) A[i + j * q] = AT(Y, i, j, ldy);
  for (int64_t c = 0; c < r; ++c) {
    double sigma = 0.0;
    for (int64_t i = c; i < q; ++i) sigma += A[i + c * q] * A[i + c * q];
    double norm = sqrt(sigma);
    double* v = &V[c * q];
    if (norm == 0.0) { beta[c] = 0.0; continue; }
    double x0 = A[c + c * q];
    double alpha = (x0 >= 0.0) ? -norm : norm;   /* avoid cancellation in x0 - alpha */
    for (int64_t i = c; i < q; ++i) v[i] = A[i + c * q];
    v[c] = x0 - alpha;
    double vtv = 0.0;
    for (int64_t i = c; i < q; ++i) vtv += v[i] * v[i];
    beta[c] = 2.0 / vtv;
    for (int64_t j = c; j < r; ++j) {
      double dot = 0.0;
      for (int64_t i = c; i < q; ++i) dot += v[i] * A[i + j * q];
      dot *= beta[c];
      for (int64_t i = c; i < q; ++i) A[i + j * q] -= dot * v[i];
    }
    A[c + c * q] = alpha;
    for (int64_t i = c + 1; i < q; ++i) A[i + c * q] = 0.0;
  }
  for (int64_t j = 0; j < r; ++j)
    for (int64_t i = 0; i < r; ++i) AT(R, i, j, ldr) = (i <= j) ? A[i + j * q] : 0.0;
  /* Q = H_0 H_1 ... H_{r-1} I[:, :r], applied right to left. */
  for (int64_t j = 0; j < r; ++j)
    for (int64_t i = 0; i < q; ++i) AT(Q, i, j, ldq) = (i == j) ? 1.0 : 0.0;
  for (int64_t c = r - 1; c >= 0; --c) {
    if (beta[c] == 0.0) continue;
    const double* v = &V[c * q];
    for (int64_t j = 0; j < r; ++j) {
      double dot = 0.0;
      for (int64_t i = c; i < q; ++i) dot += v[i] * AT(Q, i, j, ldq);
      dot *= beta[c];
      for (int64_t i = c; i < q; ++i) AT(Q, i, j, ldq) -= dot * v[i];
    }
  }
  for (int64_t i = 0; i < r; ++i) {
    if (AT(R, i, i, ldr) < 0.0) {
      for (int64_t j = i; j < r; ++j) AT(R, i, j, ldr) = -AT(R, i, j, ldr);
      for (int64_t p = 0; p < q; ++p) AT(Q, p, i, ldq) = -AT(Q, p, i, ldq);
    }
  }
  free(A); free(V); free(beta);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Solve and its adjoint (not in the paper; the factorisation's use).        */
/* ------------------------------------------------------------------------ */

/*
 * x = R^{-1} (Q^T b) for square n x n factors: c = Q^T b, then back
 * substitution on R x = c.  Returns 0, or i+1 if R_ii == 0.
 */
int ora_qr_solve(int64_t n, const double* Q, int64_t ldq, const double* R, int64_t ldr, const double* b,
                 double* x) {
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int64_t p = 0; p < n; ++p) acc += AT(Q, p, i, ldq) * b[p];
    x[i] = acc;
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    double v = x[i];
    for (int64_t j = i + 1; j < n; ++j) v -= AT(R, i, j, ldr) * x[j];
    if (AT(R, i, i, ldr) == 0.0) return (int)(i + 1);
    x[i] = v / AT(R, i, i, ldr);
  }
  return 0;
}

/*
 * Adjoint of x = A^{-1} b with A = Q R, for a loss with gradient w = dL/dx:
 *   lambda = A^{-T} w = Q (R^{-T} w)   (forward substitution on R^T u = w)
 *   dL/dA  = -lambda x^T,   dL/db = lambda.
 * dA is n x n with leading dimension ldda.  Returns 0, or i+1 if R_ii == 0.
 */
int ora_qr_solve_grad(int64_t n, const double* Q, int64_t ldq, const double* R, int64_t ldr, const double* x,
                      const double* w, double* dA, int64_t ldda, double* db) {
  double* u = (double*)malloc((size_t)(n + 1) * sizeof(double));
  for (int64_t i = 0; i < n; ++i) {
    double v = w[i];
    for (int64_t p = 0; p < i; ++p) v -= AT(R, p, i, ldr) * u[p];
    if (AT(R, i, i, ldr) == 0.0) { free(u); return (int)(i + 1); }
    u[i] = v / AT(R, i, i, ldr);
  }
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int64_t p = 0; p < n; ++p) acc += AT(Q, i, p, ldq) * u[p];
    db[i] = acc;
  }
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i) AT(dA, i, j, ldda) = -db[i] * x[j];
  free(u);
  return 0;
}

/* Number of OpenMP threads the oracle's parallel loops use (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int ora_num_threads(void) { return omp_get_max_threads(); }
#else
int ora_num_threads(void) { return 1; }
#endif
