// Truncated SVD drivers of the paper's Section 2 on one GPU: RandSVD
// (Algorithm 1, randomized subspace iteration) and LancSVD (Algorithm 2, block
// Golub-Kahan-Lanczos with full one-sided orthogonalisation and the basic
// restart), built on the library's CGS-QR (Algorithm 3), CholeskyQR2
// (Algorithm 4) and CGS-CQR2 (Algorithm 5).
//
// Every step runs on the device, stream-ordered, with no host round trip:
//   * the products with A (A X and A^T X, Table 1 "SpMM*/GEMM" rows; HBM-bound
//     for the paper's block widths) on the FP64 MFMA GEMM kernels, or on the
//     CSR kernels of spmm.hip for a sparse A;
//   * the orthogonalisations through cqr_orth / cqr_orth_against /
//     cqr_factor, breakdown fallback included (device-side);
//   * the small r x r SVD (the paper runs LAPACK's GESVD on the CPU after a
//     PCIe transfer) by a one-workgroup one-sided Jacobi kernel;
//   * B_k assembled from the triangular factors by a small kernel.
//
// Readings (where the text is garbled): LancSVD S8 computes V = P_k Vbar (the
// printed Vbar^T does not follow from B_k = Ubar S Vbar^T); B_k carries L_i =
// (R factor of S3)^T on its diagonal blocks and R_i (R factor of S5) below
// them; the start blocks are caller inputs (the random numbers are passed in).
#include <cmath>
#include <cstring>

#include "internal.h"
#include "../../include/cqr.h"

namespace cqr {
namespace {

#define SVD_TRY(expr)                                        \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return CQR_ERR_HIP_BASE - (int)e_; \
  } while (0)
#define SVD_RC(expr)          \
  do {                        \
    int rc_ = (expr);         \
    if (rc_ != CQR_OK) return rc_; \
  } while (0)

constexpr int kJThreads = 1024;
constexpr int kJWaves = kJThreads / 64;
constexpr int kMaxR = 256;
constexpr int kMaxSweeps = 60;

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Player at seat x in round t of the circle-method tournament of rr (even)
// players: seat 0 is fixed, the others rotate; seats x and rr-1-x meet.
__device__ __forceinline__ int seat(int x, int t, int rr) { return x == 0 ? 0 : (x - 1 + t) % (rr - 1) + 1; }

// One-sided Jacobi (Hestenes) SVD of a small r x r matrix B in one workgroup:
// columns i < j of U := B are rotated so that they become orthogonal
// (u_i^T u_j = 0), the same rotations accumulate in V := I, until a sweep over
// all pairs leaves every pair with |u_i^T u_j| <= tol sqrt(|u_i|^2 |u_j|^2).
// Then B V = U diag(|u_i|): sigma_i = |u_i|, the columns of U normalised, and
// the triplets sorted by decreasing sigma.  The pairs of a sweep are visited in
// rr - 1 rounds of disjoint pairs (one wave per pair), so every round is one
// parallel step.  Uw, Vw: r x r work arrays (ld r) in global memory.
__global__ void __launch_bounds__(kJThreads)
jacobi_svd_kernel(int r, const double* __restrict__ B, int64_t ldb, double* Uw, double* Vw, double* U, int64_t ldu,
                  double* sigma, double* V, int64_t ldv, int32_t* sweeps_out, double tol) {
  __shared__ int sRot;
  __shared__ double sS[kMaxR];
  __shared__ int sPerm[kMaxR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int idx = tid; idx < r * r; idx += kJThreads) {
    const int i = idx % r, j = idx / r;
    Uw[idx] = B[i + (int64_t)j * ldb];
    Vw[idx] = (i == j) ? 1.0 : 0.0;
  }
  const int rr = r + (r & 1);
  int sweep = 0;
  bool converged = (r < 2);
  __syncthreads();
  for (; sweep < kMaxSweeps && !converged; ++sweep) {
    if (tid == 0) sRot = 0;
    __syncthreads();
    for (int t = 0; t < rr - 1; ++t) {
      for (int pi = wave; pi < rr / 2; pi += kJWaves) {
        const int a = seat(pi, t, rr), c = seat(rr - 1 - pi, t, rr);
        if (a >= r || c >= r) continue;
        const int i = a < c ? a : c, j = a < c ? c : a;
        double* ui = Uw + (int64_t)i * r;
        double* uj = Uw + (int64_t)j * r;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int e = lane; e < r; e += 64) {
          const double x = ui[e], y = uj[e];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
        al = wsum(al);
        be = wsum(be);
        ga = wsum(ga);
        if (fabs(ga) > tol * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double tt = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
          double* vi = Vw + (int64_t)i * r;
          double* vj = Vw + (int64_t)j * r;
          for (int e = lane; e < r; e += 64) {
            const double x = ui[e], y = uj[e];
            ui[e] = cs * x - sn * y;
            uj[e] = sn * x + cs * y;
            const double p = vi[e], q = vj[e];
            vi[e] = cs * p - sn * q;
            vj[e] = sn * p + cs * q;
          }
          if (lane == 0) atomicAdd(&sRot, 1);
        }
      }
      __syncthreads();
    }
    converged = (sRot == 0);
    __syncthreads();
  }
  // sigma_i = |u_i| (fixed-order sums), then the ranks of the sort.
  for (int col = wave; col < r; col += kJWaves) {
    const double* u = Uw + (int64_t)col * r;
    double s = 0.0;
    for (int e = lane; e < r; e += 64) s += u[e] * u[e];
    s = wsum(s);
    if (lane == 0) sS[col] = sqrt(s);
  }
  __syncthreads();
  for (int i = tid; i < r; i += kJThreads) {
    const double si = sS[i];
    int rank = 0;
    for (int j = 0; j < r; ++j) rank += (sS[j] > si || (sS[j] == si && j < i)) ? 1 : 0;
    sPerm[rank] = i;
  }
  __syncthreads();
  for (int k = wave; k < r; k += kJWaves) {
    const int src = sPerm[k];
    const double s = sS[src];
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    for (int e = lane; e < r; e += 64) {
      U[e + (int64_t)k * ldu] = Uw[e + (int64_t)src * r] * inv;
      V[e + (int64_t)k * ldv] = Vw[e + (int64_t)src * r];
    }
    if (lane == 0) sigma[k] = s;
  }
  if (tid == 0 && sweeps_out) sweeps_out[0] = converged ? sweep : -sweep;
}

// B_k (r x r, k = r / b blocks): diagonal blocks L_i = (R factor of S3)^T,
// the blocks below them R_i (R factor of S5), zero elsewhere.  Rl and Rr hold
// the b x b upper triangles side by side (b x r, ld b).
__global__ void assemble_bk_kernel(int r, int b, const double* __restrict__ Rl, const double* __restrict__ Rr,
                                   double* Bk) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= r * r) return;
  const int i = idx % r, j = idx / r;
  const int bi = i / b, bj = j / b, ii = i % b, jj = j % b;
  double v = 0.0;
  if (bi == bj && ii >= jj) v = Rl[jj + (int64_t)(bj * b + ii) * b];        // (R_S3^T)(ii, jj) = R_S3(jj, ii)
  else if (bi == bj + 1 && ii <= jj) v = Rr[ii + (int64_t)(bj * b + jj) * b];  // R_i(ii, jj)
  Bk[idx] = v;
}

// res[j] = |T[:, j] - sigma_j U[:, j]|_2 / sigma_j, one workgroup per column
// (fixed-order reduction).
__global__ void __launch_bounds__(256)
residual_kernel(int64_t m, const double* __restrict__ T, int64_t ldt, const double* __restrict__ U, int64_t ldu,
                const double* __restrict__ sigma, double* res) {
  __shared__ double sRed[4];
  const int j = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double s = sigma[j];
  const double* t = T + (int64_t)j * ldt;
  const double* u = U + (int64_t)j * ldu;
  double acc = 0.0;
  for (int64_t i = tid; i < m; i += 256) {
    const double d = t[i] - s * u[i];
    acc += d * d;
  }
  acc = wsum(acc);
  if (lane == 0) sRed[wave] = acc;
  __syncthreads();
  if (tid == 0) res[j] = sqrt((sRed[0] + sRed[1]) + (sRed[2] + sRed[3])) / s;
}

// Fold the info of one orthogonalisation into the driver's count.
__global__ void fold_info_kernel(const int32_t* __restrict__ one, int32_t* acc) {
  const int32_t v = one[0];
  if (v == CQR_INFO_WAIT_ABANDONED)
    acc[0] = CQR_INFO_WAIT_ABANDONED;
  else if (v != 0 && acc[0] != CQR_INFO_WAIT_ABANDONED)
    acc[0] += 1;
}

__global__ void zero_i32_kernel(int32_t* p) { p[0] = 0; }

hipError_t launch_jacobi(int r, const double* B, int64_t ldb, double* Uw, double* Vw, double* U, int64_t ldu,
                         double* sigma, double* V, int64_t ldv, int32_t* sweeps, hipStream_t st) {
  const double tol = sqrt((double)r) * 2.220446049250313e-16;
  const int slot = prof_begin(st);
  hipLaunchKernelGGL(jacobi_svd_kernel, dim3(1), dim3(kJThreads), 0, st, r, B, ldb, Uw, Vw, U, ldu, sigma, V, ldv,
                     sweeps, tol);
  const hipError_t e = hipGetLastError();
  prof_end(slot, ROLE_SVD, st, 0.0, 0.0);
  return e;
}

// ------------------------------------------------------------- workspaces
size_t gemm_part_doubles() { return (size_t)8 << 20; }  // 64 MiB of split-K partial sums

struct LancWork {
  double* Pbar;  // m x (r + b): Qbar_1 .. Qbar_{k+1}
  double* Pn;    // n x r:       Q_1 .. Q_k
  double* Rl;    // b x r: R factors of S3 (L_i^T)
  double* Rr;    // b x r: R factors of S5 (R_i)
  double* H;     // (r + b) x b: projections of the orthogonalisations (not used further)
  double* Bk;    // r x r
  double* Ub;    // r x r
  double* Vb;    // r x r
  double* Uw;    // r x r
  double* Vw;    // r x r
  double* sig;   // r
  int32_t* one;  // info of one orthogonalisation, Jacobi sweeps
  double* part;  // split-K partial sums of A^T X
  void* ow;      // workspace of the orthogonalisations
  size_t ow_bytes;
};

size_t lanc_layout(int64_t m, int64_t n, int64_t r, int64_t b, char* base, LancWork* w) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += a256(bytes);
    return p;
  };
  LancWork t;
  LancWork* o = w ? w : &t;
  const size_t d = sizeof(double);
  o->Pbar = (double*)take((size_t)m * (size_t)(r + b) * d);
  o->Pn = (double*)take((size_t)n * (size_t)r * d);
  o->Rl = (double*)take((size_t)b * (size_t)r * d);
  o->Rr = (double*)take((size_t)b * (size_t)r * d);
  o->H = (double*)take((size_t)(r + b) * (size_t)b * d);
  o->Bk = (double*)take((size_t)r * r * d);
  o->Ub = (double*)take((size_t)r * r * d);
  o->Vb = (double*)take((size_t)r * r * d);
  o->Uw = (double*)take((size_t)r * r * d);
  o->Vw = (double*)take((size_t)r * r * d);
  o->sig = (double*)take((size_t)r * d);
  o->one = (int32_t*)take(256);
  o->part = (double*)take(gemm_part_doubles() * d);
  size_t ob = 0;
  cqr_workspace_size(m > n ? m : n, r + b, b, &ob);
  o->ow_bytes = ob;
  o->ow = take(ob);
  return off;
}

struct RandWork {
  double* Ybar;  // m x r
  double* Qn;    // n x r
  double* Rbar;  // r x r
  double* Rn;    // r x r
  double* Ub;
  double* Vb;
  double* Uw;
  double* Vw;
  double* sig;
  int32_t* one;
  double* part;
  void* fw;  // workspace of the factorisations
  size_t fw_bytes;
};

size_t rand_layout(int64_t m, int64_t n, int64_t r, int64_t b, char* base, RandWork* w) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += a256(bytes);
    return p;
  };
  RandWork t;
  RandWork* o = w ? w : &t;
  const size_t d = sizeof(double);
  o->Ybar = (double*)take((size_t)m * (size_t)r * d);
  o->Qn = (double*)take((size_t)n * (size_t)r * d);
  o->Rbar = (double*)take((size_t)r * r * d);
  o->Rn = (double*)take((size_t)r * r * d);
  o->Ub = (double*)take((size_t)r * r * d);
  o->Vb = (double*)take((size_t)r * r * d);
  o->Uw = (double*)take((size_t)r * r * d);
  o->Vw = (double*)take((size_t)r * r * d);
  o->sig = (double*)take((size_t)r * d);
  o->one = (int32_t*)take(256);
  o->part = (double*)take(gemm_part_doubles() * d);
  size_t f1 = 0, f2 = 0;
  cqr_workspace_size(m, r, b, &f1);
  cqr_workspace_size(n, r, b, &f2);
  o->fw_bytes = f1 > f2 ? f1 : f2;
  o->fw = take(o->fw_bytes);
  return off;
}

// The operator A: dense column-major FP64 (lda), or CSR (with its transpose
// given as a second CSR, the form the sparse products need).
struct Op {
  int64_t m, n;
  const double* A;
  int64_t lda;
  const SparseCsr* S;
};

// C (m x w) = A X (X: n x w, ldx), or C (n x w) = A^T X (X: m x w).
int op_apply(const Op& op, bool trans, int64_t w, const double* X, int64_t ldx, double* C, int64_t ldc, double* part,
             hipStream_t st) {
  if (op.S) {
    SVD_TRY(spmm(*op.S, trans, w, X, ldx, C, ldc, st));
    return CQR_OK;
  }
  const double flops = 2.0 * (double)op.m * (double)op.n * (double)w;
  if (trans)
    SVD_TRY(gemm_tn(ROLE_APROD, op.n, w, op.m, 1.0, op.A, op.lda, X, ldx, 0.0, C, ldc, part, gemm_part_doubles(),
                    nullptr, st, flops));
  else
    SVD_TRY(gemm_nn(ROLE_APROD, op.m, w, op.n, 1.0, op.A, op.lda, X, ldx, 0.0, C, ldc, nullptr, st, flops));
  return CQR_OK;
}

int fold(const int32_t* one, int32_t* info, hipStream_t st) {
  if (!info) return CQR_OK;
  hipLaunchKernelGGL(fold_info_kernel, dim3(1), dim3(1), 0, st, one, info);
  SVD_TRY(hipGetLastError());
  return CQR_OK;
}

int lancsvd(const Op& op, int64_t r, int64_t b, int p, const double* Qbar1, int64_t ldq, double* U, int64_t ldu,
            double* sigma, double* V, int64_t ldv, int32_t* info, void* work, size_t work_bytes, hipStream_t st) {
  const int64_t m = op.m, n = op.n;
  LancWork ws;
  if (!work || work_bytes < lanc_layout(m, n, r, b, nullptr, nullptr)) return CQR_ERR_WORKSPACE;
  lanc_layout(m, n, r, b, (char*)work, &ws);
  const int64_t k = r / b;
  if (info) {
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(1), 0, st, info);
    SVD_TRY(hipGetLastError());
  }
  // S1: random orthonormal Qbar_1 (Algorithm 4) from the caller's start block.
  SVD_TRY(copy_matrix(m, b, Qbar1, ldq, ws.Pbar, m, nullptr, st));
  SVD_RC(cqr_orth(m, b, ws.Pbar, m, ws.Bk, b, ws.ow, ws.ow_bytes, ws.one, st));
  SVD_RC(fold(ws.one, info, st));
  for (int j = 0; j < p; ++j) {
    for (int64_t i = 0; i < k; ++i) {
      double* Qi = ws.Pn + i * b * n;
      double* Qbi = ws.Pbar + i * b * m;
      double* Qbn = ws.Pbar + (i + 1) * b * m;
      SVD_RC(op_apply(op, true, b, Qbi, m, Qi, n, ws.part, st));  // S2  Q_i = A^T Qbar_i
      if (i == 0)                                                  // S3a Algorithm 4
        SVD_RC(cqr_orth(n, b, Qi, n, ws.Rl, b, ws.ow, ws.ow_bytes, ws.one, st));
      else                                                         // S3b Algorithm 5 against P_{i-1}
        SVD_RC(cqr_orth_against(n, b, i * b, Qi, n, ws.Pn, n, ws.H, i * b, ws.Rl + i * b * b, b, ws.ow, ws.ow_bytes,
                                ws.one, st));
      SVD_RC(fold(ws.one, info, st));
      SVD_RC(op_apply(op, false, b, Qi, n, Qbn, m, ws.part, st));  // S4  Qbar_{i+1} = A Q_i
      SVD_RC(cqr_orth_against(m, b, (i + 1) * b, Qbn, m, ws.Pbar, m, ws.H, (i + 1) * b, ws.Rr + i * b * b, b,
                              ws.ow, ws.ow_bytes, ws.one, st));   // S5  against Pbar_i
      SVD_RC(fold(ws.one, info, st));
    }
    {
      const int slot = prof_begin(st);
      hipLaunchKernelGGL(assemble_bk_kernel, dim3((unsigned)((r * r + 255) / 256)), dim3(256), 0, st, (int)r, (int)b,
                         ws.Rl, ws.Rr, ws.Bk);
      SVD_TRY(hipGetLastError());
      prof_end(slot, ROLE_SVD, st, 0.0, 0.0);
    }
    SVD_TRY(launch_jacobi((int)r, ws.Bk, r, ws.Uw, ws.Vw, ws.Ub, r, ws.sig, ws.Vb, r, ws.one + 1, st));  // S6
    if (j < p - 1) {
      // S7: Qbar_1 = Pbar_k Ubar_1, formed in the free slot of Qbar_{k+1}.
      double* tmp = ws.Pbar + k * b * m;
      SVD_TRY(gemm_nn(ROLE_SVD, m, b, r, 1.0, ws.Pbar, m, ws.Ub, r, 0.0, tmp, m, nullptr, st,
                      2.0 * (double)b * (double)m * (double)r));
      SVD_TRY(copy_matrix(m, b, tmp, m, ws.Pbar, m, nullptr, st));
    }
  }
  SVD_TRY(gemm_nn(ROLE_SVD, n, r, r, 1.0, ws.Pn, n, ws.Vb, r, 0.0, V, ldv, nullptr, st,
                  2.0 * (double)n * (double)r * (double)r));  // S8  V = P_k Vbar
  SVD_TRY(gemm_nn(ROLE_SVD, m, r, r, 1.0, ws.Pbar, m, ws.Ub, r, 0.0, U, ldu, nullptr, st,
                  2.0 * (double)m * (double)r * (double)r));  // S9  U = Pbar_k Ubar
  SVD_TRY(copy_matrix(r, 1, ws.sig, r, sigma, r, nullptr, st));
  return CQR_OK;
}

int randsvd(const Op& op, int64_t r, int64_t b, int p, const double* Q0, int64_t ldq, double* U, int64_t ldu,
            double* sigma, double* V, int64_t ldv, int32_t* info, void* work, size_t work_bytes, hipStream_t st) {
  const int64_t m = op.m, n = op.n;
  RandWork ws;
  if (!work || work_bytes < rand_layout(m, n, r, b, nullptr, nullptr)) return CQR_ERR_WORKSPACE;
  rand_layout(m, n, r, b, (char*)work, &ws);
  if (info) {
    hipLaunchKernelGGL(zero_i32_kernel, dim3(1), dim3(1), 0, st, info);
    SVD_TRY(hipGetLastError());
  }
  SVD_TRY(copy_matrix(n, r, Q0, ldq, ws.Qn, n, nullptr, st));
  for (int j = 0; j < p; ++j) {
    SVD_RC(op_apply(op, false, r, ws.Qn, n, ws.Ybar, m, ws.part, st));                        // S1 Ybar = A Q
    SVD_RC(cqr_factor(m, r, b, ws.Ybar, m, ws.Rbar, r, ws.fw, ws.fw_bytes, ws.one, nullptr, st));  // S2
    SVD_RC(fold(ws.one, info, st));
    SVD_RC(op_apply(op, true, r, ws.Ybar, m, ws.Qn, n, ws.part, st));                         // S3 Y = A^T Qbar
    SVD_RC(cqr_factor(n, r, b, ws.Qn, n, ws.Rn, r, ws.fw, ws.fw_bytes, ws.one, nullptr, st));      // S4
    SVD_RC(fold(ws.one, info, st));
  }
  SVD_TRY(launch_jacobi((int)r, ws.Rn, r, ws.Uw, ws.Vw, ws.Ub, r, ws.sig, ws.Vb, r, ws.one + 1, st));  // S5
  SVD_TRY(gemm_nn(ROLE_SVD, m, r, r, 1.0, ws.Ybar, m, ws.Vb, r, 0.0, U, ldu, nullptr, st,
                  2.0 * (double)m * (double)r * (double)r));  // S6 U = Qbar_p Vbar
  SVD_TRY(gemm_nn(ROLE_SVD, n, r, r, 1.0, ws.Qn, n, ws.Ub, r, 0.0, V, ldv, nullptr, st,
                  2.0 * (double)n * (double)r * (double)r));  // S7 V = Q_p Ubar
  SVD_TRY(copy_matrix(r, 1, ws.sig, r, sigma, r, nullptr, st));
  return CQR_OK;
}

int check_svd_args(int64_t m, int64_t n, int64_t r, int64_t b, int p) {
  if (m < 1) return -1;
  if (n < 1) return -2;
  if (r < 1 || r > n || r > m) return -3;
  if (b < 1 || r % b != 0) return -4;
  if (p < 1) return -5;
  if (r > kMaxR || b > 256) return CQR_ERR_UNSUPPORTED;
  return CQR_OK;
}

}  // namespace
}  // namespace cqr

using namespace cqr;

extern "C" {

int cqr_svd_workspace_size(int method, int64_t m, int64_t n, int64_t r, int64_t b, size_t* bytes) {
  const int base = method & ~CQR_SVD_SPARSE;
  if (base != CQR_SVD_LANCZOS && base != CQR_SVD_RANDOMIZED) return -1;
  if (m < 1) return -2;
  if (n < 1) return -3;
  if (r < 1 || r > n || r > m) return -4;
  if (b < 1 || r % b != 0) return -5;
  if (r > kMaxR || b > 256) return CQR_ERR_UNSUPPORTED;
  if (!bytes) return -6;
  if (base == CQR_SVD_LANCZOS && r + b > m) return -4;
  *bytes = base == CQR_SVD_LANCZOS ? lanc_layout(m, n, r, b, nullptr, nullptr)
                                   : rand_layout(m, n, r, b, nullptr, nullptr);
  if (method & CQR_SVD_SPARSE) *bytes += a256(spmm_scratch_doubles(m, n) * sizeof(double));
  return CQR_OK;
}

int cqr_lancsvd(int64_t m, int64_t n, const double* A, int64_t lda, int64_t r, int64_t b, int p, const double* Q1,
                int64_t ldq, double* U, int64_t ldu, double* sigma, double* V, int64_t ldv, int32_t* info,
                void* work, size_t work_bytes, void* stream) {
  int rc = check_svd_args(m, n, r, b, p);
  if (rc) return rc;
  if (!A) return -3;
  if (lda < m) return -4;
  if (!Q1) return -8;
  if (ldq < m) return -9;
  if (!U || ldu < m) return -10;
  if (!sigma) return -12;
  if (!V || ldv < n) return -13;
  if (r + b > m) return -5;
  Op op{m, n, A, lda, nullptr};
  return lancsvd(op, r, b, p, Q1, ldq, U, ldu, sigma, V, ldv, info, work, work_bytes, (hipStream_t)stream);
}

int cqr_lancsvd_csr(int64_t m, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col, const double* val,
                    const int32_t* trowptr, const int32_t* tcol, const double* tval, int64_t r, int64_t b, int p,
                    const double* Q1, int64_t ldq, double* U, int64_t ldu, double* sigma, double* V, int64_t ldv,
                    int32_t* info, void* work, size_t work_bytes, void* stream) {
  int rc = check_svd_args(m, n, r, b, p);
  if (rc) return rc;
  if (r + b > m) return -11;
  if (nnz < 0 || nnz > INT32_MAX) return -3;
  if (!rowptr || !trowptr) return -4;
  if (nnz > 0 && (!col || !val || !tcol || !tval)) return -5;
  if (!Q1) return -13;
  if (ldq < m) return -14;
  if (!U || ldu < m) return -15;
  if (!sigma) return -17;
  if (!V || ldv < n) return -18;
  const size_t dense = lanc_layout(m, n, r, b, nullptr, nullptr);
  const size_t need = dense + a256(spmm_scratch_doubles(m, n) * sizeof(double));
  if (!work || work_bytes < need) return CQR_ERR_WORKSPACE;
  SparseCsr S{m, n, nnz, rowptr, col, val, trowptr, tcol, tval, (double*)((char*)work + dense)};
  Op op{m, n, nullptr, m, &S};
  return lancsvd(op, r, b, p, Q1, ldq, U, ldu, sigma, V, ldv, info, work, dense, (hipStream_t)stream);
}

int cqr_randsvd(int64_t m, int64_t n, const double* A, int64_t lda, int64_t r, int64_t b, int p, const double* Q0,
                int64_t ldq, double* U, int64_t ldu, double* sigma, double* V, int64_t ldv, int32_t* info,
                void* work, size_t work_bytes, void* stream) {
  int rc = check_svd_args(m, n, r, b, p);
  if (rc) return rc;
  if (!A) return -3;
  if (lda < m) return -4;
  if (!Q0) return -8;
  if (ldq < n) return -9;
  if (!U || ldu < m) return -10;
  if (!sigma) return -12;
  if (!V || ldv < n) return -13;
  Op op{m, n, A, lda, nullptr};
  return randsvd(op, r, b, p, Q0, ldq, U, ldu, sigma, V, ldv, info, work, work_bytes, (hipStream_t)stream);
}

int cqr_randsvd_csr(int64_t m, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col, const double* val,
                    const int32_t* trowptr, const int32_t* tcol, const double* tval, int64_t r, int64_t b, int p,
                    const double* Q0, int64_t ldq, double* U, int64_t ldu, double* sigma, double* V, int64_t ldv,
                    int32_t* info, void* work, size_t work_bytes, void* stream) {
  int rc = check_svd_args(m, n, r, b, p);
  if (rc) return rc;
  if (nnz < 0 || nnz > INT32_MAX) return -3;
  if (!rowptr || !trowptr) return -4;
  if (nnz > 0 && (!col || !val || !tcol || !tval)) return -5;
  if (!Q0) return -13;
  if (ldq < n) return -14;
  if (!U || ldu < m) return -15;
  if (!sigma) return -17;
  if (!V || ldv < n) return -18;
  const size_t dense = rand_layout(m, n, r, b, nullptr, nullptr);
  const size_t need = dense + a256(spmm_scratch_doubles(m, n) * sizeof(double));
  if (!work || work_bytes < need) return CQR_ERR_WORKSPACE;
  SparseCsr S{m, n, nnz, rowptr, col, val, trowptr, tcol, tval, (double*)((char*)work + dense)};
  Op op{m, n, nullptr, m, &S};
  return randsvd(op, r, b, p, Q0, ldq, U, ldu, sigma, V, ldv, info, work, dense, (hipStream_t)stream);
}

int cqr_small_svd_workspace_size(int64_t r, size_t* bytes) {
  if (r < 1 || r > kMaxR) return -1;
  if (!bytes) return -2;
  *bytes = 2 * a256((size_t)r * r * sizeof(double));
  return CQR_OK;
}

int cqr_small_svd(int64_t r, const double* B, int64_t ldb, double* U, int64_t ldu, double* sigma, double* V,
                  int64_t ldv, int32_t* sweeps, void* work, size_t work_bytes, void* stream) {
  if (r < 1) return -1;
  if (r > kMaxR) return CQR_ERR_UNSUPPORTED;
  if (!B) return -2;
  if (ldb < r) return -3;
  if (!U) return -4;
  if (ldu < r) return -5;
  if (!sigma) return -6;
  if (!V) return -7;
  if (ldv < r) return -8;
  const size_t half = a256((size_t)r * r * sizeof(double));
  if (!work || work_bytes < 2 * half) return CQR_ERR_WORKSPACE;
  double* Uw = (double*)work;
  double* Vw = (double*)((char*)work + half);
  SVD_TRY(launch_jacobi((int)r, B, ldb, Uw, Vw, U, ldu, sigma, V, ldv, sweeps, (hipStream_t)stream));
  return CQR_OK;
}

int cqr_gemm_workspace_size(size_t* bytes) {
  if (!bytes) return -1;
  *bytes = gemm_part_doubles() * sizeof(double);
  return CQR_OK;
}

int cqr_gemm(int trans_a, int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
             const double* B, int64_t ldb, double beta, double* C, int64_t ldc, void* work, size_t work_bytes,
             void* stream) {
  if (trans_a != 0 && trans_a != 1) return -1;
  if (M < 0) return -2;
  if (N < 0) return -3;
  if (K < 0) return -4;
  if (!A && M * K > 0) return -6;
  if (lda < (trans_a ? (K > 1 ? K : 1) : (M > 1 ? M : 1))) return -7;
  if (!B && K * N > 0) return -8;
  if (ldb < (K > 1 ? K : 1)) return -9;
  if (!C && M * N > 0) return -11;
  if (ldc < (M > 1 ? M : 1)) return -12;
  if (lda > 4000000 || ldb > 4000000 || ldc > 4000000) return CQR_ERR_UNSUPPORTED;
  if (M == 0 || N == 0) return CQR_OK;
  hipStream_t st = (hipStream_t)stream;
  const double flops = 2.0 * (double)M * (double)N * (double)K;
  if (trans_a) {
    double* part = (work && work_bytes >= sizeof(double) * 64) ? (double*)work : nullptr;
    SVD_TRY(gemm_tn(ROLE_APROD, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, part,
                    part ? work_bytes / sizeof(double) : 0, nullptr, st, flops));
  } else {
    SVD_TRY(gemm_nn(ROLE_APROD, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, nullptr, st, flops));
  }
  return CQR_OK;
}

int cqr_svd_residuals(int64_t m, int64_t n, const double* A, int64_t lda, int64_t count, const double* U,
                      int64_t ldu, const double* sigma, const double* V, int64_t ldv, double* res, void* work,
                      size_t work_bytes, void* stream) {
  if (m < 1) return -1;
  if (n < 1) return -2;
  if (!A) return -3;
  if (lda < m) return -4;
  if (count < 1 || count > n) return -5;
  if (!U || ldu < m) return -6;
  if (!sigma) return -8;
  if (!V || ldv < n) return -9;
  if (!res) return -11;
  if (!work || work_bytes < (size_t)m * (size_t)count * sizeof(double)) return CQR_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  double* T = (double*)work;
  Op op{m, n, A, lda, nullptr};
  int rc = op_apply(op, false, count, V, ldv, T, m, nullptr, st);
  if (rc) return rc;
  const int slot = prof_begin(st);
  hipLaunchKernelGGL(residual_kernel, dim3((unsigned)count), dim3(256), 0, st, m, T, m, U, ldu, sigma, res);
  SVD_TRY(hipGetLastError());
  prof_end(slot, ROLE_SVD, st, 0.0, 0.0);
  return CQR_OK;
}

}  // extern "C"
