// Host driver of libcqr.so: the C ABI declared in include/cqr.h.
//
// cqr_factor runs CGS-QR (Algorithm 3): column block 1 by CholeskyQR2
// (Algorithm 4), every later block j by CGS-CQR2 (Algorithm 5) against the
// s = (j-1) b finished columns.  One block is the stream-ordered kernel chain
//
//   pass 1  H = P^T Q_j        (TN GEMM, split-K, written into R[0:s, J])
//           Q_j -= P H         (NN GEMM, in place)
//           W = Q_j^T Q_j      (TN GEMM, split-K)
//           W = L L^T, L^{-1}  (one-workgroup Cholesky + inverse)
//           T = Q_j L^{-T}     (NN GEMM into workspace T)
//   pass 2  Hb = P^T T; T -= P Hb; W = T^T T; W = Lb Lb^T; Q_j = T Lb^{-T}
//   combine R_jj = Lb^T L^T and H += Hb L^T   (Alg. 5 S11/S12, see below)
//
// Readings of the paper applied here: Algorithm 4 S7 / Algorithm 5 S11 are
// evaluated as R = Lb^T L^T and S12 as H = H + Hb L^T (the orders the algebra
// of S3/S6 and S5/S10 gives; the printed forms drop or swap the factor L^T);
// r need not be a multiple of b (ragged last block).
//
// Breakdown fallback (Section 3, CholeskyQR2 subsection): the Cholesky kernel
// flags a pivot that is not > 0 in a status word; every later kernel of the
// block's chain reads the word and exits.  After each block one launch of the
// CGS2 fallback kernel follows, gated on the same word: when it is set, that
// launch restores the block from its saved copy, redoes it one column at a
// time as Algorithm 5 with b = 1 (CGS2), records info and the block's flags in
// device memory and clears the word, so the next block proceeds.  No step
// reads anything back to the host: every call is stream-ordered and
// asynchronous, and can be captured in a hipGraph.
//
// Blocks wider than 128 columns factor their Gram matrix as a 2 x 2 block
// (two 128-wide Cholesky calls, the off-diagonal block and the Schur
// complement by MFMA products).
#include <mutex>
#include <vector>
#include <cstring>

#include "internal.h"
#include "../../include/cqr.h"

namespace cqr {

// ---------------------------------------------------------------- profiling
namespace {
struct ProfRec {
  int role;
  hipEvent_t e0, e1;
  double flops, bytes;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_pool;

hipEvent_t pool_get() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

const char* const kRoleNames[ROLE_COUNT] = {"proj", "update", "gram", "trsm", "small", "reduce",
                                            "chol", "copy", "gemv", "trsv_inv", "trsv",
                                            "batch", "batch_setup", "adjoint", "fallback",
                                            "aprod", "svd", "spmm"};

// Bound of one bounded wait (grid barriers, look-back), microseconds.
std::mutex g_wait_mu;
int64_t g_wait_us = 10 * 1000 * 1000;
int g_clock_khz = 0;
int64_t g_forced_blk = -1;  // block whose breakdown is forced (testing aid), -1 none
}  // namespace

int64_t forced_breakdown_block() {
  std::lock_guard<std::mutex> lk(g_wait_mu);
  return g_forced_blk;
}

const char* role_name(int role) { return (role >= 0 && role < ROLE_COUNT) ? kRoleNames[role] : nullptr; }

uint64_t wait_limit_ticks() {
  std::lock_guard<std::mutex> lk(g_wait_mu);
  if (g_clock_khz <= 0) {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
      g_clock_khz = khz;
    else
      g_clock_khz = 100000;  // the documented 100 MHz of gfx9 devices
  }
  return (uint64_t)g_wait_us * (uint64_t)g_clock_khz / 1000u;
}

int prof_begin(hipStream_t s) {
  if (!g_prof_on) return -1;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  ProfRec r{-1, pool_get(), pool_get(), 0.0, 0.0};
  if (r.e0 == nullptr || r.e1 == nullptr) return -1;
  if (hipEventRecord(r.e0, s) != hipSuccess) return -1;
  g_prof.push_back(r);
  return (int)g_prof.size() - 1;
}

void prof_end(int slot, int role, hipStream_t s, double flops, double bytes) {
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (slot >= (int)g_prof.size()) return;
  ProfRec& r = g_prof[slot];
  r.role = role;
  r.flops = flops;
  r.bytes = bytes;
  (void)hipEventRecord(r.e1, s);
}

// ---------------------------------------------------------------- workspace
namespace {

constexpr int64_t kMaxB = 256;
constexpr int64_t kCholB = 128;  // widest Gram one Cholesky kernel factors; wider ones take the 2 x 2 split
constexpr int64_t kMaxLd = 4000000;  // 32-bit in-tile offsets of the GEMM kernels

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Work {
  int* status;   // [0] breakdown code (0 none, 1 first pass, 2 second pass), [1] block index
  double* W;     // b x b Gram matrix
  double* LT1;   // L^T of the first pass, b x b
  double* XT1;   // (L^{-1})^T of the first pass
  double* LT2;
  double* XT2;
  double* T;     // q x b block after the first pass
  double* save;  // q x b copy of the block's input (fallback restore)
  double* Hb;    // (s) x b second-pass projection
  double* ctmp;  // 128 x (b - 128) scratch of the 2 x 2 Cholesky (b > 128)
  void* fb;      // fallback workspace (counters first)
  double* part;  // split-K partial sums
  size_t part_cap;
};

size_t part_capacity(int64_t q, int64_t r, int64_t b) {
  // Enough for the split-K partial sums of the projections (about 512
  // workgroups of 128 x 128 tiles), capped at 256 MiB.
  const size_t want = (size_t)512 * 128 * 128 + (size_t)4 * (size_t)r * (size_t)b;
  const size_t cap = (size_t)32 << 20;
  size_t v = want > cap ? cap : want;
  const size_t by_size = (size_t)(q > 0 ? q : 1) * (size_t)(r > b ? r : b) * 2;
  if (v > by_size) v = by_size;
  return v < 64 ? 64 : v;
}

size_t layout(int64_t q, int64_t r, int64_t b, char* base, Work* w) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  const size_t bb = (size_t)b * (size_t)b * sizeof(double);
  const size_t qb = (size_t)q * (size_t)b * sizeof(double);
  const size_t cap = part_capacity(q, r, b);
  Work tmp;
  Work* o = w ? w : &tmp;
  o->status = (int*)take(64);
  o->W = (double*)take(bb);
  o->LT1 = (double*)take(bb);
  o->XT1 = (double*)take(bb);
  o->LT2 = (double*)take(bb);
  o->XT2 = (double*)take(bb);
  o->T = (double*)take(qb);
  o->save = (double*)take(qb);
  o->Hb = (double*)take((size_t)(r > 0 ? r : 1) * (size_t)b * sizeof(double));
  o->ctmp = (double*)take((size_t)kCholB * (size_t)(b > kCholB ? b - kCholB : 1) * sizeof(double));
  o->fb = take(fallback_workspace_bytes(r > b ? r : b));
  o->part = (double*)take(cap * sizeof(double));
  o->part_cap = cap;
  return off;
}

#define CQR_TRY(expr)                                    \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return CQR_ERR_HIP_BASE - (int)e_; \
  } while (0)

// One segment of the basis a block is orthogonalised against: columns P
// (q x s, ldp) and where their projection coefficients go (s x w, ldh).
struct Seg {
  const double* P;
  int64_t ldp;
  int64_t s;
  double* H;
  int64_t ldh;
};

// Start of a call: clear the status word and the fallback counters, and
// set info and the k block flags to 0 (device outputs; NULL skips them).
__global__ void init_kernel(int* status, unsigned* fbctr, int32_t* info, int32_t* flags, int64_t k) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    status[0] = 0;
    status[1] = 0;
    fbctr[0] = 0u;
    fbctr[1] = 0u;
    fbctr[2] = 0u;
    if (info) info[0] = 0;
  }
  if (flags && i < k) flags[i] = 0;
}

int init_call(const Work& ws, int32_t* info, int32_t* flags, int64_t k, hipStream_t st) {
  const int64_t n = k > 1 ? k : 1;
  hipLaunchKernelGGL(init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ws.status, (unsigned*)ws.fb,
                     info, flags, k);
  CQR_TRY(hipGetLastError());
  return CQR_OK;
}

// W = L L^T and (L^{-1})^T for a w x w Gram matrix (w <= 256).
hipError_t chol_block(int w, double* W, double* LT, double* XT, const Work& ws, int code, int blk, hipStream_t st) {
  if (w <= kCholB) return chol_inv(w, W, w, LT, XT, ws.status, code, blk, st);
  return chol_inv_wide(w, W, w, LT, XT, ws.ctmp, ws.status, code, blk, st);
}

// Enqueue CGS-CQR2 (nseg >= 1) or CholeskyQR2 (nseg == 0) of the block Q
// (q x w, ldq), gated on the status word.  Writes the projections into the
// segments' H and the triangular factor into Rjj (w x w, ldr).
int orth_block(int64_t q, int64_t w, double* Q, int64_t ldq, const Seg* seg, int nseg, double* Rjj, int64_t ldr,
               const Work& ws, int blk, hipStream_t st, bool allow_tall = true) {
  const int* gate = ws.status;
  const double dq = (double)q, dw = (double)w;
  int64_t stot = 0;
  for (int i = 0; i < nseg; ++i) stot += seg[i].s;
  if (allow_tall && nseg <= 1 && tall_eligible(q, w, stot)) {
    // Narrow block of a tall matrix: the same steps as below, fused into
    // row-streaming sweeps (S1; S2+S3; S4; S5+S6; S7+S8; S9; S10).
    const int s = (int)stot, wi = (int)w;
    const double* P = nseg ? seg[0].P : nullptr;
    const int64_t ldp = nseg ? seg[0].ldp : 1;
    double* H = nseg ? seg[0].H : nullptr;
    const int64_t ldh = nseg ? seg[0].ldh : 1;
    // The block Q is read until the last step writes it: the first pass
    // leaves its update in T (T = Q - P H, then T L^{-T} in place).
    if (s > 0) CQR_TRY(tall_proj(q, s, wi, P, ldp, Q, ldq, H, ldh, ws.part, ws.part_cap, gate, st));
    CQR_TRY(tall_update_gram(q, s, wi, P, ldp, H, ldh, Q, ldq, ws.T, q, ws.W, ws.part, ws.part_cap, gate, st));
    CQR_TRY(chol_inv(wi, ws.W, w, ws.LT1, ws.XT1, ws.status, 1, blk, st));
    const double* X1 = s > 0 ? ws.T : Q;
    const int64_t ldx1 = s > 0 ? q : ldq;
    CQR_TRY(tall_trsm_proj(q, s, wi, X1, ldx1, ws.XT1, ws.T, q, P, ldp, ws.Hb, s > 0 ? s : 1, ws.part, ws.part_cap,
                           gate, st));
    CQR_TRY(tall_update_gram(q, s, wi, P, ldp, ws.Hb, s > 0 ? s : 1, ws.T, q, ws.T, q, ws.W, ws.part, ws.part_cap,
                             gate, st));
    CQR_TRY(chol_inv(wi, ws.W, w, ws.LT2, ws.XT2, ws.status, 2, blk, st));
    CQR_TRY(tall_trsm_proj(q, 0, wi, ws.T, q, ws.XT2, Q, ldq, nullptr, 1, nullptr, 1, ws.part, ws.part_cap, gate,
                           st));
    CQR_TRY(gemm_nn(ROLE_SMALL, w, w, w, 1.0, ws.LT2, w, ws.LT1, w, 0.0, Rjj, ldr, gate, st,
                    dw * dw * dw));  // S11 R = Lb^T L^T
    if (s > 0)
      CQR_TRY(gemm_nn(ROLE_SMALL, s, w, w, 1.0, ws.Hb, s, ws.LT1, w, 1.0, H, ldh, gate, st,
                      dw * (double)s));  // S12 H = H + Hb L^T
    return CQR_OK;
  }
  const double gram_flops = (nseg > 0 ? 2.0 : 1.0) * dw * dw * dq;  // Table 1: b^2 q (Alg. 4), 2 b^2 q (Alg. 5)
  // ---- pass 1
  for (int i = 0; i < nseg; ++i)  // S1  H = P^T Q
    CQR_TRY(gemm_tn(ROLE_PROJ, seg[i].s, w, q, 1.0, seg[i].P, seg[i].ldp, Q, ldq, 0.0, seg[i].H, seg[i].ldh, ws.part,
                    ws.part_cap, gate, st, 2.0 * dw * dq * (double)seg[i].s));
  for (int i = 0; i < nseg; ++i)  // S2  Q = Q - P H
    CQR_TRY(gemm_nn(ROLE_UPDATE, q, w, seg[i].s, -1.0, seg[i].P, seg[i].ldp, seg[i].H, seg[i].ldh, 1.0, Q, ldq, gate,
                    st, 2.0 * dw * dq * (double)seg[i].s));
  CQR_TRY(gemm_tn(ROLE_GRAM, w, w, q, 1.0, Q, ldq, Q, ldq, 0.0, ws.W, w, ws.part, ws.part_cap, gate, st,
                  gram_flops));  // S3  W = Q^T Q
  CQR_TRY(chol_block((int)w, ws.W, ws.LT1, ws.XT1, ws, 1, blk, st));  // S4  W = L L^T
  CQR_TRY(gemm_nn(ROLE_TRSM, q, w, w, 1.0, Q, ldq, ws.XT1, w, 0.0, ws.T, q, gate, st,
                  dw * dw * dq));  // S5  T = Q L^{-T}
  // ---- pass 2
  int64_t off = 0;
  for (int i = 0; i < nseg; ++i) {  // S6  Hb = P^T T
    CQR_TRY(gemm_tn(ROLE_PROJ, seg[i].s, w, q, 1.0, seg[i].P, seg[i].ldp, ws.T, q, 0.0, ws.Hb + off, stot, ws.part,
                    ws.part_cap, gate, st, 2.0 * dw * dq * (double)seg[i].s));
    off += seg[i].s;
  }
  off = 0;
  for (int i = 0; i < nseg; ++i) {  // S7  T = T - P Hb
    CQR_TRY(gemm_nn(ROLE_UPDATE, q, w, seg[i].s, -1.0, seg[i].P, seg[i].ldp, ws.Hb + off, stot, 1.0, ws.T, q, gate,
                    st, 2.0 * dw * dq * (double)seg[i].s));
    off += seg[i].s;
  }
  CQR_TRY(gemm_tn(ROLE_GRAM, w, w, q, 1.0, ws.T, q, ws.T, q, 0.0, ws.W, w, ws.part, ws.part_cap, gate, st,
                  gram_flops));  // S8  W = T^T T
  CQR_TRY(chol_block((int)w, ws.W, ws.LT2, ws.XT2, ws, 2, blk, st));  // S9  W = Lb Lb^T
  CQR_TRY(gemm_nn(ROLE_TRSM, q, w, w, 1.0, ws.T, q, ws.XT2, w, 0.0, Q, ldq, gate, st,
                  dw * dw * dq));  // S10 Q = T Lb^{-T}
  // ---- combine
  CQR_TRY(gemm_nn(ROLE_SMALL, w, w, w, 1.0, ws.LT2, w, ws.LT1, w, 0.0, Rjj, ldr, gate, st,
                  dw * dw * dw));  // S11 R = Lb^T L^T
  off = 0;
  for (int i = 0; i < nseg; ++i) {  // S12 H = H + Hb L^T
    CQR_TRY(gemm_nn(ROLE_SMALL, seg[i].s, w, w, 1.0, ws.Hb + off, stot, ws.LT1, w, 1.0, seg[i].H, seg[i].ldh, gate,
                    st, dw * (double)seg[i].s));
    off += seg[i].s;
  }
  return CQR_OK;
}

}  // namespace
}  // namespace cqr

using namespace cqr;

extern "C" {

const char* cqr_version(void) { return "cqr 0.1 (gfx950, FP64 MFMA)"; }

const char* cqr_status_string(int code) {
  if (code == CQR_OK) return "success";
  if (code == CQR_ERR_UNSUPPORTED) return "unsupported parameters (block width must be 1..256, leading dimensions at most 4e6)";
  if (code == CQR_ERR_WORKSPACE) return "workspace missing or too small";
  if (code == CQR_ERR_TOO_LARGE) return "size above the fixed scratch of the no-allocation entry point (n <= 65536)";
  if (code <= CQR_ERR_HIP_BASE) return hipGetErrorString((hipError_t)(CQR_ERR_HIP_BASE - code));
  if (code < 0 && code > -64) return "invalid argument (the negated return value is its 1-based position)";
  return "unknown status";
}

int cqr_workspace_size(int64_t q, int64_t r, int64_t b, size_t* bytes) {
  if (q < 0) return -1;
  if (r < 0 || r > q) return -2;
  if (b < 1) return -3;
  if (b > kMaxB) return CQR_ERR_UNSUPPORTED;
  if (!bytes) return -4;
  *bytes = layout(q, r, b, nullptr, nullptr);
  return CQR_OK;
}

int cqr_factor(int64_t q, int64_t r, int64_t b, double* Y, int64_t ldy, double* R, int64_t ldr, void* work,
               size_t work_bytes, int32_t* info, int32_t* block_flags, void* stream) {
  if (q < 0) return -1;
  if (r < 0 || r > q) return -2;
  if (b < 1) return -3;
  if (b > kMaxB) return CQR_ERR_UNSUPPORTED;
  if (!Y && q * r > 0) return -4;
  if (ldy < (q > 1 ? q : 1)) return -5;
  if (!R && r > 0) return -6;
  if (ldr < (r > 1 ? r : 1)) return -7;
  if (ldy > kMaxLd || ldr > kMaxLd) return CQR_ERR_UNSUPPORTED;
  const int64_t k = (r + b - 1) / b;
  const size_t need = layout(q, r, b, nullptr, nullptr);
  if (!work || work_bytes < need) return CQR_ERR_WORKSPACE;
  Work ws;
  layout(q, r, b, (char*)work, &ws);
  hipStream_t st = (hipStream_t)stream;
  int rc = init_call(ws, info, block_flags, k, st);
  if (rc) return rc;
  if (r == 0) return CQR_OK;
  CQR_TRY(zero_matrix(r, r, R, ldr, st));
  const int64_t forced_blk = forced_breakdown_block();
  for (int64_t blk = 0; blk < k; ++blk) {
    const int64_t s = blk * b;
    const int64_t w = (r - s < b) ? (r - s) : b;
    double* Qj = Y + s * ldy;
    // The row-streaming form leaves the block intact on a breakdown; the
    // GEMM form works in place and keeps a copy for the fallback.
    const bool forced = blk == forced_blk;
    const bool keep = forced || !tall_eligible(q, w, s);
    if (keep) CQR_TRY(copy_matrix(q, w, Qj, ldy, ws.save, q, ws.status, st));
    Seg seg{Y, ldy, s, R + s * ldr, ldr};
    rc = orth_block(q, w, Qj, ldy, &seg, s > 0 ? 1 : 0, R + s + s * ldr, ldr, ws, (int)blk, st);
    if (rc) return rc;
    if (forced) CQR_TRY(force_breakdown(ws.status, (int)blk, st));
    CQR_TRY(cgs2_fallback(q, s, w, Y, ldy, Qj, ldy, R + s * ldr, ldr, R + s + s * ldr, ldr, keep ? ws.save : nullptr,
                          q, ws.status, info, block_flags, (int)blk, ws.fb, st));
  }
  return CQR_OK;
}

int cqr_orth(int64_t q, int64_t b, double* Q, int64_t ldq, double* R, int64_t ldr, void* work, size_t work_bytes,
             int32_t* info, void* stream) {
  if (q < 0) return -1;
  if (b < 1 || b > q) return -2;
  if (b > kMaxB) return CQR_ERR_UNSUPPORTED;
  return cqr_factor(q, b, b, Q, ldq, R, ldr, work, work_bytes, info, nullptr, stream);
}

int cqr_orth_against(int64_t q, int64_t b, int64_t s, double* Q, int64_t ldq, const double* P, int64_t ldp,
                     double* H, int64_t ldh, double* R, int64_t ldr, void* work, size_t work_bytes, int32_t* info,
                     void* stream) {
  if (q < 0) return -1;
  if (b < 1) return -2;
  if (b > kMaxB) return CQR_ERR_UNSUPPORTED;
  if (s < 0 || s + b > q) return -3;
  if (!Q) return -4;
  if (ldq < (q > 1 ? q : 1)) return -5;
  if (!P && s > 0) return -6;
  if (ldp < (q > 1 ? q : 1)) return -7;
  if (!H && s > 0) return -8;
  if (ldh < (s > 1 ? s : 1)) return -9;
  if (!R) return -10;
  if (ldr < b) return -11;
  if (ldq > kMaxLd || ldp > kMaxLd || ldh > kMaxLd || ldr > kMaxLd) return CQR_ERR_UNSUPPORTED;
  const size_t need = layout(q, s + b, b, nullptr, nullptr);
  if (!work || work_bytes < need) return CQR_ERR_WORKSPACE;
  Work ws;
  layout(q, s + b, b, (char*)work, &ws);
  hipStream_t st = (hipStream_t)stream;
  int rc = init_call(ws, info, nullptr, 0, st);
  if (rc) return rc;
  CQR_TRY(zero_matrix(b, b, R, ldr, st));
  const bool keep = !tall_eligible(q, b, s);
  if (keep) CQR_TRY(copy_matrix(q, b, Q, ldq, ws.save, q, nullptr, st));
  Seg seg{P, ldp, s, H, ldh};
  rc = orth_block(q, b, Q, ldq, &seg, s > 0 ? 1 : 0, R, ldr, ws, 0, st);
  if (rc) return rc;
  CQR_TRY(cgs2_fallback(q, s, b, P, ldp, Q, ldq, H, ldh, R, ldr, keep ? ws.save : nullptr, q, ws.status, info, nullptr,
                        0, ws.fb, st));
  return CQR_OK;
}

int cqr_set_forced_breakdown(int64_t blk) {
  if (blk < -1) return -1;
  std::lock_guard<std::mutex> lk(g_wait_mu);
  g_forced_blk = blk;
  return CQR_OK;
}

int cqr_set_wait_limit_us(int64_t us) {
  if (us < 0) return -1;
  std::lock_guard<std::mutex> lk(g_wait_mu);
  g_wait_us = us;
  return CQR_OK;
}

int cqr_solve_workspace_size(int64_t n, size_t* bytes) {
  if (n < 0) return -1;
  if (!bytes) return -2;
  *bytes = align256((size_t)(n > 0 ? n : 1) * sizeof(double)) + trsv_workspace_bytes(n);
  return CQR_OK;
}

int cqr_solve(int64_t n, const double* Q, int64_t ldq, const double* R, int64_t ldr, double* x, void* work,
              size_t work_bytes, int32_t* status, void* stream) {
  if (n < 0) return -1;
  if (!Q && n > 0) return -2;
  if (ldq < (n > 1 ? n : 1)) return -3;
  if (!R && n > 0) return -4;
  if (ldr < (n > 1 ? n : 1)) return -5;
  if (!x && n > 0) return -6;
  if (n == 0) return CQR_OK;
  size_t need = 0;
  cqr_solve_workspace_size(n, &need);
  if (!work || work_bytes < need) return CQR_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  double* y = (double*)work;
  void* tw = (char*)work + align256((size_t)n * sizeof(double));
  CQR_TRY(gemv_t(n, Q, ldq, x, y, st));
  CQR_TRY(trsv_prepare(n, false, R, ldr, tw, st));
  CQR_TRY(trsv_solve(n, false, R, ldr, tw, y, 0, st));
  CQR_TRY(copy_matrix(n, 1, y, n, x, n, nullptr, st));
  if (status) CQR_TRY(trsv_status(n, tw, status, st));
  return CQR_OK;
}

int cqr_prof_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return CQR_OK;
}

int cqr_prof_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof) {
    (void)hipEventSynchronize(r.e1);
    g_pool.push_back(r.e0);
    g_pool.push_back(r.e1);
  }
  g_prof.clear();
  return CQR_OK;
}

int cqr_prof_query(const char* name, int64_t* launches, double* total_ms, double* flops, double* bytes) {
  if (!name) return -1;
  int role = -1;
  for (int i = 0; i < ROLE_COUNT; ++i)
    if (std::strcmp(name, role_name(i)) == 0) role = i;
  if (role < 0) return -1;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  int64_t n = 0;
  double ms = 0.0, fl = 0.0, by = 0.0;
  for (auto& r : g_prof) {
    if (r.role != role) continue;
    hipError_t e = hipEventSynchronize(r.e1);
    if (e != hipSuccess) return CQR_ERR_HIP_BASE - (int)e;
    float t = 0.0f;
    e = hipEventElapsedTime(&t, r.e0, r.e1);
    if (e != hipSuccess) return CQR_ERR_HIP_BASE - (int)e;
    ++n;
    ms += t;
    fl += r.flops;
    by += r.bytes;
  }
  if (launches) *launches = n;
  if (total_ms) *total_ms = ms;
  if (flops) *flops = fl;
  if (bytes) *bytes = by;
  return CQR_OK;
}

const char* cqr_prof_name(int i) { return role_name(i); }

}  // extern "C"
