// The solve x = R^{-1} (Q^T rhs) for callers that cannot allocate device
// memory (code under stream capture, serving loops, harnesses that forbid
// hipMalloc): the same kernels as cqr_solve, with their workspace -- the
// staged Q^T rhs, the inverses of R's 64 x 64 diagonal blocks and the
// look-back counters -- in a fixed file-scope device array instead of a
// caller buffer.
//
// Each GPU the library runs on holds its own copy of the array at its own
// address, from the first call on that device until the process ends.  The
// address is taken once per device (hipGetSymbolAddress, with that device
// current) and kept; host code passes only that address to kernels, never
// the array's name.  Every call on one GPU shares the array: calls that
// overlap on one GPU (other streams, other threads) race and are not
// allowed.  The counters that must start at zero are cleared by the solve's
// own first kernel on every call.
#include <mutex>

#include "internal.h"
#include "../../include/cqr.h"

namespace cqr {
namespace {

// Workspace of cqr_solve at n = 65536: 64 KiB-row staging (512 KiB) plus
// 1024 inverted 64 x 64 blocks (32 MiB) plus the counters; rounded up.
constexpr size_t kScratchBytes = (size_t)33 << 20;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// The device address of this GPU's copy of `scratch` (looked up on the first
// call with this device current, then reused).
int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return CQR_ERR_HIP_BASE - (int)e;
  if (dev < 0 || dev >= kMaxDevices) return CQR_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return CQR_ERR_HIP_BASE - (int)e;
    if (p == nullptr) return CQR_ERR_HIP_BASE - (int)hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return CQR_OK;
}

}  // namespace
}  // namespace cqr

using namespace cqr;

extern "C" {

int cqr_solve_noalloc(int64_t n, const double* Q, int64_t ldq, const double* R, int64_t ldr, double* x,
                      int32_t* status, void* stream) {
  if (n < 0) return -1;
  if (!Q && n > 0) return -2;
  if (ldq < (n > 1 ? n : 1)) return -3;
  if (!R && n > 0) return -4;
  if (ldr < (n > 1 ? n : 1)) return -5;
  if (!x && n > 0) return -6;
  if (n > CQR_NOALLOC_MAX_N) return CQR_ERR_TOO_LARGE;
  if (n == 0) return CQR_OK;
  size_t need = 0;
  int rc = cqr_solve_workspace_size(n, &need);
  if (rc) return rc;
  if (need > kScratchBytes) return CQR_ERR_TOO_LARGE;
  void* work = nullptr;
  rc = scratch_address(&work);
  if (rc) return rc;
  return cqr_solve(n, Q, ldq, R, ldr, x, work, need, status, stream);
}

}  // extern "C"
