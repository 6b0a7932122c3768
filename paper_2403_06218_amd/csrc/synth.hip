// Seeded synthetic inputs in device memory: SplitMix64 counter stream, as
// defined in include/cqr_synth.h.  No arithmetic of the factorisation here.
#include <hip/hip_runtime.h>
#include <cstdint>

#include "../../include/cqr_synth.h"

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256)
uniform_kernel(int64_t rows, int64_t cols, double* __restrict__ A, int64_t lda, uint64_t key, double lo,
               double scale) {
  const int64_t total = rows * cols;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t z = mix64(key + (uint64_t)(t + 1) * kGamma);
    const double u = (double)(z >> 11) * 0x1p-53;
    const int64_t i = t % rows, j = t / rows;
    A[i + j * lda] = __dadd_rn(lo, __dmul_rn(scale, u));
  }
}

}  // namespace

extern "C" int cqr_synth_uniform(int64_t rows, int64_t cols, double* A, int64_t lda, uint64_t seed, double lo,
                                 double hi, void* stream) {
  if (rows < 0) return -1;
  if (cols < 0) return -2;
  if (rows * cols == 0) return 0;
  if (!A) return -3;
  if (lda < rows) return -4;
  const uint64_t key = mix64(seed + kGamma);
  int64_t blocks = (rows * cols + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(uniform_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, rows, cols, A, lda,
                     key, lo, hi - lo);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : -1000 - (int)e;
}
