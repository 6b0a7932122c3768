/*
 * cqr_synth.h -- C ABI of libcqr_synth.so, the seeded synthetic-input
 * generator used by the tests and the benchmark.  It holds no arithmetic of
 * the factorisation; it exists so that inputs of any size can be made
 * directly in device memory and regenerated element by element on the CPU.
 *
 * Definition (shared with the CPU generator, implemented independently):
 * SplitMix64 (Steele, Lea, Flood, OOPSLA 2014).  For seed s the stream key is
 * key = mix(s + G) with G = 0x9E3779B97F4A7C15, and element t of the stream is
 * z = mix(key + (t + 1) G) (mod 2^64), where mix is the SplitMix64 output
 * function.  u = (z >> 11) * 2^-53 in [0, 1); the value is lo + (hi - lo) * u,
 * rounded as a product followed by a sum.  Element (i, j) of a rows x cols
 * matrix is stream element t = i + j * rows.
 */
#ifndef CQR_SYNTH_H
#define CQR_SYNTH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Fill A (device, rows x cols, column-major, lda >= rows) with i.i.d.
 * U[lo, hi) from `seed` as defined above, on `stream` (hipStream_t as void*).
 * Returns 0, -1..-4 for an invalid rows/cols/A/lda, or -1000 - hipError_t.
 */
int cqr_synth_uniform(int64_t rows, int64_t cols, double* A, int64_t lda, uint64_t seed, double lo, double hi,
                      void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CQR_SYNTH_H */
