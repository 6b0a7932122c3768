// Cholesky factorisation of a small SPD block (WP <= 32) held by one wave:
// lane i < WP owns row i.  Shared by the single-matrix factor kernel (its
// 16 x 16 diagonal blocks) and the batched form (its block Grams); and the
// wave broadcast used by the solve kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace cqr {

__device__ __forceinline__ double wave_bcast(double x, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float wave_bcast(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// W = L L^T computed as W = U D U^T (U unit lower, D diagonal), then
// L = U D^{1/2}.  On entry lane i holds a[j] = W(i, j) for j <= i (lanes >= WP
// and entries j > i may hold anything).  On return
// lane i holds a[j] = L(i, j) for j < i (entries j >= i are garbage),
// lii = L(i, i) and linv = 1 / L(i, i).  Returns false if a pivot is not
// > 0 (NaN included); the outputs are then meaningless.
//
// Step k needs one division (1 / d_k) on its critical chain; the broadcasts of
// column k (readlane) depend only on values present at the start of the step,
// so they overlap the division, and the square roots are all taken at the
// end, one per lane.
template <typename T, int WP>
__device__ __forceinline__ bool wave_chol(T (&a)[WP], T& lii, T& linv, int lane) {
  // Every update runs unpredicated on all lanes: it also rewrites entries
  // j > i (the upper triangle) of lane i, which no later step reads -- the
  // broadcasts of step k take lane k's diagonal and the lower entries of
  // lanes j > k only -- and which callers discard.
  bool ok = true;
  T dmine = T(1);
#pragma unroll
  for (int k = 0; k < WP; ++k) {
    const T d = wave_bcast(a[k], k);
    ok = ok && (d > T(0));
    const T r = T(1) / d;
    const T c = a[k];   // lane i > k: W^(k)(i, k) = u_ik d_k
    const T u = c * r;  // u_ik
#pragma unroll
    for (int j = k + 1; j < WP; ++j) a[j] -= u * wave_bcast(c, j);
    dmine = (lane == k) ? d : dmine;
    a[k] = u;
  }
  const T s = sqrt(dmine);
  lii = s;
  linv = T(1) / s;
#pragma unroll
  for (int j = 0; j < WP; ++j) a[j] *= wave_bcast(s, j);
  return ok;
}

}  // namespace cqr
