// Cholesky factorisation of a small SPD block (WP <= 32) held by one wave:
// lane i < WP owns row i.  Shared by the single-matrix factor kernel (its
// 16 x 16 diagonal blocks) and the batched form (its block Grams); and the
// wave broadcasts used by the solve kernels.
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

// Lane 16 r + N's value to every lane of its row of 16 (lanes 16 r .. 16 r +
// 15): the DPP row_newbcast control, one VALU move straight into a vector
// register (v_mov_b64_dpp for a double).  A readlane goes through a scalar
// register instead, with a wait before every use and one scalar pair reused
// by every broadcast, so that a run of them executes strictly one after the
// other.
template <int N>
__device__ __forceinline__ double dpp_row_bcast(double x) {
  static_assert(N >= 0 && N < 16, "row lane");
  const long v = __builtin_amdgcn_mov_dpp(__builtin_bit_cast(long, x), 0x150 + N, 0xF, 0xF, false);
  return __builtin_bit_cast(double, v);
}
template <int N>
__device__ __forceinline__ float dpp_row_bcast(float x) {
  static_assert(N >= 0 && N < 16, "row lane");
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x150 + N, 0xF, 0xF, false));
}

// row_bcast(x, j): dpp_row_bcast<j>(x) for a j that is a constant once the
// caller's loops are unrolled (the switch then folds away).
template <typename T>
__device__ __forceinline__ T row_bcast(T x, int j) {
  switch (j) {
    case 0: return dpp_row_bcast<0>(x);
    case 1: return dpp_row_bcast<1>(x);
    case 2: return dpp_row_bcast<2>(x);
    case 3: return dpp_row_bcast<3>(x);
    case 4: return dpp_row_bcast<4>(x);
    case 5: return dpp_row_bcast<5>(x);
    case 6: return dpp_row_bcast<6>(x);
    case 7: return dpp_row_bcast<7>(x);
    case 8: return dpp_row_bcast<8>(x);
    case 9: return dpp_row_bcast<9>(x);
    case 10: return dpp_row_bcast<10>(x);
    case 11: return dpp_row_bcast<11>(x);
    case 12: return dpp_row_bcast<12>(x);
    case 13: return dpp_row_bcast<13>(x);
    case 14: return dpp_row_bcast<14>(x);
    default: return dpp_row_bcast<15>(x);
  }
}

// Lane j's value for lanes 0 .. WP-1: the row broadcast when WP <= 16 (all
// consumers sit in the first row of 16 lanes), else readlane.
template <int WP, typename T>
__device__ __forceinline__ T small_bcast(T x, int j) {
  if constexpr (WP <= 16) return row_bcast(x, j);
  else return wave_bcast(x, j);
}

// W = L L^T computed as W = U D U^T (U unit lower, D diagonal), then
// L = U D^{1/2}.  On entry lane i holds a[j] = W(i, j) for j <= i (lanes >= WP
// and entries j > i may hold anything).  On return
// lane i holds a[j] = L(i, j) for j < i (entries j >= i are garbage),
// lii = L(i, i) and linv = 1 / L(i, i).  Returns false if a pivot is not
// > 0 (NaN included); the outputs are then meaningless.
//
// Step k needs one division (1 / d_k) on its critical chain; the broadcasts of
// column k depend only on values present at the start of the step, so they
// overlap the division, and the square roots are all taken at the end, one
// per lane.  The return value, lii and linv are those of lanes < WP; with
// WP <= 16 the other lanes take their broadcasts from their own row of 16
// lanes, so what they compute is meaningless.
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
    const T d = small_bcast<WP>(a[k], k);
    ok = ok && (d > T(0));
    const T r = T(1) / d;
    const T c = a[k];   // lane i > k: W^(k)(i, k) = u_ik d_k
    const T u = c * r;  // u_ik
#pragma unroll
    for (int j = k + 1; j < WP; ++j) a[j] -= u * small_bcast<WP>(c, j);
    dmine = (lane == k) ? d : dmine;
    a[k] = u;
  }
  const T s = sqrt(dmine);
  lii = s;
  linv = T(1) / s;
#pragma unroll
  for (int j = 0; j < WP; ++j) a[j] *= small_bcast<WP>(s, j);
  return ok;
}

// wave_chol that also forms the inverse: on return lane i < WP additionally
// holds y[j] = (U^{-1})(i, j) for j <= i (zero above), so that
// L^{-1}(i, j) = linv * y[j] with this lane's linv (L^{-1} = D^{-1/2} U^{-1}).
// Row k of U^{-1} is final once step k begins (it has received the updates
// of steps 0 .. k-1), and at step k every row i > k subtracts u_ik times it;
// these updates sit beside the step's division, off its dependent chain.
template <typename T, int WP>
__device__ __forceinline__ bool wave_chol_inv(T (&a)[WP], T (&y)[WP], T& lii, T& linv, int lane) {
  bool ok = true;
  T dmine = T(1);
#pragma unroll
  for (int j = 0; j < WP; ++j) y[j] = (j == lane) ? T(1) : T(0);
#pragma unroll
  for (int k = 0; k < WP; ++k) {
    const T d = small_bcast<WP>(a[k], k);
    ok = ok && (d > T(0));
    const T r = T(1) / d;
    const T c = a[k];
    const T u = c * r;
#pragma unroll
    for (int j = k + 1; j < WP; ++j) a[j] -= u * small_bcast<WP>(c, j);
    const T uk = (lane > k) ? u : T(0);
#pragma unroll
    for (int j = 0; j <= k; ++j) y[j] -= uk * small_bcast<WP>(y[j], k);
    dmine = (lane == k) ? d : dmine;
    a[k] = u;
  }
  const T s = sqrt(dmine);
  lii = s;
  linv = T(1) / s;
#pragma unroll
  for (int j = 0; j < WP; ++j) a[j] *= small_bcast<WP>(s, j);
  return ok;
}

}  // namespace cqr
