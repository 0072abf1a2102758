// Wave-local transforms of short vectors (columns of the two-pass transform): a wave
// runs the stages of V vectors of 2^K words at once, radix-2^R clusters per round, with
// no workgroup barrier (section 5.1's Algorithm 1, step 1 and its inverse).
#pragma once
#include "ntt_wave.hpp"

namespace nttgpu {

// Stages [T0, T0+R) of V vectors of 2^K words (K <= 10) at LDS stride vs, processed by
// one wave: work items (vector, cluster) are spread over the 64 lanes.
template <typename T, int LAZY, bool INV, int R, int K, int T0, int V>
__device__ __forceinline__ void vec_round(const Arith<T>& ar, T* s, int vs, int lane, gcptr<TwPair<T>> tw) {
  constexpr int C = 1 << R;
  constexpr int LS = K - T0 - R;
  constexpr int NCL = 1 << (K - R);
  constexpr int ITEMS = V * NCL;
#pragma unroll 1
  for (int qq = lane; qq < ITEMS; qq += 64) {
    const int v = qq / NCL, q = qq % NCL;
    const int b = q >> LS;
    const int base = (b << (K - T0)) + (q & ((1 << LS) - 1));
    T* sv = s + v * vs;
    const int lb = lidx(base);
    TwPair<T> w[C - 1];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      gcptr<TwPair<T>> p = tw + ((1u << (T0 + u)) + ((uint32_t)b << u));
#pragma unroll
      for (int vv = 0; vv < (1 << u); ++vv) w[(1 << u) - 1 + vv] = ldtw<T>(p + vv);
    }
    T x[1][C];
#pragma unroll
    for (int c = 0; c < C; ++c) x[0][c] = sv[lb + ClusterOff<R, LS>::off(c)];
    if constexpr (INV) cluster_inv<T, LAZY, R>(ar, x[0], w);
    else cluster_fwd<T, LAZY, R, 1>(ar, x, 0, w);
#pragma unroll
    for (int c = 0; c < C; ++c) sv[lb + ClusterOff<R, LS>::off(c)] = x[0][c];
  }
}

template <typename T, int LAZY, int K, int V, int T0>
__device__ __forceinline__ void vec_fwd_rounds(const Arith<T>& ar, T* s, int vs, int lane, gcptr<TwPair<T>> tw) {
  if constexpr (T0 < K) {
    constexpr int R = (T0 == 0 && (K & 3)) ? (K & 3) : 4;
    vec_round<T, LAZY, false, R, K, T0, V>(ar, s, vs, lane, tw);
    wave_sync();
    vec_fwd_rounds<T, LAZY, K, V, T0 + R>(ar, s, vs, lane, tw);
  }
}

template <typename T, int LAZY, int K, int V, int T0END>
__device__ __forceinline__ void vec_inv_rounds(const Arith<T>& ar, T* s, int vs, int lane, gcptr<TwPair<T>> twi) {
  if constexpr (T0END > 0) {
    constexpr int R = (T0END == (K & 3)) ? (K & 3) : 4;
    constexpr int T0 = T0END - R;
    vec_round<T, LAZY, true, R, K, T0, V>(ar, s, vs, lane, twi);
    wave_sync();
    vec_inv_rounds<T, LAZY, K, V, T0>(ar, s, vs, lane, twi);
  }
}

}  // namespace nttgpu
