// Wave-local transform of LDS-resident vectors of 2^M words, 10 <= M <= 15.
//
// The M index bits are split into a workgroup part G (bits M-1 .. 10, radix
// 2^(M-10) clusters at stride 1024, one barrier-separated round) and three
// wave-local rounds on the 1024-word block that wave w owns (block B = w):
//   W1: bits 9..6  lane l holds elements l + 64 c            (c < 16)
//   W2: bits 5..2  lane (h4, l2) holds elements 64 h4 + 4 c + l2
//   W3: bits 1..0  lane l holds 4 radix-4 clusters 4 (l + 64 k) + c
// A wave exchanges data between its rounds through its own LDS block, so no
// workgroup barrier is needed there (LDS operations of one wave complete in issue
// order; wave_barrier only stops the compiler from moving them).  After W3 the
// forward transform leaves its result in registers, where the fused product applies
// the entry-wise product and starts the inverse.
//
// Stage t of the block (global stage d + t) uses twiddle TW[2^(d+t) + (h << t) + b],
// b = the top t bits of the element's index inside the 2^M vector (see ntt_lds.hpp).
// In G and W1 that index is the same for every lane of a wave, so those twiddles
// are held in scalar registers (read by scalar loads where the caller asks for it:
// their waits then do not cover the vector loads in flight).
#pragma once
#include "ntt_lds.hpp"

namespace nttgpu {

__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

// Radix-2^R butterflies on a register cluster x[0 .. 2^R): cluster stage u pairs
// (c, c + 2^(R-1-u)) with twiddle w[2^u - 1 + (c >> (R-u))].
template <typename T, int LAZY, int R, int NV, bool UNI = false>
__device__ __forceinline__ void cluster_fwd(const Arith<T>& ar, T (&x)[NV][1 << R], int off, const TwPair<T>* w) {
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int half = 1 << (R - 1 - u);
#pragma unroll
    for (int vv = 0; vv < (1 << u); ++vv) {
      const TwPair<T> ww = w[(1 << u) - 1 + vv];
#pragma unroll
      for (int c2 = 0; c2 < half; ++c2) {
        const int c = (vv << (R - u)) + c2;
#pragma unroll
        for (int v = 0; v < NV; ++v) ct_bfly<LAZY, UNI>(ar, x[v][c], x[v][c + half], ww);
      }
    }
  }
  (void)off;
}

template <typename T, int LAZY, int R, bool UNI = false>
__device__ __forceinline__ void cluster_inv(const Arith<T>& ar, T* x, const TwPair<T>* w) {
#pragma unroll
  for (int u = R - 1; u >= 0; --u) {
    const int half = 1 << (R - 1 - u);
#pragma unroll
    for (int vv = 0; vv < (1 << u); ++vv) {
      const TwPair<T> ww = w[(1 << u) - 1 + vv];
#pragma unroll
      for (int c2 = 0; c2 < half; ++c2) {
        const int c = (vv << (R - u)) + c2;
        gs_bfly<LAZY, UNI>(ar, x[c], x[c + half], ww);
      }
    }
  }
}

// Twiddles of a radix-2^R cluster whose top-t-bits index at its first stage t0 is
// b0 (so at cluster stage u it is (b0 << u) | vv): w[2^u - 1 + vv].
// UNIFORM: b0 is the same in every lane of the wave; the twiddles are then kept in
// scalar registers.
// SCALAR (with UNIFORM): scalar loads (ldtw_s) instead of vector loads and moves.
template <typename T, int R, bool UNIFORM = false, bool SCALAR = false>
__device__ __forceinline__ void cluster_twiddles(TwPair<T>* w, gcptr<TwPair<T>> tw, int d, int t0, uint32_t h,
                                                 uint32_t b0) {
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const uint32_t t = (uint32_t)(t0 + u);
    gcptr<TwPair<T>> p = tw + ((1u << (d + t)) + ((h << t) | (b0 << u)));
#pragma unroll
    for (int vv = 0; vv < (1 << u); ++vv) {
      if constexpr (UNIFORM && SCALAR) {
        w[(1 << u) - 1 + vv] = ldtw_s<T>(p + vv);
      } else {
        const TwPair<T> x = ldtw<T>(p + vv);
        w[(1 << u) - 1 + vv] = UNIFORM ? uni(x) : x;
      }
    }
  }
}

// ------------------------------------------------------------------ forward
// Round G: local stages 0 .. M-11 on clusters {q + 1024 c}.  Ends with a barrier.
template <typename T, int LAZY, int NT, int NV, int M>
__device__ __forceinline__ void fwd_G(const Arith<T>& ar, T* const (&sv)[NV], int d, uint32_t h,
                                      gcptr<TwPair<T>> tw) {
  constexpr int R = M - 10;
  if constexpr (R > 0) {
    constexpr int C = 1 << R;
    TwPair<T> w[C - 1];
    cluster_twiddles<T, R, true>(w, tw, d, 0, h, 0u);
#pragma unroll 1
    for (int q = opaque_tid(); q < 1024; q += NT) {
      const int lb = lidx(q);
      T x[NV][C];
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int c = 0; c < C; ++c) x[v][c] = sv[v][lb + c * 1056];  // lidx(q + 1024 c) = lidx(q) + 1056 c
      cluster_fwd<T, LAZY, R, NV, true>(ar, x, 0, w);
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int c = 0; c < C; ++c) sv[v][lb + c * 1056] = x[v][c];
    }
    __syncthreads();
  }
}

// Rounds W1..W3 of block B = wave id (or of block `blk` when it is given: a wave
// may own several blocks); the result stays in x[v][16] with
// x[v][4 k + c] = element 1024 B + 4 (lane + 64 k) + c.
// PF: each round's twiddles are requested one round ahead (W2's before W1's
// arithmetic, all of W3's before W2's), so that their L2 latency overlaps the round
// before; without it every round waits for its own twiddles.
template <typename T, int LAZY, int NV, int M, bool PF = false>
__device__ __forceinline__ void fwd_W(const Arith<T>& ar, T* const (&sv)[NV], int d, uint32_t h,
                                      gcptr<TwPair<T>> tw, T (&x)[NV][16], int blk = -1) {
  const int tid = opaque_tid();
  const int lane = tid & 63;
  const uint32_t B = blk >= 0 ? (uint32_t)blk : (uint32_t)__builtin_amdgcn_readfirstlane(tid >> 6);
  const int base = (int)B << 10;
  const int lbase = base + ((int)B << 5);  // lidx(base)
  TwPair<T> w[15];
  // W1: bits 9..6; twiddles uniform across the wave (scalar loads with PF).
  cluster_twiddles<T, 4, true, PF>(w, tw, d, M - 10, h, B);
  TwPair<T> w2[PF ? 15 : 1];
  if constexpr (PF) cluster_twiddles<T, 4>(w2, tw, d, M - 6, h, (B << 4) | (uint32_t)(lane >> 2));
  {
    const int lb = lbase + lane + (lane >> 5);
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int c = 0; c < 16; ++c) x[v][c] = sv[v][lb + c * 66];  // lidx(base + lane + 64 c)
    cluster_fwd<T, LAZY, 4, NV, true>(ar, x, 0, w);
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int c = 0; c < 16; ++c) sv[v][lb + c * 66] = x[v][c];
  }
  wave_sync();
  TwPair<T> w3p[PF ? 4 : 1][3];
  if constexpr (PF) {
#pragma unroll
    for (int k = 0; k < 4; ++k) cluster_twiddles<T, 2>(w3p[k], tw, d, M - 2, h, (B << 8) | (uint32_t)(lane + 64 * k));
  }
  // W2: bits 5..2.
  {
    const int h4 = lane >> 2, l2 = lane & 3;
    if constexpr (!PF) cluster_twiddles<T, 4>(w, tw, d, M - 6, h, (B << 4) | (uint32_t)h4);
    const int e0 = base + 64 * h4 + l2;
    const int lb = e0 + (e0 >> 5);  // 4 c + l2 < 32 iff c < 8, since l2 < 4
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int c = 0; c < 16; ++c) x[v][c] = sv[v][lb + 4 * c + (c >> 3)];  // lidx(e0 + 4 c)
    if constexpr (PF)
      cluster_fwd<T, LAZY, 4, NV>(ar, x, 0, w2);
    else
      cluster_fwd<T, LAZY, 4, NV>(ar, x, 0, w);
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int c = 0; c < 16; ++c) sv[v][lb + 4 * c + (c >> 3)] = x[v][c];
  }
  wave_sync();
  // W3: bits 1..0, four radix-4 clusters per lane.
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int g = lane + 64 * k;
    TwPair<T> w3[3];
    if constexpr (PF) {
#pragma unroll
      for (int c = 0; c < 3; ++c) w3[c] = w3p[k][c];
    } else {
      cluster_twiddles<T, 2>(w3, tw, d, M - 2, h, (B << 8) | (uint32_t)g);
    }
    const int e0 = base + 4 * g;
    const int lb = e0 + (e0 >> 5);
    T y[NV][4];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int c = 0; c < 4; ++c) y[v][c] = sv[v][lb + c];
    cluster_fwd<T, LAZY, 2, NV>(ar, y, 0, w3);
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int c = 0; c < 4; ++c) x[v][4 * k + c] = y[v][c];
  }
}

// ------------------------------------------------------------------ inverse
// Twiddles of W3' and W2' requested ahead of inv_W (with PF), for instance before the
// entry-wise product that precedes it.
template <typename T>
struct InvWTw {
  TwPair<T> w3[4][3];
  TwPair<T> w2[15];
};
template <typename T, int M>
__device__ __forceinline__ void inv_W_twiddles(InvWTw<T>& t, int d, uint32_t h, gcptr<TwPair<T>> twi, int blk = -1) {
  const int tid = opaque_tid();
  const int lane = tid & 63;
  const uint32_t B = blk >= 0 ? (uint32_t)blk : (uint32_t)__builtin_amdgcn_readfirstlane(tid >> 6);
#pragma unroll
  for (int k = 0; k < 4; ++k) cluster_twiddles<T, 2>(t.w3[k], twi, d, M - 2, h, (B << 8) | (uint32_t)(lane + 64 * k));
  cluster_twiddles<T, 4>(t.w2, twi, d, M - 6, h, (B << 4) | (uint32_t)(lane >> 2));
}

// Rounds W3'..W1' from registers (layout of fwd_W), result stored to LDS.
// PF: the twiddles of W3' and W2' come from `pre` (inv_W_twiddles of the same block), and
// those of W1' are requested before the arithmetic of W2' (as in fwd_W).
template <typename T, int LAZY, int M, bool PF = false>
__device__ __forceinline__ void inv_W(const Arith<T>& ar, T* sa, int d, uint32_t h, gcptr<TwPair<T>> twi,
                                      T (&x)[16], int blk = -1, const InvWTw<T>* pre = nullptr) {
  const int tid = opaque_tid();
  const int lane = tid & 63;
  const uint32_t B = blk >= 0 ? (uint32_t)blk : (uint32_t)__builtin_amdgcn_readfirstlane(tid >> 6);
  const int base = (int)B << 10;
  const int lbase = base + ((int)B << 5);
  (void)pre;
  // W3': bits 1..0.
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int g = lane + 64 * k;
    TwPair<T> w3[3];
    if constexpr (PF) {
#pragma unroll
      for (int c = 0; c < 3; ++c) w3[c] = pre->w3[k][c];
    } else {
      cluster_twiddles<T, 2>(w3, twi, d, M - 2, h, (B << 8) | (uint32_t)g);
    }
    cluster_inv<T, LAZY, 2>(ar, x + 4 * k, w3);
    const int e0 = base + 4 * g;
    const int lb = e0 + (e0 >> 5);
#pragma unroll
    for (int c = 0; c < 4; ++c) sa[lb + c] = x[4 * k + c];
  }
  wave_sync();
  TwPair<T> w[15];
  // (kept in vector registers: moved to scalar registers, they would be waited for
  // inside W2')
  if constexpr (PF) cluster_twiddles<T, 4>(w, twi, d, M - 10, h, B);
  // W2': bits 5..2.
  {
    const int h4 = lane >> 2, l2 = lane & 3;
    if constexpr (!PF) cluster_twiddles<T, 4>(w, twi, d, M - 6, h, (B << 4) | (uint32_t)h4);
    const int e0 = base + 64 * h4 + l2;
    const int lb = e0 + (e0 >> 5);
#pragma unroll
    for (int c = 0; c < 16; ++c) x[c] = sa[lb + 4 * c + (c >> 3)];
    if constexpr (PF)
      cluster_inv<T, LAZY, 4>(ar, x, pre->w2);
    else
      cluster_inv<T, LAZY, 4>(ar, x, w);
#pragma unroll
    for (int c = 0; c < 16; ++c) sa[lb + 4 * c + (c >> 3)] = x[c];
  }
  wave_sync();
  // W1': bits 9..6; twiddles uniform across the wave.
  if constexpr (!PF) cluster_twiddles<T, 4, true>(w, twi, d, M - 10, h, B);
  {
    const int lb = lbase + lane + (lane >> 5);
#pragma unroll
    for (int c = 0; c < 16; ++c) x[c] = sa[lb + c * 66];
    cluster_inv<T, LAZY, 4, !PF>(ar, x, w);
#pragma unroll
    for (int c = 0; c < 16; ++c) sa[lb + c * 66] = x[c];
  }
}

// Round G': local stages M-11 .. 0.  Starts with a barrier (the wave-local rounds
// of every wave must have stored their blocks), ends with one.
template <typename T, int LAZY, int NT, int M>
__device__ __forceinline__ void inv_G(const Arith<T>& ar, T* sa, int d, uint32_t h, gcptr<TwPair<T>> twi) {
  __syncthreads();
  constexpr int R = M - 10;
  if constexpr (R > 0) {
    constexpr int C = 1 << R;
    TwPair<T> w[C - 1];
    cluster_twiddles<T, R, true>(w, twi, d, 0, h, 0u);
#pragma unroll 1
    for (int q = opaque_tid(); q < 1024; q += NT) {
      const int lb = lidx(q);
      T x[C];
#pragma unroll
      for (int c = 0; c < C; ++c) x[c] = sa[lb + c * 1056];
      cluster_inv<T, LAZY, R, true>(ar, x, w);
#pragma unroll
      for (int c = 0; c < C; ++c) sa[lb + c * 1056] = x[c];
    }
    __syncthreads();
  }
}

}  // namespace nttgpu
