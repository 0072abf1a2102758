// Workgroup-level transforms of a vector resident in LDS (section 5.1).
//
// The forward transform is the in-place Cooley-Tukey form that takes natural order
// to bit-reversed (TFT) order; the inverse is the Gentleman-Sande form that takes
// bit-reversed order back to natural order.  Stage s of a length-2^L transform
// pairs indices that differ in bit L-1-s; the pair in block i (the top s bits of
// the index) uses the universal bit-reversed table
//     TW[2^s + i] = w_{2^(s+1)}^([i]_s),  w_{2^j} = g^((p-1)/2^j),
// which does not depend on L, so one table serves every length.
//
// A vector held in LDS may be a sub-problem: block h (of size 2^m) at depth d of a
// length-2^(d+m) transform.  Its stages are the global stages d .. d+m-1 and the
// table index of local block b at local stage t is 2^(d+t) + (h << t) + b.  This is
// Algorithm 1's split (n1 = 2^d vectors of length 2^m) with the twiddle step of its
// step 2 folded into the table.
//
// Threads work on radix-2^R clusters: 2^R elements at stride 2^(m-t0-R) that stay
// together for R consecutive stages t0 .. t0+R-1, so one LDS round trip serves R
// stages.  LDS indices are padded (one word per 32) against bank conflicts.
#pragma once
#include "arith.hpp"

namespace nttgpu {

__device__ __forceinline__ int lidx(int e) { return e + (e >> 5); }

// threadIdx.x behind an empty asm barrier: address arithmetic derived from it is
// recomputed where it is used instead of being hoisted out of the item and
// sub-problem loops (which would keep dozens of addresses live and spill).
__device__ __forceinline__ int opaque_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}
__host__ __device__ constexpr int lds_words(int n) { return n + (n >> 5); }

template <typename T, int LAZY, int R, int NT, bool TWO>
__device__ __forceinline__ void fwd_round(const Arith<T>& ar, T* sa, T* sb, int m, int t0, int d, uint32_t h,
                                          const TwPair<T>* __restrict__ tw) {
  constexpr int C = 1 << R;
  const int ls = m - t0 - R;  // log2 of the element stride inside a cluster
  const int nclust = 1 << (m - R);
  for (int q = threadIdx.x; q < nclust; q += NT) {
    const int b = q >> ls;
    const int base = (b << (m - t0)) + (q & ((1 << ls) - 1));
    T xa[C], xb[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      xa[c] = sa[lidx(base + (c << ls))];
      if constexpr (TWO) xb[c] = sb[lidx(base + (c << ls))];
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int s = d + t0 + u;
      const int half = 1 << (R - 1 - u);
      const uint32_t blk0 = (1u << s) + (h << (t0 + u)) + ((uint32_t)b << u);
#pragma unroll
      for (int v = 0; v < (1 << u); ++v) {
        const TwPair<T> w = tw[blk0 + v];
#pragma unroll
        for (int c2 = 0; c2 < half; ++c2) {
          const int c = (v << (R - u)) + c2;
          ct_bfly<LAZY>(ar, xa[c], xa[c + half], w);
          if constexpr (TWO) ct_bfly<LAZY>(ar, xb[c], xb[c + half], w);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      sa[lidx(base + (c << ls))] = xa[c];
      if constexpr (TWO) sb[lidx(base + (c << ls))] = xb[c];
    }
  }
}

template <typename T, int LAZY, int R, int NT>
__device__ __forceinline__ void inv_round(const Arith<T>& ar, T* sa, int m, int t0, int d, uint32_t h,
                                          const TwPair<T>* __restrict__ twi) {
  constexpr int C = 1 << R;
  const int ls = m - t0 - R;
  const int nclust = 1 << (m - R);
  for (int q = threadIdx.x; q < nclust; q += NT) {
    const int b = q >> ls;
    const int base = (b << (m - t0)) + (q & ((1 << ls) - 1));
    T x[C];
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = sa[lidx(base + (c << ls))];
#pragma unroll
    for (int u = R - 1; u >= 0; --u) {
      const int s = d + t0 + u;
      const int half = 1 << (R - 1 - u);
      const uint32_t blk0 = (1u << s) + (h << (t0 + u)) + ((uint32_t)b << u);
#pragma unroll
      for (int v = 0; v < (1 << u); ++v) {
        const TwPair<T> w = twi[blk0 + v];
#pragma unroll
        for (int c2 = 0; c2 < half; ++c2) {
          const int c = (v << (R - u)) + c2;
          gs_bfly<LAZY>(ar, x[c], x[c + half], w);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) sa[lidx(base + (c << ls))] = x[c];
  }
}

// All m stages of the forward transform of the LDS vector(s); the first round takes
// the m mod 4 leftover stages, the others radix 16.  Ends with a barrier.
template <typename T, int LAZY, int NT, bool TWO>
__device__ void fwd_lds(const Arith<T>& ar, T* sa, T* sb, int m, int d, uint32_t h, const TwPair<T>* __restrict__ tw) {
  int t0 = 0;
  switch (m & 3) {
    case 1: fwd_round<T, LAZY, 1, NT, TWO>(ar, sa, sb, m, 0, d, h, tw); t0 = 1; __syncthreads(); break;
    case 2: fwd_round<T, LAZY, 2, NT, TWO>(ar, sa, sb, m, 0, d, h, tw); t0 = 2; __syncthreads(); break;
    case 3: fwd_round<T, LAZY, 3, NT, TWO>(ar, sa, sb, m, 0, d, h, tw); t0 = 3; __syncthreads(); break;
    default: break;
  }
  for (; t0 < m; t0 += 4) {
    fwd_round<T, LAZY, 4, NT, TWO>(ar, sa, sb, m, t0, d, h, tw);
    __syncthreads();
  }
}

// Inverse of fwd_lds's stage sequence (rounds in reverse order).  Ends with a barrier.
template <typename T, int LAZY, int NT>
__device__ void inv_lds(const Arith<T>& ar, T* sa, int m, int d, uint32_t h, const TwPair<T>* __restrict__ twi) {
  const int r0 = m & 3;
  for (int t0 = m - 4; t0 >= r0; t0 -= 4) {
    inv_round<T, LAZY, 4, NT>(ar, sa, m, t0, d, h, twi);
    __syncthreads();
  }
  switch (r0) {
    case 1: inv_round<T, LAZY, 1, NT>(ar, sa, m, 0, d, h, twi); __syncthreads(); break;
    case 2: inv_round<T, LAZY, 2, NT>(ar, sa, m, 0, d, h, twi); __syncthreads(); break;
    case 3: inv_round<T, LAZY, 3, NT>(ar, sa, m, 0, d, h, twi); __syncthreads(); break;
    default: break;
  }
}

// ---------------------------------------------------------------------------
// The same stage sequence on `nvec` independent vectors of length 2^m stored at
// LDS offsets v * vs (plain transforms: depth 0, block 0).  Work items are
// (vector, cluster) pairs spread over the workgroup.
template <typename T, int LAZY, int R, int NT>
__device__ __forceinline__ void fwd_round_multi(const Arith<T>& ar, T* s, int vs, int nvec, int m, int t0,
                                                const TwPair<T>* __restrict__ tw) {
  constexpr int C = 1 << R;
  const int ls = m - t0 - R;
  const int lcl = m - R;  // log2 clusters per vector
  const int nitems = nvec << lcl;
  for (int q = threadIdx.x; q < nitems; q += NT) {
    T* sv = s + (q >> lcl) * vs;
    const int qc = q & ((1 << lcl) - 1);
    const int b = qc >> ls;
    const int base = (b << (m - t0)) + (qc & ((1 << ls) - 1));
    T x[C];
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = sv[lidx(base + (c << ls))];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int st = t0 + u;
      const int half = 1 << (R - 1 - u);
      const uint32_t blk0 = (1u << st) + ((uint32_t)b << u);
#pragma unroll
      for (int v = 0; v < (1 << u); ++v) {
        const TwPair<T> w = tw[blk0 + v];
#pragma unroll
        for (int c2 = 0; c2 < half; ++c2) {
          const int c = (v << (R - u)) + c2;
          ct_bfly<LAZY>(ar, x[c], x[c + half], w);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) sv[lidx(base + (c << ls))] = x[c];
  }
}

template <typename T, int LAZY, int R, int NT>
__device__ __forceinline__ void inv_round_multi(const Arith<T>& ar, T* s, int vs, int nvec, int m, int t0,
                                                const TwPair<T>* __restrict__ twi) {
  constexpr int C = 1 << R;
  const int ls = m - t0 - R;
  const int lcl = m - R;
  const int nitems = nvec << lcl;
  for (int q = threadIdx.x; q < nitems; q += NT) {
    T* sv = s + (q >> lcl) * vs;
    const int qc = q & ((1 << lcl) - 1);
    const int b = qc >> ls;
    const int base = (b << (m - t0)) + (qc & ((1 << ls) - 1));
    T x[C];
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = sv[lidx(base + (c << ls))];
#pragma unroll
    for (int u = R - 1; u >= 0; --u) {
      const int st = t0 + u;
      const int half = 1 << (R - 1 - u);
      const uint32_t blk0 = (1u << st) + ((uint32_t)b << u);
#pragma unroll
      for (int v = 0; v < (1 << u); ++v) {
        const TwPair<T> w = twi[blk0 + v];
#pragma unroll
        for (int c2 = 0; c2 < half; ++c2) {
          const int c = (v << (R - u)) + c2;
          gs_bfly<LAZY>(ar, x[c], x[c + half], w);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) sv[lidx(base + (c << ls))] = x[c];
  }
}

template <typename T, int LAZY, int NT>
__device__ void fwd_lds_multi(const Arith<T>& ar, T* s, int vs, int nvec, int m, const TwPair<T>* __restrict__ tw) {
  int t0 = 0;
  switch (m & 3) {
    case 1: fwd_round_multi<T, LAZY, 1, NT>(ar, s, vs, nvec, m, 0, tw); t0 = 1; __syncthreads(); break;
    case 2: fwd_round_multi<T, LAZY, 2, NT>(ar, s, vs, nvec, m, 0, tw); t0 = 2; __syncthreads(); break;
    case 3: fwd_round_multi<T, LAZY, 3, NT>(ar, s, vs, nvec, m, 0, tw); t0 = 3; __syncthreads(); break;
    default: break;
  }
  for (; t0 < m; t0 += 4) {
    fwd_round_multi<T, LAZY, 4, NT>(ar, s, vs, nvec, m, t0, tw);
    __syncthreads();
  }
}

template <typename T, int LAZY, int NT>
__device__ void inv_lds_multi(const Arith<T>& ar, T* s, int vs, int nvec, int m, const TwPair<T>* __restrict__ twi) {
  const int r0 = m & 3;
  for (int t0 = m - 4; t0 >= r0; t0 -= 4) {
    inv_round_multi<T, LAZY, 4, NT>(ar, s, vs, nvec, m, t0, twi);
    __syncthreads();
  }
  switch (r0) {
    case 1: inv_round_multi<T, LAZY, 1, NT>(ar, s, vs, nvec, m, 0, twi); __syncthreads(); break;
    case 2: inv_round_multi<T, LAZY, 2, NT>(ar, s, vs, nvec, m, 0, twi); __syncthreads(); break;
    case 3: inv_round_multi<T, LAZY, 3, NT>(ar, s, vs, nvec, m, 0, twi); __syncthreads(); break;
    default: break;
  }
}

// ---------------------------------------------------------------------------
// Compile-time-size variants.  With the vector length 2^M and the round's first
// stage t0 known at compile time, the padded LDS offset of every cluster element
// is lidx(base) + off(c), off(c) = (c << ls) + ((c << ls) >> 5): one address per
// cluster, the rest are instruction immediates.  (Every cluster spans an aligned
// block of 2^(M-t0) elements whose start is a multiple of 32 or which lies inside
// one 32-word line, which is what makes the offset independent of the cluster.)
template <int R, int LS>
struct ClusterOff {
  static constexpr int off(int c) { return (c << LS) + ((c << LS) >> 5); }
};

template <typename T, int LAZY, int R, int NT, int NV, int M, int T0>
__device__ __forceinline__ void fwd_round_ct(const Arith<T>& ar, T* const (&sv)[NV], int d, uint32_t h,
                                             gcptr<TwPair<T>> tw) {
  constexpr int C = 1 << R;
  constexpr int LS = M - T0 - R;
  constexpr int NCL = 1 << (M - R);
#pragma unroll 1
  for (int q = opaque_tid(); q < NCL; q += NT) {
    const int b = q >> LS;
    const int base = (b << (M - T0)) + (q & ((1 << LS) - 1));
    const int lb = lidx(base);
    // all 2^R - 1 twiddles of the cluster, requested before the LDS reads
    TwPair<T> w[C - 1];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const uint32_t s = (uint32_t)(d + T0 + u);
      gcptr<TwPair<T>> twu = tw + ((1u << s) + ((h << (T0 + u)) | ((uint32_t)b << u)));
#pragma unroll
      for (int vv = 0; vv < (1 << u); ++vv) w[(1 << u) - 1 + vv] = ldtw<T>(twu + vv);
    }
    T x[NV][C];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int c = 0; c < C; ++c) x[v][c] = sv[v][lb + ClusterOff<R, LS>::off(c)];
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
          for (int v = 0; v < NV; ++v) ct_bfly<LAZY>(ar, x[v][c], x[v][c + half], ww);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int c = 0; c < C; ++c) sv[v][lb + ClusterOff<R, LS>::off(c)] = x[v][c];
  }
}

template <typename T, int LAZY, int R, int NT, int M, int T0>
__device__ __forceinline__ void inv_round_ct(const Arith<T>& ar, T* sa, int d, uint32_t h, gcptr<TwPair<T>> twi) {
  constexpr int C = 1 << R;
  constexpr int LS = M - T0 - R;
  constexpr int NCL = 1 << (M - R);
#pragma unroll 1
  for (int q = opaque_tid(); q < NCL; q += NT) {
    const int b = q >> LS;
    const int base = (b << (M - T0)) + (q & ((1 << LS) - 1));
    const int lb = lidx(base);
    TwPair<T> w[C - 1];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const uint32_t s = (uint32_t)(d + T0 + u);
      gcptr<TwPair<T>> twu = twi + ((1u << s) + ((h << (T0 + u)) | ((uint32_t)b << u)));
#pragma unroll
      for (int vv = 0; vv < (1 << u); ++vv) w[(1 << u) - 1 + vv] = ldtw<T>(twu + vv);
    }
    T x[C];
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = sa[lb + ClusterOff<R, LS>::off(c)];
#pragma unroll
    for (int u = R - 1; u >= 0; --u) {
      const int half = 1 << (R - 1 - u);
#pragma unroll
      for (int vv = 0; vv < (1 << u); ++vv) {
        const TwPair<T> ww = w[(1 << u) - 1 + vv];
#pragma unroll
        for (int c2 = 0; c2 < half; ++c2) {
          const int c = (vv << (R - u)) + c2;
          gs_bfly<LAZY>(ar, x[c], x[c + half], ww);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) sa[lb + ClusterOff<R, LS>::off(c)] = x[c];
  }
}

// Rounds of the forward transform: first the M mod 4 leftover stages, then radix 16.
template <typename T, int LAZY, int NT, int NV, int M, int T0>
__device__ __forceinline__ void fwd_rounds_ct(const Arith<T>& ar, T* const (&sv)[NV], int d, uint32_t h,
                                              gcptr<TwPair<T>> tw) {
  if constexpr (T0 < M) {
    constexpr int R = (T0 == 0 && (M & 3)) ? (M & 3) : 4;
    fwd_round_ct<T, LAZY, R, NT, NV, M, T0>(ar, sv, d, h, tw);
    __syncthreads();
    fwd_rounds_ct<T, LAZY, NT, NV, M, T0 + R>(ar, sv, d, h, tw);
  }
}

template <typename T, int LAZY, int NT, int M, int T0END>
__device__ __forceinline__ void inv_rounds_ct(const Arith<T>& ar, T* sa, int d, uint32_t h, gcptr<TwPair<T>> twi) {
  // processes the round that ends at T0END (exclusive), then the earlier ones
  if constexpr (T0END > 0) {
    constexpr int R = (T0END == (M & 3)) ? (M & 3) : 4;
    constexpr int T0 = T0END - R;
    inv_round_ct<T, LAZY, R, NT, M, T0>(ar, sa, d, h, twi);
    __syncthreads();
    inv_rounds_ct<T, LAZY, NT, M, T0>(ar, sa, d, h, twi);
  }
}

template <typename T, int LAZY, int NT, int NV, int M>
__device__ __forceinline__ void fwd_lds_ct(const Arith<T>& ar, T* const (&sv)[NV], int d, uint32_t h,
                                           gcptr<TwPair<T>> tw) {
  fwd_rounds_ct<T, LAZY, NT, NV, M, 0>(ar, sv, d, h, tw);
}

template <typename T, int LAZY, int NT, int M>
__device__ __forceinline__ void inv_lds_ct(const Arith<T>& ar, T* sa, int d, uint32_t h, gcptr<TwPair<T>> twi) {
  inv_rounds_ct<T, LAZY, NT, M, M>(ar, sa, d, h, twi);
}

}  // namespace nttgpu
