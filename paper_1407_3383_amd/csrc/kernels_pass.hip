// Two-pass transforms (section 5.1, Algorithm 1) on the wave-local machinery.
//
// The vector (length 2^L) is read as 2^L1 rows of 2^L2 contiguous words.
//  * Column pass: the global stages 0 .. L1-1 are independent length-2^L1
//    transforms of the 2^L2 strided columns.  A workgroup loads a tile of C adjacent
//    columns into LDS with coalesced runs of C words, every wave transforms whole
//    columns with wave-local rounds (no workgroup barrier), and the tile is stored
//    back.  Columns longer than 2^10 use workgroup rounds.
//  * Row pass: row r is twisted by G^j, G = w_N^([r]_L1) (step 2; G^j is the product
//    of two table entries) and transformed (step 3) with the split of ntt_wave.hpp:
//    the top L2-10 stages on clusters loaded straight from HBM, the other 10 inside
//    each wave, the result written from registers in the TFT order of step 4.  The
//    inverse mirrors it; the fused product row pass runs both operands, the
//    entry-wise product and the inverse in one workgroup.
#include <string.h>

#include <type_traits>

#include "kernels.hpp"
#include "ntt_cols.hpp"
#include "ntt_wave.hpp"

namespace nttgpu {

__device__ __forceinline__ uint32_t brev_u(uint32_t i, int L) { return L == 0 ? 0u : (__brev(i) >> (32 - L)); }

template <typename T>
__device__ __forceinline__ Arith<T> arith_uni(const void* pcv) {
  gcptr<PassConst<T>> pc = gconst<PassConst<T>>(uni(pcv));
  Arith<T> ar;
  ar.p = uni(pc->p);
  ar.p2 = uni(pc->p2);
  ar.pinv = uni(pc->pinv);
  return ar;
}

// x * G^j with G^j = w_N^e read as lo[e mod 2^B] * hi[e >> B]; any word x -> [0, 2p).
// Residues held in doubles: each multiplicand is first reduced by one p (values below 2p,
// or below 4p for p < 2^48, keep x w below 2^50 p as Function 16 needs).
template <typename T>
__device__ __forceinline__ T twist2(const Arith<T>& ar, T x, uint32_t e, int B, gcptr<TwPair<T>> lo,
                                    gcptr<TwPair<T>> hi) {
  const TwPair<T> h = ldtw<T>(hi + (e >> B));
  const TwPair<T> l = ldtw<T>(lo + (e & ((1u << B) - 1)));
  if constexpr (std::is_same<T, double>::value) return ar.shoup(ar.red1(ar.shoup(ar.red1(x), h.w, h.ws)), l.w, l.ws);
  else return ar.shoup(ar.shoup(x, h.w, h.ws), l.w, l.ws);
}

// Shoup companion floor(w 2^32 / p) of a residue w < p: the double estimate is within
// 2^-20 of the exact quotient, so one correction step makes it exact.
__device__ __forceinline__ uint32_t companion32(uint32_t w, uint32_t p, double rcp32) {
  uint32_t q = (uint32_t)((double)w * rcp32);
  const int64_t r = (int64_t)((uint64_t)w << 32) - (int64_t)((uint64_t)q * p);
  if (r < 0) --q;
  else if (r >= (int64_t)p) ++q;
  return q;
}

// The per-thread twist factor w_N^e = lo[e mod 2^B] * hi[e >> B] as a Shoup pair.
__device__ __forceinline__ TwPair<uint32_t> thread_factor(const Arith<uint32_t>& ar, uint32_t e, int B,
                                                          gcptr<TwPair<uint32_t>> lo, gcptr<TwPair<uint32_t>> hi,
                                                          double rcp32) {
  const TwPair<uint32_t> h = ldtw<uint32_t>(hi + (e >> B));
  const TwPair<uint32_t> l = ldtw<uint32_t>(lo + (e & ((1u << B) - 1)));
  TwPair<uint32_t> f;
  f.w = ar.red1(ar.shoup(l.w, h.w, h.ws));
  f.ws = companion32(f.w, ar.p, rcp32);
  return f;
}

// The row's factors w_(2^S)^(c Rr mod 2^S), c < C, from the universal table
// (t[2^(S-1) + i] = w_(2^S)^([i]_(S-1)); the upper half of the circle is its negation,
// whose companion is the bitwise complement).  The same in every lane.
template <int C>
__device__ __forceinline__ void row_factors(TwPair<uint32_t> (&D)[C], gcptr<TwPair<uint32_t>> t, int S, uint32_t Rr,
                                            uint32_t p) {
  const uint32_t mask = (1u << S) - 1, half = 1u << (S - 1);
  // every scalar load first (their wait covers no vector load), then the negations
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const uint32_t e = ((uint32_t)c * Rr) & mask;
    D[c] = ldtw_s<uint32_t>(t + (half + brev_u(e & (half - 1), S - 1)));
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const uint32_t e = ((uint32_t)c * Rr) & mask;
    if (e >= half) {
      D[c].w = p - D[c].w;
      D[c].ws = ~D[c].ws;
    }
  }
}

// Column pass for columns of 2^K words, K <= 10: tiles of C = 2^(TILELOG-K) columns.
template <typename T, int LAZY, int NT, int TILELOG, int K, bool INV, typename IN_T>
__device__ void col_wave_body(const PassArgs& A, T* s, uint64_t tile, int L2, const Arith<T>& ar) {
  constexpr int LC0 = TILELOG - K;
  const int LC = LC0 < L2 ? LC0 : L2;
  const int C = 1 << LC;
  constexpr int VS = lds_words(1 << K) + 1;
  const uint64_t tiles_per_vec = 1ull << (L2 - LC);
  const uint64_t vec = tile / tiles_per_vec;
  const uint32_t col0 = (uint32_t)(tile % tiles_per_vec) << LC;
  const int cnt = C << K;
  const int tid = opaque_tid();
  const gcptr<PassConst<T>> pc = gconst<PassConst<T>>(uni(A.pc));
  if constexpr (!INV) {
    const gcptr<IN_T> in = gconst<IN_T>(uni(A.in)) + vec * A.in_stride;
    // scale 1: times sigma; 2: times 1 (reduction of words that may exceed p)
    // scale 3: times sigma_row (products whose columns are inverted by the inverse TFT)
    const TwPair<T> sig = uni(ldtw<T>(A.scale == 2 ? &pc->one : (A.scale == 3 ? &pc->sigma_row : &pc->sigma)));
    const bool scale = A.scale != 0;
    bool vec4 = false;
    if constexpr (sizeof(T) == 4 && sizeof(IN_T) <= 4)
      vec4 = C >= 4 && ((uintptr_t)(const IN_T*)in % (4 * sizeof(IN_T))) == 0 && (A.in_stride % 4) == 0;
    // A full-width tile with A.valid a positive multiple of 4 (every run of 4 words then
    // lies wholly below A.valid or wholly at or above it): every load of the thread is
    // requested before the first LDS store, one memory round trip per tile instead of
    // one per iteration of the loop below.  A run at or above A.valid loads the
    // vector's first words (present, since A.valid >= 4) and is replaced by zeros, so
    // that no branch separates the loads.
    constexpr int IT4 = ((1 << TILELOG) >> 2) / NT;
    bool staged = false;
    if constexpr (sizeof(T) == 4 && sizeof(IN_T) <= 4 && IT4 >= 1 && IT4 <= 8 && IT4 * 4 * NT == (1 << TILELOG)) {
      if (vec4 && LC == LC0 && A.valid != 0 && (A.valid & 3) == 0) {
        constexpr int lc4 = LC0 - 2;
        using V4 = typename std::conditional<sizeof(IN_T) == 4, uint4, uint2>::type;
        V4 q[IT4];
#pragma unroll
        for (int it = 0; it < IT4; ++it) {
          const uint32_t idx = (uint32_t)(tid + it * NT);
          const uint32_t r = idx >> lc4, cc = (idx & ((1u << lc4) - 1)) << 2;
          const uint64_t gi = ((uint64_t)r << L2) + col0 + cc;
          q[it] = *(const V4*)((const IN_T*)in + (gi < A.valid ? gi : 0));
        }
#pragma unroll
        for (int it = 0; it < IT4; ++it) {
          const uint32_t idx = (uint32_t)(tid + it * NT);
          const uint32_t r = idx >> lc4, cc = (idx & ((1u << lc4) - 1)) << 2;
          const bool ok = ((uint64_t)r << L2) + col0 + cc < A.valid;
          T x[4];
          if constexpr (sizeof(IN_T) == 4) {
            x[0] = q[it].x;
            x[1] = q[it].y;
            x[2] = q[it].z;
            x[3] = q[it].w;
          } else {
            x[0] = q[it].x & 0xFFFFu;
            x[1] = q[it].x >> 16;
            x[2] = q[it].y & 0xFFFFu;
            x[3] = q[it].y >> 16;
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            T y = ok ? x[i] : (T)0;
            if (scale) y = ar.red1(ar.shoup_u(y, sig.w, sig.ws));
            s[(cc + i) * VS + lidx(r)] = y;
          }
        }
        staged = true;
      }
    }
    if (staged) {
      // the tile is in LDS already
    } else if (vec4) {
      // runs of 4 columns as one 16-byte (8-byte for 16-bit limbs) access per thread
      const int lc4 = LC - 2;
#pragma unroll 2
      for (int idx = tid; idx < (cnt >> 2); idx += NT) {
        const uint32_t r = (uint32_t)idx >> lc4, cc = ((uint32_t)idx & ((C >> 2) - 1)) << 2;
        const uint64_t gi = ((uint64_t)r << L2) + col0 + cc;
        T x[4];
        if (gi + 3 < A.valid) {
          if constexpr (sizeof(IN_T) == 4) {
            const uint4 q = *(const uint4*)((const IN_T*)in + gi);
            x[0] = q.x;
            x[1] = q.y;
            x[2] = q.z;
            x[3] = q.w;
          } else {
            const uint2 q = *(const uint2*)((const IN_T*)in + gi);
            x[0] = q.x & 0xFFFFu;
            x[1] = q.x >> 16;
            x[2] = q.y & 0xFFFFu;
            x[3] = q.y >> 16;
          }
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) x[i] = gi + i < A.valid ? (T)in[gi + i] : (T)0;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          T y = x[i];
          if (scale) y = ar.red1(ar.shoup_u(y, sig.w, sig.ws));
          s[(cc + i) * VS + lidx(r)] = y;
        }
      }
    } else {
#pragma unroll 4
      for (int idx = tid; idx < cnt; idx += NT) {
        const uint32_t r = (uint32_t)idx >> LC, cc = (uint32_t)idx & (C - 1);
        const uint64_t gi = ((uint64_t)r << L2) + col0 + cc;
        T x = gi < A.valid ? (T)in[gi] : (T)0;
        if (scale) x = ar.red1(ar.shoup_u(x, sig.w, sig.ws));
        s[cc * VS + lidx(r)] = x;
      }
    }
  } else {
    const gcptr<T> in = gconst<T>(uni(A.in)) + vec * A.in_stride;
    bool vec4 = false;
    if constexpr (sizeof(T) == 4) vec4 = C >= 4 && ((uintptr_t)(const T*)in % 16) == 0 && (A.in_stride % 4) == 0;
    // a full-width tile: every load of the thread before the first LDS store
    constexpr int IT4 = ((1 << TILELOG) >> 2) / NT;
    bool staged = false;
    if constexpr (sizeof(T) == 4 && IT4 >= 1 && IT4 <= 8 && IT4 * 4 * NT == (1 << TILELOG)) {
      if (vec4 && LC == LC0) {
        constexpr int lc4 = LC0 - 2;
        uint4 q[IT4];
#pragma unroll
        for (int it = 0; it < IT4; ++it) {
          const uint32_t idx = (uint32_t)(tid + it * NT);
          const uint32_t r = idx >> lc4, cc = (idx & ((1u << lc4) - 1)) << 2;
          q[it] = *(const uint4*)((const T*)in + (((uint64_t)r << L2) + col0 + cc));
        }
#pragma unroll
        for (int it = 0; it < IT4; ++it) {
          const uint32_t idx = (uint32_t)(tid + it * NT);
          const uint32_t r = idx >> lc4, cc = (idx & ((1u << lc4) - 1)) << 2;
          s[cc * VS + lidx(r)] = q[it].x;
          s[(cc + 1) * VS + lidx(r)] = q[it].y;
          s[(cc + 2) * VS + lidx(r)] = q[it].z;
          s[(cc + 3) * VS + lidx(r)] = q[it].w;
        }
        staged = true;
      }
    }
    if (staged) {
      // the tile is in LDS already
    } else if (vec4) {
      const int lc4 = LC - 2;
#pragma unroll 2
      for (int idx = tid; idx < (cnt >> 2); idx += NT) {
        const uint32_t r = (uint32_t)idx >> lc4, cc = ((uint32_t)idx & ((C >> 2) - 1)) << 2;
        const uint4 q = *(const uint4*)((const T*)in + ((uint64_t)r << L2) + col0 + cc);
        s[cc * VS + lidx(r)] = q.x;
        s[(cc + 1) * VS + lidx(r)] = q.y;
        s[(cc + 2) * VS + lidx(r)] = q.z;
        s[(cc + 3) * VS + lidx(r)] = q.w;
      }
    } else {
#pragma unroll 4
      for (int idx = tid; idx < cnt; idx += NT) {
        const uint32_t r = (uint32_t)idx >> LC, cc = (uint32_t)idx & (C - 1);
        s[cc * VS + lidx(r)] = in[((uint64_t)r << L2) + col0 + cc];
      }
    }
  }
  __syncthreads();
  {
    constexpr int V = (1 << K) >= 1024 ? 1 : (1024 >> K);  // vectors per wave step: 64 lanes busy
    const int lane = tid & 63;
    const int wave = tid >> 6;
    constexpr int NW = NT / 64;
    for (int v0 = wave * V; v0 < C; v0 += NW * V) {
      if constexpr (INV) vec_inv_rounds<T, LAZY, K, V, K>(ar, s + v0 * VS, VS, lane, gconst<TwPair<T>>(uni(A.twi)));
      else vec_fwd_rounds<T, LAZY, K, V, 0>(ar, s + v0 * VS, VS, lane, gconst<TwPair<T>>(uni(A.tw)));
    }
  }
  __syncthreads();
  const gptr<T> out = gmut<T>(uni(A.out)) + vec * A.out_stride;
  // forward: only the first `rows` rows of the TFT order are stored (truncated transforms)
  const uint32_t nrow = (!INV && A.rows) ? A.rows : (1u << K);
  bool vec4o = false;
  if constexpr (sizeof(T) == 4) vec4o = C >= 4 && ((uintptr_t)(T*)out % 16) == 0 && (A.out_stride % 4) == 0;
  if (vec4o) {
    const int lc4 = LC - 2;
#pragma unroll 2
    for (int idx = tid; idx < (cnt >> 2); idx += NT) {
      const uint32_t r = (uint32_t)idx >> lc4, cc = ((uint32_t)idx & ((C >> 2) - 1)) << 2;
      const uint64_t gi = ((uint64_t)r << L2) + col0 + cc;
      if (r >= nrow) continue;
      T x[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        x[i] = s[(cc + i) * VS + lidx(r)];
        if constexpr (INV) x[i] = canon_from_inv<LAZY>(ar, x[i]);
      }
      if (!INV || gi + 3 < A.valid) {
        uint4 q;
        q.x = x[0];
        q.y = x[1];
        q.z = x[2];
        q.w = x[3];
        *(uint4*)((T*)out + gi) = q;
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (gi + i < A.valid) out[gi + i] = x[i];
      }
    }
  } else {
#pragma unroll 4
    for (int idx = tid; idx < cnt; idx += NT) {
      const uint32_t r = (uint32_t)idx >> LC, cc = (uint32_t)idx & (C - 1);
      const uint64_t gi = ((uint64_t)r << L2) + col0 + cc;
      if (r >= nrow) continue;
      const T x = s[cc * VS + lidx(r)];
      if constexpr (INV) {
        if (gi < A.valid) out[gi] = canon_from_inv<LAZY>(ar, x);
      } else {
        out[gi] = x;
      }
    }
  }
  __syncthreads();
}

// Two workgroups per CU (at most 64 VGPRs for 1024-thread 32-bit tiles) so that one
// tile's HBM phases overlap the other's arithmetic.
template <typename T, int NT, int TILELOG, int K, bool INV, typename IN_T>
__global__ __launch_bounds__(NT, (NT == 1024 ? 8 : 4)) void col_wave_kernel(PassJobs J, uint64_t ntiles, int L2) {
  const PassArgs& A = J.j[blockIdx.y];
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* s = (T*)smem_raw;
  const Arith<T> ar = arith_uni<T>(A.pc);
  const int mode = (int)uni(gconst<PassConst<T>>(uni(A.pc))->lazy);
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    with_mode<T>(mode, [&](auto m) {
      col_wave_body<T, decltype(m)::value, NT, TILELOG, K, INV, IN_T>(A, s, t, L2, ar);
    });
  }
}

// ------------------------------------------------------------------ rows
// KIND 0: forward (twist, transform); 1: inverse (transform, inverse twist);
// 2: fused product of two operands (twist both, forward, entry-wise product,
// inverse, inverse twist).  Rows of 2^M words, 10 <= M <= 14.
template <typename T, int LAZY, int NT, int M, int KIND>
__device__ void row_wave_body(const PassArgs& A, T* sa, T* sb, uint64_t rowid, const Arith<T>& ar) {
  constexpr int R = M - 10;
  constexpr int C = 1 << R;
  constexpr int CPT = 1024 / NT > 0 ? 1024 / NT : 1;
  const gcptr<PassConst<T>> pc = gconst<PassConst<T>>(uni(A.pc));
  const int L1 = (int)uni(pc->L1);
  const int B = (int)uni(pc->B);
  const int S = (int)uni(pc->L) - 10;
  const double rcp32 = pc->rcp32;
  // rows [0, A.rows) of every vector (truncated transforms), or all 2^L1
  const uint32_t nr = A.rows ? A.rows : (1u << L1);
  const uint64_t vec = rowid / nr;
  const uint32_t r = (uint32_t)(rowid % nr);
  const uint32_t Rr = brev_u(r, L1);
  const uint64_t off = (uint64_t)r << M;
  const gcptr<TwPair<T>> tw = gconst<TwPair<T>>(uni(A.tw));
  const gcptr<TwPair<T>> twi = gconst<TwPair<T>>(uni(A.twi));
  const int t0 = opaque_tid();
  const int lane = t0 & 63;
  const uint32_t Bw = (uint32_t)__builtin_amdgcn_readfirstlane(t0 >> 6);
  const bool wave_active = Bw < (1u << (M - 10));
  const int wbase = (int)Bw << 10;

  if constexpr (KIND == 0 || KIND == 2) {
    const gcptr<TwPair<T>> lo = gconst<TwPair<T>>(uni(A.tlo));
    const gcptr<TwPair<T>> hi = gconst<TwPair<T>>(uni(A.thi));
    const gcptr<T> ina = gconst<T>(uni(A.in)) + vec * A.in_stride + off;
    const gcptr<T> inb = gconst<T>(uni(A.in2)) + vec * A.in_stride + off;
    // the row's words are requested first (from memory), the twiddles after them
    // (scalar loads from L2, waited for separately)
    constexpr int NV = KIND == 2 ? 2 : 1;
    T vin[CPT][NV][C];
#pragma unroll
    for (int i = 0; i < CPT; ++i)
#pragma unroll
      for (int cc = 0; cc < C; ++cc) {
        const uint32_t j = (uint32_t)(t0 + i * NT + 1024 * cc);
        vin[i][0][cc] = ina[j];
        if constexpr (KIND == 2) vin[i][1][cc] = inb[j];
      }
    __builtin_amdgcn_sched_barrier(0);  // the machine scheduler keeps the loads above this point
    TwPair<T> wf[C > 1 ? C - 1 : 1];
    if constexpr (R > 0) cluster_twiddles<T, R, true, true>(wf, tw, 0, 0, 0u, 0u);
    TwPair<T> D[C];
    if constexpr (sizeof(T) == 4) row_factors<C>(D, tw, S, Rr, ar.p);
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int q = t0 + i * NT;
      T v[NV][C];
#pragma unroll
      for (int vv = 0; vv < NV; ++vv)
#pragma unroll
        for (int cc = 0; cc < C; ++cc) v[vv][cc] = vin[i][vv][cc];
      if constexpr (sizeof(T) == 4) {
        const TwPair<T> V = thread_factor(ar, (uint32_t)q * Rr, B, lo, hi, rcp32);
#pragma unroll
        for (int cc = 0; cc < C; ++cc) {
          v[0][cc] = ar.shoup_u(ar.shoup(v[0][cc], V.w, V.ws), D[cc].w, D[cc].ws);
          if constexpr (KIND == 2) v[1][cc] = ar.shoup_u(ar.shoup(v[1][cc], V.w, V.ws), D[cc].w, D[cc].ws);
        }
      } else {
#pragma unroll
        for (int cc = 0; cc < C; ++cc) {
          const uint32_t e = (uint32_t)(q + 1024 * cc) * Rr;
          v[0][cc] = twist2(ar, v[0][cc], e, B, lo, hi);
          if constexpr (KIND == 2) v[1][cc] = twist2(ar, v[1][cc], e, B, lo, hi);
        }
      }
      if constexpr (R > 0) cluster_fwd<T, LAZY, R, NV, true>(ar, v, 0, wf);
      const int lb0 = lidx(q);
#pragma unroll
      for (int cc = 0; cc < C; ++cc) {
        sa[lb0 + cc * 1056] = v[0][cc];
        if constexpr (KIND == 2) sb[lb0 + cc * 1056] = v[1][cc];
      }
    }
    __syncthreads();
    if constexpr (KIND == 0) {
      if (wave_active) {
        T x[1][16];
        T* const sv[1] = {sa};
        fwd_W<T, LAZY, 1, M>(ar, sv, 0, 0u, tw, x);
        const gptr<T> out = gmut<T>(uni(A.out)) + vec * A.out_stride + off;
        // positions >= valid of the vector are not stored (a TFT of valid values)
        const uint64_t lim = A.valid == 0 ? ~0ull : (A.valid > off ? A.valid - off : 0);
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const uint32_t j = (uint32_t)(wbase + 4 * (lane + 64 * k) + c);
            if (j < lim) out[j] = canon_from_fwd<LAZY>(ar, x[0][4 * k + c]);
          }
      }
      __syncthreads();
      return;
    } else {
      if (wave_active) {
        T x[2][16];
        T* const sv[2] = {sa, sb};
        fwd_W<T, LAZY, 2, M>(ar, sv, 0, 0u, tw, x);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          T xa = x[0][i], yb = x[1][i];
          if constexpr (LAZY == kLazy) {
            xa = ar.red1(ar.red2(xa));  // xa < p, yb < 4p: xa yb < 2^bits p
          } else {  // xa < p, yb < 2p: xa yb < 2p^2 < 2^bits p (Function 13's bound)
            xa = ar.red1(xa);
            if constexpr (LAZY == kBand) yb = ar.red1(yb);  // Function 16 needs xa yb < 2^50 p
          }
          T z = ar.mont(xa, yb);  // (0, 2p); the Montgomery scale was applied to b
          if constexpr (LAZY != kLazy) z = ar.red1(z);
          x[0][i] = z;
        }
        inv_W<T, LAZY, M>(ar, sa, 0, 0u, twi, x[0]);
      }
      __syncthreads();
    }
  } else {
    // KIND 1: canonical input in the TFT order
    if (wave_active) {
      const gcptr<T> in = gconst<T>(uni(A.in)) + vec * A.in_stride + off;
      T x[16];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int c = 0; c < 4; ++c) x[4 * k + c] = in[wbase + 4 * (lane + 64 * k) + c];
      inv_W<T, LAZY, M>(ar, sa, 0, 0u, twi, x);
    }
    __syncthreads();
  }
  // top inverse stages, inverse twist, store
  {
    const gcptr<TwPair<T>> ilo = gconst<TwPair<T>>(uni(A.tilo));
    const gcptr<TwPair<T>> ihi = gconst<TwPair<T>>(uni(A.tihi));
    const gptr<T> out = gmut<T>(uni(A.out)) + vec * A.out_stride + off;
    TwPair<T> wi[C > 1 ? C - 1 : 1];
    if constexpr (R > 0) cluster_twiddles<T, R, true, true>(wi, twi, 0, 0, 0u, 0u);
    TwPair<T> Di[C];
    if constexpr (sizeof(T) == 4) row_factors<C>(Di, twi, S, Rr, ar.p);
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int q = t0 + i * NT;
      const int lb0 = lidx(q);
      T v[C];
#pragma unroll
      for (int cc = 0; cc < C; ++cc) v[cc] = sa[lb0 + cc * 1056];
      if constexpr (R > 0) cluster_inv<T, LAZY, R, true>(ar, v, wi);
      if constexpr (sizeof(T) == 4) {
        const TwPair<T> V = thread_factor(ar, (uint32_t)q * Rr, B, ilo, ihi, rcp32);
#pragma unroll
        for (int cc = 0; cc < C; ++cc) {
          T y = ar.shoup_u(ar.shoup(v[cc], V.w, V.ws), Di[cc].w, Di[cc].ws);
          if constexpr (LAZY != kLazy) y = ar.red1(y);
          out[q + 1024 * cc] = y;
        }
      } else {
#pragma unroll
        for (int cc = 0; cc < C; ++cc) {
          const uint32_t j = (uint32_t)(q + 1024 * cc);
          T y = twist2(ar, v[cc], j * Rr, B, ilo, ihi);
          if constexpr (LAZY != kLazy) y = ar.red1(y);
          out[j] = y;
        }
      }
    }
    __syncthreads();
  }
}

template <typename T, int NT, int M, int KIND>
__global__ __launch_bounds__(NT, (KIND == 2 ? (sizeof(T) == 4 && NT < 1024 ? 4 : 1) : (sizeof(T) == 4 ? 8 : 4)))
void row_wave_kernel(PassJobs J, uint64_t nrows) {
  const PassArgs& A = J.j[blockIdx.y];
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sa = (T*)smem_raw;
  T* sb = sa + lds_words(1 << M);
  const Arith<T> ar = arith_uni<T>(A.pc);
  const int mode = (int)uni(gconst<PassConst<T>>(uni(A.pc))->lazy);
  for (uint64_t t = blockIdx.x; t < nrows; t += gridDim.x) {
    with_mode<T>(mode, [&](auto m) { row_wave_body<T, decltype(m)::value, NT, M, KIND>(A, sa, sb, t, ar); });
  }
}

// ------------------------------------------------------------------ launchers
static int grid_of(uint64_t items) { return (int)(items < 1048576ull ? items : 1048576ull); }

template <typename T, int NT, int TILELOG, int K, bool INV, typename IN_T>
static hipError_t launch_col_wave_k(const PassJobs& a, int L2, hipStream_t stream) {
  constexpr int LC0 = TILELOG - K;
  const int LC = LC0 < L2 ? LC0 : L2;
  const uint64_t ntiles = (uint64_t)a.j[0].batch << (L2 - LC);
  const size_t lds = (size_t)(1 << LC) * (lds_words(1 << K) + 1) * sizeof(T);
  auto k = col_wave_kernel<T, NT, TILELOG, K, INV, IN_T>;
  hipError_t e = allow_dynamic_lds((const void*)k, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(grid_of(ntiles), a.n), dim3(NT), lds, stream, a, ntiles, L2);
  return hipGetLastError();
}

// 32-bit columns of 2^10 words take tiles of 2^15 words (32 columns: 128-byte row
// segments, one workgroup per CU; 2^24 round trip 0.212 -> 0.203 ms); shorter columns
// keep 2^14-word tiles, whose launches have twice the workgroups (measured faster there).
template <typename T, int NT, int TILELOG, bool INV, typename IN_T>
static hipError_t launch_col_wave(const PassJobs& a, int L1, int L2, hipStream_t stream) {
  constexpr int TL10 = sizeof(T) == 4 ? TILELOG + 1 : TILELOG;
  switch (L1) {
#define NTT_COL(KK) \
  case KK: return launch_col_wave_k<T, NT, TILELOG, KK, INV, IN_T>(a, L2, stream);
    NTT_COL(1) NTT_COL(2) NTT_COL(3) NTT_COL(4) NTT_COL(5) NTT_COL(6) NTT_COL(7) NTT_COL(8) NTT_COL(9)
#undef NTT_COL
    case 10: return launch_col_wave_k<T, NT, TL10, 10, INV, IN_T>(a, L2, stream);
  }
  return hipErrorInvalidValue;
}

// Columns longer than 2^10 (transforms beyond 2^24) keep the workgroup rounds.
hipError_t launch_col_fwd_rounds(int word_bits, const PassArgs& a, int L1, int L2, hipStream_t stream);
hipError_t launch_col_inv_rounds(int word_bits, const PassArgs& a, int L1, int L2, hipStream_t stream);
hipError_t launch_row_rounds(int word_bits, int kind, const PassArgs& a, int L1, int L2, hipStream_t stream);

static PassJobs one_job(const PassArgs& a) {
  PassJobs j;
  memset(&j, 0, sizeof(j));
  j.j[0] = a;
  j.n = 1;
  return j;
}

hipError_t launch_col_fwd_jobs(int word_bits, const PassJobs& a, int L1, int L2, hipStream_t stream) {
  if (a.n < 1 || a.n > kMaxPassJobs) return hipErrorInvalidValue;
  if (word_bits == kWordF64) {
    if (L1 > 10) return hipErrorInvalidValue;  // the workgroup-round column kernels take integer words
    return launch_col_wave<double, 512, 13, false, double>(a, L1, L2, stream);
  }
  if (L1 > 10) {
    for (int i = 0; i < a.n; ++i) {
      hipError_t e = launch_col_fwd_rounds(word_bits, a.j[i], L1, L2, stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if (word_bits == 32) {
    if (a.j[0].in_u16) return launch_col_wave<uint32_t, 1024, 14, false, uint16_t>(a, L1, L2, stream);
    return launch_col_wave<uint32_t, 1024, 14, false, uint32_t>(a, L1, L2, stream);
  }
  return launch_col_wave<uint64_t, 512, 13, false, uint64_t>(a, L1, L2, stream);
}

hipError_t launch_col_inv_jobs(int word_bits, const PassJobs& a, int L1, int L2, hipStream_t stream) {
  if (a.n < 1 || a.n > kMaxPassJobs) return hipErrorInvalidValue;
  if (word_bits == kWordF64) {
    if (L1 > 10) return hipErrorInvalidValue;
    return launch_col_wave<double, 512, 13, true, double>(a, L1, L2, stream);
  }
  if (L1 > 10) {
    for (int i = 0; i < a.n; ++i) {
      hipError_t e = launch_col_inv_rounds(word_bits, a.j[i], L1, L2, stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if (word_bits == 32) return launch_col_wave<uint32_t, 1024, 14, true, uint32_t>(a, L1, L2, stream);
  return launch_col_wave<uint64_t, 512, 13, true, uint64_t>(a, L1, L2, stream);
}

hipError_t launch_col_fwd(int word_bits, const PassArgs& a, int L1, int L2, hipStream_t stream) {
  return launch_col_fwd_jobs(word_bits, one_job(a), L1, L2, stream);
}

hipError_t launch_col_inv(int word_bits, const PassArgs& a, int L1, int L2, hipStream_t stream) {
  return launch_col_inv_jobs(word_bits, one_job(a), L1, L2, stream);
}

template <typename T, int NT, int M, int KIND>
static hipError_t launch_row_wave(const PassJobs& a, int L1, hipStream_t stream) {
  const uint64_t nrows = (uint64_t)a.j[0].batch * (a.j[0].rows ? a.j[0].rows : (1u << L1));
  const size_t lds = (KIND == 2 ? 2 : 1) * (size_t)lds_words(1 << M) * sizeof(T);
  auto k = row_wave_kernel<T, NT, M, KIND>;
  hipError_t e = allow_dynamic_lds((const void*)k, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(grid_of(nrows), a.n), dim3(NT), lds, stream, a, nrows);
  return hipGetLastError();
}

// Rows of 2^12 .. 2^14 words (the split is a tuning choice): one wave per 1024-word block.
template <int KIND>
static hipError_t launch_row_kind(int word_bits, const PassJobs& a, int L1, int L2, hipStream_t stream) {
  if (a.n < 1 || a.n > kMaxPassJobs) return hipErrorInvalidValue;
  if (word_bits == kWordF64) {
    if (L2 == 13) return launch_row_wave<double, 512, 13, KIND>(a, L1, stream);
    if (L2 == 12) return launch_row_wave<double, 256, 12, KIND>(a, L1, stream);
    return hipErrorInvalidValue;
  }
  if (word_bits == 32) {
    if (L2 == 14) return launch_row_wave<uint32_t, 1024, 14, KIND>(a, L1, stream);
    if (L2 == 13) return launch_row_wave<uint32_t, 512, 13, KIND>(a, L1, stream);
    if (L2 == 12) return launch_row_wave<uint32_t, 256, 12, KIND>(a, L1, stream);
  } else {
    if (L2 == 13) return launch_row_wave<uint64_t, 512, 13, KIND>(a, L1, stream);
    if (L2 == 12) return launch_row_wave<uint64_t, 256, 12, KIND>(a, L1, stream);
  }
  for (int i = 0; i < a.n; ++i) {
    hipError_t e = launch_row_rounds(word_bits, KIND, a.j[i], L1, L2, stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_row_fwd(int word_bits, const PassArgs& a, int L1, int L2, hipStream_t stream) {
  return launch_row_kind<0>(word_bits, one_job(a), L1, L2, stream);
}
hipError_t launch_row_fwd_jobs(int word_bits, const PassJobs& a, int L1, int L2, hipStream_t stream) {
  return launch_row_kind<0>(word_bits, a, L1, L2, stream);
}
hipError_t launch_row_inv(int word_bits, const PassArgs& a, int L1, int L2, bool scale_ninv, hipStream_t stream) {
  (void)scale_ninv;  // the caller passes the twist table with n^-1 folded in when asked
  return launch_row_kind<1>(word_bits, one_job(a), L1, L2, stream);
}
hipError_t launch_row_polymul(int word_bits, const PassArgs& a, int L1, int L2, hipStream_t stream) {
  return launch_row_kind<2>(word_bits, one_job(a), L1, L2, stream);
}
hipError_t launch_row_polymul_jobs(int word_bits, const PassJobs& a, int L1, int L2, hipStream_t stream) {
  return launch_row_kind<2>(word_bits, a, L1, L2, stream);
}

}  // namespace nttgpu
