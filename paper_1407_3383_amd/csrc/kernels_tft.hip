// Inverse truncated Fourier transform (section 5.1).
//
// The forward TFT keeps the first l values of the transform in the TFT order (position i
// holds A(w^[i]_k)).  Its inverse recovers the l coefficients of a polynomial of degree
// < l from those l values.  The transform of a block of 2^m words (block h at depth d of
// the in-place Cooley-Tukey form, whose first stage pairs y_j and y_(j + 2^(m-1)) with the
// twiddle w = TW[2^d + h]) splits into the transforms of u = y_j + w y_(j+half) (block 2h
// at depth d+1, the first half of the outputs) and v = y_j - w y_(j+half) (block 2h+1, the
// second half).  Given the first l outputs and the inputs at positions >= l:
//   l <= half: the u_j with j >= l are known (both inputs known), so the first half is
//     the same problem one level down with l values; then y_j = u_j - w y_(j+half).
//   l >  half: all of u is known: one full normalized inverse of the first half; for
//     j >= l - half the input y_(j+half) is known, which gives y_j and v_j; the second
//     half is then the same problem one level down with l - half values; finally
//     y_j = (u_j + v_j) / 2 and y_(j+half) = (u_j - v_j) w^-1 / 2.
// The recursion follows a single path, fixed by the bits of l - 1: at level i the block
// is block (l-1) >> (m0 - i) at depth i, at offset ((l-1) >> (m0 - i)) << (m0 - i), and
// it stops at the first level whose block is entirely known (a full normalized inverse).
// Every vector of a launch has the same l, so all threads follow the same path, one
// barrier per step.  All values are canonical residues.
//
// Kernels: the column pass of the two-pass inverse (tiles of C adjacent columns, like the
// transform's column pass), the one row that a general l leaves partially known, and one
// LDS-resident vector per batch item.
#include <type_traits>

#include "kernels.hpp"
#include "ntt_cols.hpp"

namespace nttgpu {

namespace {

template <typename T>
struct TftOps {
  Arith<T> ar;
  T half;  // (p + 1) / 2
  __device__ __forceinline__ T add(T x, T y) const { return ar.red1(x + y); }
  __device__ __forceinline__ T sub(T x, T y) const { return ar.red1(x - y + ar.p); }
  __device__ __forceinline__ T mul(T x, const TwPair<T>& w) const { return ar.red1(ar.shoup(x, w.w, w.ws)); }
  // x / 2 mod p for a canonical x (p odd): x / 2 when x is even, (x + p) / 2 otherwise
  __device__ __forceinline__ T halve(T x) const {
    if constexpr (std::is_same<T, double>::value) {
      const double q = x * 0.5;
      return q == floor(q) ? q : __dadd_rn(floor(q), half);
    } else {
      return (x >> 1) + ((x & 1) ? half : (T)0);
    }
  }
};

template <typename T>
__device__ __forceinline__ TftOps<T> tft_ops(const void* pcv) {
  const gcptr<PassConst<T>> pc = gconst<PassConst<T>>(uni(pcv));
  TftOps<T> o;
  o.ar.p = uni(pc->p);
  o.ar.p2 = uni(pc->p2);
  o.ar.pinv = uni(pc->pinv);
  o.half = uni(pc->half);
  return o;
}

// Threads that work on a set of vectors together: a whole workgroup (barriers between
// steps) or one wave (its own vectors; LDS operations of a wave complete in order, so
// only the compiler needs a fence).
template <int NTH>
struct Group {
  int tid;
  __device__ __forceinline__ void sync() const {
    if constexpr (NTH == 64) __builtin_amdgcn_wave_barrier();
    else __syncthreads();
  }
};

// Normalized inverse of the block (d, h) transform of 2^m words at offset `off` of 2^lnv
// vectors (vector v at s + v vs, element j at lidx(j)): Gentleman-Sande stages, then the
// factor 2^-m.  Consecutive threads take consecutive vectors at the same position, so a
// wave reads one twiddle.  tw / twi: the universal tables (LDS or global).
template <typename T, int NTH>
__device__ void inv_block_norm(const TftOps<T>& o, const Group<NTH>& g, T* s, int vs, int lnv, int off, int d,
                               uint32_t h, int m, const TwPair<T>* twi, gcptr<PassConst<T>> pc) {
  if (m <= 0) return;
  const int nv = 1 << lnv;
  const int np = 1 << (m - 1);
  for (int t = m - 1; t >= 0; --t) {
    const int lh = m - t - 1;
    const int half = 1 << lh;
    for (int idx = g.tid; idx < (np << lnv); idx += NTH) {
      const int v = idx & (nv - 1), q = idx >> lnv;
      const int b = q >> lh, j = q & (half - 1);
      const int e0 = off + (b << (lh + 1)) + j;
      const TwPair<T> wi = twi[(1u << (d + t)) + (h << t) + (uint32_t)b];
      T* sv = s + v * vs;
      const T X = sv[lidx(e0)], Y = sv[lidx(e0 + half)];
      sv[lidx(e0)] = o.add(X, Y);
      sv[lidx(e0 + half)] = o.mul(o.sub(X, Y), wi);
    }
    g.sync();
  }
  const TwPair<T> sc = ldtw<T>(&pc->inv2pow[m]);
  for (int idx = g.tid; idx < (1 << (m + lnv)); idx += NTH) {
    const int v = idx & (nv - 1), j = idx >> lnv;
    T* sv = s + v * vs;
    sv[lidx(off + j)] = o.mul(sv[lidx(off + j)], sc);
  }
  g.sync();
}

// Inverse TFT of 2^lnv vectors of 2^K words in LDS: on entry positions [0, lam) hold the
// first lam TFT values and positions [lam, 2^K) the known inputs; on exit positions
// [0, lam) hold the inputs (positions >= lam are overwritten).  1 <= lam <= 2^K.  The
// vectors are block h0 at depth d0 of a longer transform, and their elements start at
// element eoff of each LDS vector.
template <typename T, int NTH>
__device__ void itft_vectors(const TftOps<T>& o, const Group<NTH>& g, T* s, int vs, int lnv, int K, uint32_t lam,
                             const TwPair<T>* tw, const TwPair<T>* twi, gcptr<PassConst<T>> pc, int d0 = 0,
                             uint32_t h0 = 0, int eoff = 0) {
  const int nv = 1 << lnv;
  const uint32_t lm = lam - 1;
  int stop = K;
  // descent (the vectors are block h0 at depth d0; level i handles block h of depth d0 + i)
  for (int i = 0; i <= K; ++i) {
    const int m = K - i;
    const uint32_t mask = (1u << m) - 1;
    const uint32_t hl = m == K ? 0u : lm >> m;  // block index inside the vector
    const uint32_t h = (h0 << i) | hl;
    const int d = d0 + i;
    const int off = eoff + (int)(hl << m);  // element offset of the level's block
    if ((lm & mask) == mask) {  // the whole block is known: one normalized inverse
      inv_block_norm<T, NTH>(o, g, s, vs, lnv, off, d, h, m, twi, pc);
      stop = i;
      break;
    }
    const int half = 1 << (m - 1);
    const int l = (int)(lm & mask) + 1;
    const TwPair<T> w = tw[(1u << d) + h];
    if (l <= half) {
      for (int idx = g.tid; idx < ((half - l) << lnv); idx += NTH) {
        const int v = idx & (nv - 1), j = l + (idx >> lnv);
        T* sv = s + v * vs;
        sv[lidx(off + j)] = o.add(sv[lidx(off + j)], o.mul(sv[lidx(off + j + half)], w));
      }
      g.sync();
    } else {
      inv_block_norm<T, NTH>(o, g, s, vs, lnv, off, d + 1, 2 * h, m - 1, twi, pc);
      const int lo = l - half;
      for (int idx = g.tid; idx < ((half - lo) << lnv); idx += NTH) {
        const int v = idx & (nv - 1), j = lo + (idx >> lnv);
        T* sv = s + v * vs;
        const T y1 = sv[lidx(off + j + half)];
        const T wy = o.mul(y1, w);
        const T y0 = o.sub(sv[lidx(off + j)], wy);
        sv[lidx(off + j)] = y0;
        sv[lidx(off + j + half)] = o.sub(y0, wy);
      }
      g.sync();
    }
  }
  // ascent
  for (int i = stop - 1; i >= 0; --i) {
    const int m = K - i;
    const uint32_t mask = (1u << m) - 1;
    const uint32_t hl = m == K ? 0u : lm >> m;
    const uint32_t h = (h0 << i) | hl;
    const int d = d0 + i;
    const int off = eoff + (int)(hl << m);  // element offset of the level's block
    const int half = 1 << (m - 1);
    const int l = (int)(lm & mask) + 1;
    if (l <= half) {
      const TwPair<T> w = tw[(1u << d) + h];
      for (int idx = g.tid; idx < (l << lnv); idx += NTH) {
        const int v = idx & (nv - 1), j = idx >> lnv;
        T* sv = s + v * vs;
        sv[lidx(off + j)] = o.sub(sv[lidx(off + j)], o.mul(sv[lidx(off + j + half)], w));
      }
    } else {
      const TwPair<T> wi = twi[(1u << d) + h];
      for (int idx = g.tid; idx < ((l - half) << lnv); idx += NTH) {
        const int v = idx & (nv - 1), j = idx >> lnv;
        T* sv = s + v * vs;
        const T u = sv[lidx(off + j)], x = sv[lidx(off + j + half)];
        sv[lidx(off + j)] = o.halve(o.add(u, x));
        sv[lidx(off + j + half)] = o.halve(o.mul(o.sub(u, x), wi));
      }
    }
    g.sync();
  }
}

__device__ __forceinline__ uint32_t brev_n(uint32_t i, int L) { return L == 0 ? 0u : (__brev(i) >> (32 - L)); }

// x w_N^e with w_N^e = lo[e mod 2^B] hi[e >> B] (canonical result).
template <typename T>
__device__ __forceinline__ T twist_e(const TftOps<T>& o, T x, uint64_t e, int B, gcptr<TwPair<T>> lo,
                                     gcptr<TwPair<T>> hi) {
  const TwPair<T> a = ldtw<T>(hi + (e >> B));
  const TwPair<T> b = ldtw<T>(lo + (e & ((1ull << B) - 1)));
  return o.mul(o.mul(x, a), b);
}

// Column pass: tiles of C = 2^(TILELOG - K) adjacent columns of one vector (K = L1).
// The inputs of a column at rows >= lam are zero (a product's coefficients above its
// length, a TFT's inputs above l).  When lam > 2^(K-1), the first half of every column's
// TFT values is known in full: its plain inverse runs as wave-local radix-16 rounds,
// and then y_j = u_j and v_j = u_j for j >= lam - 2^(K-1) (the partner input is zero),
// which leaves the inverse TFT of the second half (block 1 at depth 1) with lam - 2^(K-1)
// values, then y_j = (u_j + v_j) / 2, y_(j+half) = (u_j - v_j) / 2 (the twiddle of the
// first stage is 1).  The universal tables' first 2^K entries are copied to LDS once;
// each wave inverts its own columns.
template <typename T, int LAZY, int NT, int TILELOG, int K>
__device__ void col_itft_body(const TftArgs& A, T* s, TwPair<T>* stw, TwPair<T>* stwi, uint64_t tile,
                              const TftOps<T>& o, gcptr<PassConst<T>> pc) {
  const int L2 = (int)A.L2;
  constexpr int LC0 = TILELOG - K;
  const int LC = LC0 < L2 ? LC0 : L2;
  const int C = 1 << LC;
  constexpr int VS = lds_words(1 << K) + 1;
  const uint64_t tiles_per_vec = 1ull << (L2 - LC);
  const uint32_t lam = A.lam;
  const int B = (int)uni(pc->B);
  constexpr int NW = NT / 64;
  const int lcw = LC > (NW == 16 ? 4 : 3) ? LC - (NW == 16 ? 4 : 3) : 0;  // log2 columns per wave
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  Group<64> g;
  g.tid = lane;
  const uint64_t vec = tile / tiles_per_vec;
  const uint32_t col0 = (uint32_t)(tile % tiles_per_vec) << LC;
  if (col0 + (uint32_t)C <= A.c_lo || col0 >= A.c_hi) return;  // the same in every thread
  const gcptr<T> in = gconst<T>(A.in) + vec * A.in_stride;
  for (int idx = threadIdx.x; idx < (C << K); idx += NT) {
    const uint32_t r = (uint32_t)idx >> LC, cc = (uint32_t)idx & (C - 1);
    // the row passes leave values in [0, 2p) (lazy ranges): reduce on the way in
    s[cc * VS + lidx((int)r)] = r < lam ? o.ar.red1(in[((uint64_t)r << L2) + col0 + cc]) : (T)0;
  }
  __syncthreads();
  if constexpr (K >= 1) {
    constexpr int H = 1 << (K - 1);
    if (lam > (uint32_t)H) {
      // plain inverse of the first half of every column (unnormalized): V half-columns per
      // wave step, so that every wave of the tile has some
      constexpr int CT = 1 << (LC0 > 0 ? LC0 : 0);
      constexpr int V = CT / NW > 0 ? CT / NW : 1;
      for (int v0 = wave * V; v0 < C; v0 += NW * V)
        vec_inv_rounds<T, LAZY, K - 1, V, K - 1>(o.ar, s + v0 * VS, VS, lane, gconst<TwPair<T>>(A.twi));
      __syncthreads();
      const TwPair<T> sc = ldtw<T>(&pc->inv2pow[K - 1]);
      const int lo = (int)lam - H;
      if ((wave << lcw) < C) {
        T* sw = s + (wave << lcw) * VS;
        const int nvw = 1 << lcw;
        for (int idx = lane; idx < (H << lcw); idx += 64) {
          const int v = idx & (nvw - 1), j = idx >> lcw;
          T* sv = sw + v * VS;
          const T u = o.mul(o.ar.red1(sv[lidx(j)]), sc);  // u_j, canonical
          sv[lidx(j)] = u;
          if (j >= lo) sv[lidx(j + H)] = u;  // y_j = u_j and v_j = u_j: the partner input is 0
        }
        g.sync();
        // the second half: block 1 at depth 1, its elements H words into each column
        if (lo > 0) itft_vectors<T, 64>(o, g, sw, VS, lcw, K - 1, (uint32_t)lo, stw, stwi, pc, 1, 1u, H);
        for (int idx = lane; idx < (lo << lcw); idx += 64) {
          const int v = idx & (nvw - 1), j = idx >> lcw;
          T* sv = sw + v * VS;
          const T u = sv[lidx(j)], x = sv[lidx(j + H)];
          sv[lidx(j)] = o.halve(o.add(u, x));
          sv[lidx(j + H)] = o.halve(o.sub(u, x));
        }
      }
    } else if ((wave << lcw) < C) {
      itft_vectors<T, 64>(o, g, s + (wave << lcw) * VS, VS, lcw, K, lam, stw, stwi, pc);
    }
  }
  __syncthreads();
  const gptr<T> out = gmut<T>(A.out) + vec * A.out_stride;
  for (int idx = threadIdx.x; idx < ((int)lam << LC); idx += NT) {
    const uint32_t r = (uint32_t)idx >> LC, cc = (uint32_t)idx & (C - 1);
    const uint32_t c = col0 + cc;
    const uint64_t gi = ((uint64_t)r << L2) + c;
    if (c >= A.c_lo && c < A.c_hi && gi < A.valid) out[gi] = s[cc * VS + lidx((int)r)];
  }
  if (A.eval_next) {
    // each column's TFT value at position lam (Horner at w_(2^K)^([lam]_K)), twisted by
    // w_N^([lam]_K c) as the row pass twists row lam
    TwPair<T> z;
    z.w = (T)0;
    z.ws = (T)0;
    if constexpr (std::is_same<T, double>::value) z.w = A.zeta_d;
    else {
      z.w = (T)A.zeta;
      z.ws = (T)A.zeta_s;
    }
    const uint64_t rr = brev_n(lam, K);
    for (int cc = threadIdx.x; cc < C; cc += NT) {
      const uint32_t c = col0 + (uint32_t)cc;
      if (c < A.c_lo || c >= A.c_hi) continue;
      T acc = (T)0;
      for (int r = (int)lam - 1; r >= 0; --r) acc = o.add(o.mul(acc, z), s[cc * VS + lidx(r)]);
      const T tv = twist_e(o, acc, rr * c, B, gconst<TwPair<T>>(A.tlo), gconst<TwPair<T>>(A.thi));
      gmut<T>(A.rowbuf)[vec * A.rowbuf_stride + c] = tv;
    }
  }
  __syncthreads();
}

template <typename T, int NT, int TILELOG, int K>
__global__ __launch_bounds__(NT) void col_itft_kernel(TftArgs A, uint64_t ntiles) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TftOps<T> o = tft_ops<T>(A.pc);
  const gcptr<PassConst<T>> pc = gconst<PassConst<T>>(uni(A.pc));
  TwPair<T>* stw = (TwPair<T>*)smem_raw;
  TwPair<T>* stwi = stw + (1 << K);
  T* s = (T*)(stwi + (1 << K));
  {
    const gcptr<TwPair<T>> tw = gconst<TwPair<T>>(A.tw), twi = gconst<TwPair<T>>(A.twi);
    for (int i = threadIdx.x; i < (1 << K); i += NT) {
      stw[i] = ldtw<T>(tw + i);
      stwi[i] = ldtw<T>(twi + i);
    }
  }
  __syncthreads();
  const bool lazy = uni(pc->lazy) != 0;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    if (lazy) col_itft_body<T, true, NT, TILELOG, K>(A, s, stw, stwi, tile, o, pc);
    else col_itft_body<T, false, NT, TILELOG, K>(A, s, stw, stwi, tile, o, pc);
  }
}

// The partially known row r = lastrow of each vector (one workgroup per vector).
template <typename T, int NT>
__global__ __launch_bounds__(NT) void row_itft_kernel(TftArgs A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* s = (T*)smem_raw;
  const TftOps<T> o = tft_ops<T>(A.pc);
  const gcptr<PassConst<T>> pc = gconst<PassConst<T>>(uni(A.pc));
  const int L2 = (int)A.L2, L1 = (int)A.L1;
  const int n1 = 1 << L2;
  const uint32_t lam = A.lam, r = A.lastrow;
  const int B = (int)uni(pc->B);
  const uint64_t rr = brev_n(r, L1);
  for (uint64_t vec = blockIdx.x; vec < A.batch; vec += gridDim.x) {
    const gcptr<T> in = gconst<T>(A.in) + vec * A.in_stride + ((uint64_t)r << L2);
    const gcptr<T> rb = gconst<T>(A.rowbuf) + vec * A.rowbuf_stride;
    for (int j = threadIdx.x; j < n1; j += NT) s[lidx(j)] = (uint32_t)j < lam ? in[j] : rb[j];
    __syncthreads();
    Group<NT> g;
    g.tid = threadIdx.x;
    itft_vectors<T, NT>(o, g, s, 0, 0, L2, lam, (const TwPair<T>*)A.tw, (const TwPair<T>*)A.twi, pc);
    const gptr<T> out = gmut<T>(A.out) + vec * A.out_stride + ((uint64_t)r << L2);
    for (int j = threadIdx.x; j < (int)lam; j += NT)
      out[j] = twist_e(o, s[lidx(j)], rr * (uint64_t)j, B, gconst<TwPair<T>>(A.tilo), gconst<TwPair<T>>(A.tihi));
    __syncthreads();
  }
}

// One LDS-resident vector of 2^L words per batch item.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void vec_itft_kernel(TftArgs A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* s = (T*)smem_raw;
  const TftOps<T> o = tft_ops<T>(A.pc);
  const gcptr<PassConst<T>> pc = gconst<PassConst<T>>(uni(A.pc));
  const int L = (int)A.L;
  const int n = 1 << L;
  const uint32_t lam = A.lam;
  for (uint64_t vec = blockIdx.x; vec < A.batch; vec += gridDim.x) {
    const gcptr<T> in = gconst<T>(A.in) + vec * A.in_stride;
    for (int j = threadIdx.x; j < n; j += NT) s[lidx(j)] = (uint32_t)j < lam ? in[j] : (T)0;
    __syncthreads();
    Group<NT> g;
    g.tid = threadIdx.x;
    itft_vectors<T, NT>(o, g, s, 0, 0, L, lam, (const TwPair<T>*)A.tw, (const TwPair<T>*)A.twi, pc);
    const gptr<T> out = gmut<T>(A.out) + vec * A.out_stride;
    for (int j = threadIdx.x; j < (int)lam; j += NT)
      if ((uint64_t)j < A.valid) out[j] = s[lidx(j)];
    __syncthreads();
  }
}

int grid_for(uint64_t items) { return (int)(items < 65536ull ? (items ? items : 1) : 65536ull); }

template <typename T, int NT, int TILELOG, int K>
hipError_t launch_col_itft_k(const TftArgs& a, hipStream_t stream) {
  const int L2 = (int)a.L2;
  if (a.lam == 0 || a.lam > (1u << K)) return hipErrorInvalidValue;
  const int LC = TILELOG - K < L2 ? TILELOG - K : L2;
  const uint64_t ntiles = (uint64_t)a.batch << (L2 - LC);
  const size_t lds = (size_t)(1 << LC) * (lds_words(1 << K) + 1) * sizeof(T) + 2 * ((size_t)1 << K) * sizeof(TwPair<T>);
  auto k = col_itft_kernel<T, NT, TILELOG, K>;
  hipError_t e = allow_dynamic_lds((const void*)k, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(grid_for(ntiles)), dim3(NT), lds, stream, a, ntiles);
  return hipGetLastError();
}

template <typename T, int NT, int TILELOG>
hipError_t launch_col_itft_t(const TftArgs& a, hipStream_t stream) {
  switch (a.L1) {
#define NTT_ITFT_COL(KK) \
  case KK: return launch_col_itft_k<T, NT, TILELOG, KK>(a, stream);
    NTT_ITFT_COL(1) NTT_ITFT_COL(2) NTT_ITFT_COL(3) NTT_ITFT_COL(4) NTT_ITFT_COL(5) NTT_ITFT_COL(6) NTT_ITFT_COL(7)
    NTT_ITFT_COL(8) NTT_ITFT_COL(9) NTT_ITFT_COL(10)
#undef NTT_ITFT_COL
  }
  return hipErrorInvalidValue;
}

template <typename T, int NT, int MAXLOG>
hipError_t launch_one_vector(bool row, const TftArgs& a, hipStream_t stream) {
  const int K = row ? (int)a.L2 : (int)a.L;
  if (K > MAXLOG || a.lam == 0 || a.lam > (1u << K)) return hipErrorInvalidValue;
  const size_t lds = (size_t)lds_words(1 << K) * sizeof(T);
  if (row) {
    auto k = row_itft_kernel<T, NT>;
    hipError_t e = allow_dynamic_lds((const void*)k, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(grid_for(a.batch)), dim3(NT), lds, stream, a);
  } else {
    auto k = vec_itft_kernel<T, NT>;
    hipError_t e = allow_dynamic_lds((const void*)k, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(grid_for(a.batch)), dim3(NT), lds, stream, a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_col_itft(int word_bits, const TftArgs& a, hipStream_t stream) {
  if (a.batch == 0) return hipSuccess;
  if (word_bits == 32) return launch_col_itft_t<uint32_t, 1024, 14>(a, stream);
  return launch_col_itft_t<uint64_t, 512, 13>(a, stream);
}

hipError_t launch_row_itft(int word_bits, const TftArgs& a, hipStream_t stream) {
  if (a.batch == 0) return hipSuccess;
  if (word_bits == 32) return launch_one_vector<uint32_t, 1024, 14>(true, a, stream);
  return launch_one_vector<uint64_t, 512, 13>(true, a, stream);
}

hipError_t launch_vec_itft(int word_bits, const TftArgs& a, hipStream_t stream) {
  if (a.batch == 0) return hipSuccess;
  if (word_bits == 32) return launch_one_vector<uint32_t, 1024, 14>(false, a, stream);
  return launch_one_vector<uint64_t, 512, 13>(false, a, stream);
}

}  // namespace nttgpu
