// Transform kernels (section 5.1).
//
// * lds_ntt_kernel: one workgroup per vector for lengths that fit LDS.
// * Two-pass transforms for longer vectors, following Algorithm 1 with the vector
//   laid out as 2^L1 rows of 2^L2 contiguous elements:
//     column pass: the 2^L2 columns (stride 2^L2) are length-2^L1 transforms, i.e.
//       the global stages 0 .. L1-1 of the in-place Cooley-Tukey form; a workgroup
//       takes C adjacent columns so that every HBM access is a run of C words;
//     row pass: row r is twisted by G^j, G = w_N^([r]_L1) (Algorithm 1, step 2) and
//       transformed (step 3); the output stays in place, which is the TFT order of
//       step 4.  The inverse runs the mirror sequence with G^-j.
//   A fused row pass serves the polynomial product: twist, forward both operands,
//   entry-wise product, inverse, inverse twist, all in LDS.
#include <mutex>
#include <unordered_map>

#include "kernels.hpp"

namespace nttgpu {

hipError_t allow_dynamic_lds(const void* kernel, size_t bytes) {
  static std::mutex mu;
  static std::unordered_map<const void*, size_t> granted;
  std::lock_guard<std::mutex> lk(mu);
  size_t& g = granted[kernel];
  if (bytes <= g) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) g = bytes;
  return e;
}

__device__ __forceinline__ uint32_t brev_bits(uint32_t i, int L) { return L == 0 ? 0u : (__brev(i) >> (32 - L)); }

template <typename T>
__device__ __forceinline__ Arith<T> arith_from(const PassConst<T>* pc) {
  Arith<T> ar;
  ar.p = pc->p;
  ar.p2 = pc->p2;
  ar.pinv = pc->pinv;
  return ar;
}

// ----------------------------------------------------------------------------- LDS-resident
template <typename T, int LAZY, int NT>
__device__ void lds_fwd_body(const LdsNttArgs& A, T* s, uint64_t vec) {
  const PassConst<T>* pc = (const PassConst<T>*)A.pc;
  const Arith<T> ar = arith_from(pc);
  const int L = (int)A.L;
  const int n = 1 << L;
  const T* in = (const T*)A.in + vec * A.stride;
  T* out = (T*)A.out + vec * (A.out_stride ? A.out_stride : A.stride);
  // truncated transforms: inputs at positions >= nin read as 0, outputs >= nout not stored
  const int nin = A.nin ? (int)A.nin : n, nout = A.nout ? (int)A.nout : n;
  for (int i = threadIdx.x; i < n; i += NT) s[lidx(i)] = i < nin ? in[i] : (T)0;
  __syncthreads();
  fwd_lds<T, LAZY, NT, false>(ar, s, nullptr, L, 0, 0u, (const TwPair<T>*)A.tw);
  for (int i = threadIdx.x; i < nout; i += NT) {
    const int src = A.bitrev ? i : (int)brev_bits((uint32_t)i, L);
    out[i] = canon_from_fwd<LAZY>(ar, s[lidx(src)]);
  }
  __syncthreads();
}

template <typename T, int LAZY, int NT>
__device__ void lds_inv_body(const LdsNttArgs& A, T* s, uint64_t vec) {
  const PassConst<T>* pc = (const PassConst<T>*)A.pc;
  const Arith<T> ar = arith_from(pc);
  const int L = (int)A.L;
  const int n = 1 << L;
  const T* in = (const T*)A.in + vec * A.stride;
  T* out = (T*)A.out + vec * (A.out_stride ? A.out_stride : A.stride);
  const TwPair<T> ninv = pc->ninv;
  for (int i = threadIdx.x; i < n; i += NT) {
    T x = ar.shoup(in[i], ninv.w, ninv.ws);  // n^-1 applied on the way in
    if constexpr (LAZY != kLazy) x = ar.red1(x);
    const int dst = A.bitrev ? i : (int)brev_bits((uint32_t)i, L);
    s[lidx(dst)] = x;
  }
  __syncthreads();
  inv_lds<T, LAZY, NT>(ar, s, L, 0, 0u, (const TwPair<T>*)A.twi);
  for (int i = threadIdx.x; i < n; i += NT) out[i] = canon_from_inv<LAZY>(ar, s[lidx(i)]);
  __syncthreads();
}

template <typename T, int NT, int LOGS, bool INV>
__global__ __launch_bounds__(NT) void lds_ntt_kernel(LdsNttArgs A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* s = (T*)smem_raw;
  const PassConst<T>* pc = (const PassConst<T>*)A.pc;
  const int mode = (int)pc->lazy;
  for (uint64_t v = blockIdx.x; v < A.batch; v += gridDim.x) {
    with_mode<T>(mode, [&](auto m) {
      if constexpr (INV) lds_inv_body<T, decltype(m)::value, NT>(A, s, v);
      else lds_fwd_body<T, decltype(m)::value, NT>(A, s, v);
    });
  }
}

int lds_max_log2n(int word_bits) { return word_bits == 32 ? 14 : 13; }

template <typename T, int NT, int LOGS>
static hipError_t launch_lds_cls(bool inverse, const LdsNttArgs& a, hipStream_t stream) {
  const size_t lds = (size_t)lds_words(1 << LOGS) * sizeof(T);
  const int grid = (int)(a.batch < 65536u ? a.batch : 65536u);
  if (inverse) {
    auto k = lds_ntt_kernel<T, NT, LOGS, true>;
    hipError_t e = allow_dynamic_lds((const void*)k, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(grid), dim3(NT), lds, stream, a);
  } else {
    auto k = lds_ntt_kernel<T, NT, LOGS, false>;
    hipError_t e = allow_dynamic_lds((const void*)k, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(grid), dim3(NT), lds, stream, a);
  }
  return hipGetLastError();
}

hipError_t launch_lds_ntt(int word_bits, bool inverse, const LdsNttArgs& a, hipStream_t stream) {
  if (a.batch == 0) return hipSuccess;
  const int L = (int)a.L;
  if (word_bits == 32) {
    if (L <= 10) return launch_lds_cls<uint32_t, 64, 10>(inverse, a, stream);
    if (L <= 12) return launch_lds_cls<uint32_t, 256, 12>(inverse, a, stream);
    return launch_lds_cls<uint32_t, 1024, 14>(inverse, a, stream);
  }
  if (word_bits == kWordF64) {
    if (L <= 10) return launch_lds_cls<double, 64, 10>(inverse, a, stream);
    if (L <= 12) return launch_lds_cls<double, 256, 12>(inverse, a, stream);
    return launch_lds_cls<double, 1024, 13>(inverse, a, stream);
  }
  if (L <= 10) return launch_lds_cls<uint64_t, 64, 10>(inverse, a, stream);
  if (L <= 12) return launch_lds_cls<uint64_t, 256, 12>(inverse, a, stream);
  return launch_lds_cls<uint64_t, 1024, 13>(inverse, a, stream);
}

// ----------------------------------------------------------------------------- two-pass
constexpr int kColTileLog32 = 14;  // words per column tile (C columns x 2^L1 rows)
constexpr int kColTileLog64 = 13;
constexpr int kRowMaxLog32 = 14;
constexpr int kRowMaxLog64 = 13;

int pass_max_row_log2(int word_bits) { return word_bits == 32 ? kRowMaxLog32 : kRowMaxLog64; }
int pass_col_tile_log2(int word_bits) { return word_bits == 32 ? kColTileLog32 : kColTileLog64; }

__device__ __forceinline__ int col_vs(int L1) { return lds_words(1 << L1) + 1; }  // odd: columns in different banks

template <typename T, int LAZY, int NT, int TILELOG, typename IN_T>
__device__ void col_fwd_body(const PassArgs& A, T* s, uint64_t tile) {
  const PassConst<T>* pc = (const PassConst<T>*)A.pc;
  const Arith<T> ar = arith_from(pc);
  const int L1 = (int)pc->L1, L2 = (int)pc->L2;
  const int LC = (TILELOG - L1) < L2 ? (TILELOG - L1) : L2;
  const int C = 1 << LC;
  const uint64_t tiles_per_vec = 1ull << (L2 - LC);
  const uint64_t vec = tile / tiles_per_vec;
  const uint32_t col0 = (uint32_t)(tile % tiles_per_vec) << LC;
  const int vs = col_vs(L1);
  const IN_T* in = (const IN_T*)A.in + vec * A.in_stride;
  T* out = (T*)A.out + vec * A.out_stride;
  const int cnt = C << L1;
  const TwPair<T> sig = pc->sigma;
  for (int idx = threadIdx.x; idx < cnt; idx += NT) {
    const uint32_t r = (uint32_t)idx >> LC, cc = (uint32_t)idx & (C - 1);
    const uint64_t gi = ((uint64_t)r << L2) + col0 + cc;
    T x = gi < A.valid ? (T)in[gi] : (T)0;
    if (A.scale) x = ar.red1(ar.shoup(x, sig.w, sig.ws));
    s[cc * vs + lidx(r)] = x;
  }
  __syncthreads();
  fwd_lds_multi<T, LAZY, NT>(ar, s, vs, C, L1, (const TwPair<T>*)A.tw);
  for (int idx = threadIdx.x; idx < cnt; idx += NT) {
    const uint32_t r = (uint32_t)idx >> LC, cc = (uint32_t)idx & (C - 1);
    const uint64_t gi = ((uint64_t)r << L2) + col0 + cc;
    out[gi] = s[cc * vs + lidx(r)];
  }
  __syncthreads();
}

template <typename T, int LAZY, int NT, int TILELOG>
__device__ void col_inv_body(const PassArgs& A, T* s, uint64_t tile) {
  const PassConst<T>* pc = (const PassConst<T>*)A.pc;
  const Arith<T> ar = arith_from(pc);
  const int L1 = (int)pc->L1, L2 = (int)pc->L2;
  const int LC = (TILELOG - L1) < L2 ? (TILELOG - L1) : L2;
  const int C = 1 << LC;
  const uint64_t tiles_per_vec = 1ull << (L2 - LC);
  const uint64_t vec = tile / tiles_per_vec;
  const uint32_t col0 = (uint32_t)(tile % tiles_per_vec) << LC;
  const int vs = col_vs(L1);
  const T* in = (const T*)A.in + vec * A.in_stride;
  T* out = (T*)A.out + vec * A.out_stride;
  const int cnt = C << L1;
  for (int idx = threadIdx.x; idx < cnt; idx += NT) {
    const uint32_t r = (uint32_t)idx >> LC, cc = (uint32_t)idx & (C - 1);
    s[cc * vs + lidx(r)] = in[((uint64_t)r << L2) + col0 + cc];
  }
  __syncthreads();
  inv_lds_multi<T, LAZY, NT>(ar, s, vs, C, L1, (const TwPair<T>*)A.twi);
  for (int idx = threadIdx.x; idx < cnt; idx += NT) {
    const uint32_t r = (uint32_t)idx >> LC, cc = (uint32_t)idx & (C - 1);
    const uint64_t gi = ((uint64_t)r << L2) + col0 + cc;
    if (gi < A.valid) out[gi] = canon_from_inv<LAZY>(ar, s[cc * vs + lidx(r)]);
  }
  __syncthreads();
}

template <typename T, int NT, int TILELOG, bool INV, typename IN_T>
__global__ __launch_bounds__(NT) void col_kernel(PassArgs A, uint64_t ntiles) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* s = (T*)smem_raw;
  const int mode = (int)((const PassConst<T>*)A.pc)->lazy;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    with_mode<T>(mode, [&](auto m) {
      if constexpr (INV) col_inv_body<T, decltype(m)::value, NT, TILELOG>(A, s, t);
      else col_fwd_body<T, decltype(m)::value, NT, TILELOG, IN_T>(A, s, t);
    });
  }
}

// Twist factor G^j = w_N^(j [r]_L1) as the product of two table entries (both with
// their Shoup companions); x may be any word, the result lies in [0, 2p).
template <typename T>
__device__ __forceinline__ T twist(const Arith<T>& ar, T x, uint32_t e, int B, const TwPair<T>* __restrict__ lo,
                                   const TwPair<T>* __restrict__ hi) {
  const TwPair<T> h = hi[e >> B];
  const TwPair<T> l = lo[e & ((1u << B) - 1)];
  return ar.shoup(ar.shoup(x, h.w, h.ws), l.w, l.ws);
}

template <typename T, int LAZY, int NT>
__device__ void row_fwd_body(const PassArgs& A, T* s, uint64_t rowid) {
  const PassConst<T>* pc = (const PassConst<T>*)A.pc;
  const Arith<T> ar = arith_from(pc);
  const int L1 = (int)pc->L1, L2 = (int)pc->L2, B = (int)pc->B;
  const int n2 = 1 << L2;
  const uint64_t vec = rowid >> L1;
  const uint32_t r = (uint32_t)(rowid & ((1u << L1) - 1));
  const uint32_t R = brev_bits(r, L1);
  const T* in = (const T*)A.in + vec * A.in_stride + ((uint64_t)r << L2);
  T* out = (T*)A.out + vec * A.out_stride + ((uint64_t)r << L2);
  const TwPair<T>* lo = (const TwPair<T>*)A.tlo;
  const TwPair<T>* hi = (const TwPair<T>*)A.thi;
  for (int j = threadIdx.x; j < n2; j += NT) s[lidx(j)] = twist(ar, in[j], (uint32_t)j * R, B, lo, hi);
  __syncthreads();
  fwd_lds<T, LAZY, NT, false>(ar, s, nullptr, L2, 0, 0u, (const TwPair<T>*)A.tw);
  for (int j = threadIdx.x; j < n2; j += NT) out[j] = canon_from_fwd<LAZY>(ar, s[lidx(j)]);
  __syncthreads();
}

template <typename T, int LAZY, int NT>
__device__ void row_inv_body(const PassArgs& A, T* s, uint64_t rowid) {
  const PassConst<T>* pc = (const PassConst<T>*)A.pc;
  const Arith<T> ar = arith_from(pc);
  const int L1 = (int)pc->L1, L2 = (int)pc->L2, B = (int)pc->B;
  const int n2 = 1 << L2;
  const uint64_t vec = rowid >> L1;
  const uint32_t r = (uint32_t)(rowid & ((1u << L1) - 1));
  const uint32_t R = brev_bits(r, L1);
  const T* in = (const T*)A.in + vec * A.in_stride + ((uint64_t)r << L2);
  T* out = (T*)A.out + vec * A.out_stride + ((uint64_t)r << L2);
  for (int j = threadIdx.x; j < n2; j += NT) s[lidx(j)] = in[j];  // canonical input
  __syncthreads();
  inv_lds<T, LAZY, NT>(ar, s, L2, 0, 0u, (const TwPair<T>*)A.twi);
  const TwPair<T>* lo = (const TwPair<T>*)A.tilo;
  const TwPair<T>* hi = (const TwPair<T>*)A.tihi;
  for (int j = threadIdx.x; j < n2; j += NT) {
    T x = twist(ar, s[lidx(j)], (uint32_t)j * R, B, lo, hi);
    if constexpr (LAZY != kLazy) x = ar.red1(x);
    out[j] = x;
  }
  __syncthreads();
}

template <typename T, int LAZY, int NT>
__device__ void row_polymul_body(const PassArgs& A, T* sa, T* sb, uint64_t rowid) {
  const PassConst<T>* pc = (const PassConst<T>*)A.pc;
  const Arith<T> ar = arith_from(pc);
  const int L1 = (int)pc->L1, L2 = (int)pc->L2, B = (int)pc->B;
  const int n2 = 1 << L2;
  const uint64_t vec = rowid >> L1;
  const uint32_t r = (uint32_t)(rowid & ((1u << L1) - 1));
  const uint32_t R = brev_bits(r, L1);
  const uint64_t off = (uint64_t)r << L2;
  const T* ina = (const T*)A.in + vec * A.in_stride + off;
  const T* inb = (const T*)A.in2 + vec * A.in_stride + off;
  T* out = (T*)A.out + vec * A.out_stride + off;
  const TwPair<T>* lo = (const TwPair<T>*)A.tlo;
  const TwPair<T>* hi = (const TwPair<T>*)A.thi;
  for (int j = threadIdx.x; j < n2; j += NT) {
    const uint32_t e = (uint32_t)j * R;
    sa[lidx(j)] = twist(ar, ina[j], e, B, lo, hi);
    sb[lidx(j)] = twist(ar, inb[j], e, B, lo, hi);
  }
  __syncthreads();
  fwd_lds<T, LAZY, NT, true>(ar, sa, sb, L2, 0, 0u, (const TwPair<T>*)A.tw);
  for (int j = threadIdx.x; j < n2; j += NT) {
    T x = sa[lidx(j)], y = sb[lidx(j)];
    if constexpr (LAZY == kLazy) {
      x = ar.red1(ar.red2(x));
    } else {  // x < p, y < 2p: x y < 2p^2 < 2^bits p (Function 13's bound)
      x = ar.red1(x);
      if constexpr (LAZY == kBand) y = ar.red1(y);  // Function 16 needs x y < 2^50 p
    }
    T z = ar.mont(x, y);
    if constexpr (LAZY != kLazy) z = ar.red1(z);
    sa[lidx(j)] = z;
  }
  __syncthreads();
  inv_lds<T, LAZY, NT>(ar, sa, L2, 0, 0u, (const TwPair<T>*)A.twi);
  const TwPair<T>* ilo = (const TwPair<T>*)A.tilo;
  const TwPair<T>* ihi = (const TwPair<T>*)A.tihi;
  for (int j = threadIdx.x; j < n2; j += NT) {
    T x = twist(ar, sa[lidx(j)], (uint32_t)j * R, B, ilo, ihi);
    if constexpr (LAZY != kLazy) x = ar.red1(x);
    out[j] = x;
  }
  __syncthreads();
}

// KIND: 0 forward, 1 inverse, 2 fused product
template <typename T, int NT, int KIND>
__global__ __launch_bounds__(NT) void row_kernel(PassArgs A, uint64_t nrows) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* s = (T*)smem_raw;
  const PassConst<T>* pc = (const PassConst<T>*)A.pc;
  const int mode = (int)pc->lazy;
  T* s2 = s + lds_words(1 << pc->L2);
  for (uint64_t t = blockIdx.x; t < nrows; t += gridDim.x) {
    with_mode<T>(mode, [&](auto m) {
      constexpr int MODE = decltype(m)::value;
      if constexpr (KIND == 0) row_fwd_body<T, MODE, NT>(A, s, t);
      else if constexpr (KIND == 1) row_inv_body<T, MODE, NT>(A, s, t);
      else row_polymul_body<T, MODE, NT>(A, s, s2, t);
    });
  }
}

static int grid_for(uint64_t items) { return (int)(items < 1048576ull ? items : 1048576ull); }

template <typename T, int NT, int TILELOG, bool INV, typename IN_T>
static hipError_t launch_col_t(const PassArgs& a, int L1, int L2, hipStream_t stream) {
  const int LC = (TILELOG - L1) < L2 ? (TILELOG - L1) : L2;
  const uint64_t ntiles = (uint64_t)a.batch << (L2 - LC);
  const size_t lds = (size_t)(1 << LC) * (lds_words(1 << L1) + 1) * sizeof(T);
  auto k = col_kernel<T, NT, TILELOG, INV, IN_T>;
  hipError_t e = allow_dynamic_lds((const void*)k, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(grid_for(ntiles)), dim3(NT), lds, stream, a, ntiles);
  return hipGetLastError();
}

hipError_t launch_col_fwd_rounds(int word_bits, const PassArgs& a, int L1, int L2, hipStream_t stream) {
  if (word_bits == 32) {
    if (a.in_u16) return launch_col_t<uint32_t, 1024, kColTileLog32, false, uint16_t>(a, L1, L2, stream);
    return launch_col_t<uint32_t, 1024, kColTileLog32, false, uint32_t>(a, L1, L2, stream);
  }
  return launch_col_t<uint64_t, 512, kColTileLog64, false, uint64_t>(a, L1, L2, stream);
}

hipError_t launch_col_inv_rounds(int word_bits, const PassArgs& a, int L1, int L2, hipStream_t stream) {
  if (word_bits == 32) return launch_col_t<uint32_t, 1024, kColTileLog32, true, uint32_t>(a, L1, L2, stream);
  return launch_col_t<uint64_t, 512, kColTileLog64, true, uint64_t>(a, L1, L2, stream);
}

template <typename T, int NT, int KIND>
static hipError_t launch_row_t(const PassArgs& a, int L1, int L2, hipStream_t stream) {
  const uint64_t nrows = (uint64_t)a.batch << L1;
  const size_t lds = (KIND == 2 ? 2 : 1) * (size_t)lds_words(1 << L2) * sizeof(T);
  auto k = row_kernel<T, NT, KIND>;
  hipError_t e = allow_dynamic_lds((const void*)k, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(grid_for(nrows)), dim3(NT), lds, stream, a, nrows);
  return hipGetLastError();
}

template <int KIND>
static hipError_t launch_row_kind_rounds(int word_bits, const PassArgs& a, int L1, int L2, hipStream_t stream) {
  if (word_bits == 32) {
    if (L2 <= 10) return launch_row_t<uint32_t, 64, KIND>(a, L1, L2, stream);
    if (L2 <= 12) return launch_row_t<uint32_t, 256, KIND>(a, L1, L2, stream);
    return launch_row_t<uint32_t, 1024, KIND>(a, L1, L2, stream);
  }
  if (L2 <= 10) return launch_row_t<uint64_t, 64, KIND>(a, L1, L2, stream);
  if (L2 <= 12) return launch_row_t<uint64_t, 256, KIND>(a, L1, L2, stream);
  return launch_row_t<uint64_t, 512, KIND>(a, L1, L2, stream);
}

hipError_t launch_row_rounds(int word_bits, int kind, const PassArgs& a, int L1, int L2, hipStream_t stream) {
  if (kind == 0) return launch_row_kind_rounds<0>(word_bits, a, L1, L2, stream);
  if (kind == 1) return launch_row_kind_rounds<1>(word_bits, a, L1, L2, stream);
  return launch_row_kind_rounds<2>(word_bits, a, L1, L2, stream);
}

// ----------------------------------------------------------------------------- permutation
// Bit reversal of 2^L indices, i = (a, b, c) with a, c of K bits: [i]_L =
// ([c]_K, [b]_(L-2K), [a]_K).  A workgroup moves the 2^K x 2^K tile of fixed b
// through LDS so that reads and writes are runs of 2^K words.
template <typename T, int K>
__global__ __launch_bounds__(256) void bitrev_tile_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                          uint64_t in_stride, uint64_t out_stride, uint32_t L,
                                                          uint64_t ntiles) {
  constexpr int W = 1 << K;
  __shared__ T tile[W][W + 1];
  const int M = (int)L - 2 * K;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t vec = t >> M;
    const uint32_t bm = (uint32_t)(t & ((1ull << M) - 1));
    const T* src = in + vec * in_stride;
    T* dst = out + vec * out_stride;
    for (int idx = threadIdx.x; idx < W * W; idx += 256) {
      const int a = idx >> K, c = idx & (W - 1);
      tile[a][c] = src[((uint64_t)a << (L - K)) | ((uint64_t)bm << K) | (uint64_t)c];
    }
    __syncthreads();
    const uint32_t rb = brev_bits(bm, M);
    for (int idx = threadIdx.x; idx < W * W; idx += 256) {
      const int rc = idx >> K, ra = idx & (W - 1);  // output (rc, rb, ra)
      const int a = (int)brev_bits((uint32_t)ra, K), c = (int)brev_bits((uint32_t)rc, K);
      dst[((uint64_t)rc << (L - K)) | ((uint64_t)rb << K) | (uint64_t)ra] = tile[a][c];
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void bitrev_small_kernel(const T* __restrict__ in, T* __restrict__ out, uint64_t in_stride,
                                    uint64_t out_stride, uint32_t L, uint64_t total) {
  for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < total; g += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t vec = g >> L;
    const uint32_t i = (uint32_t)(g & ((1ull << L) - 1));
    out[vec * out_stride + i] = in[vec * in_stride + brev_bits(i, (int)L)];
  }
}

template <typename T>
static hipError_t launch_bitrev_t(const void* in, void* out, uint64_t is, uint64_t os, uint32_t L, uint32_t batch,
                                  hipStream_t stream) {
  constexpr int K = 5;
  if (L >= 2 * K) {
    const uint64_t ntiles = (uint64_t)batch << (L - 2 * K);
    hipLaunchKernelGGL((bitrev_tile_kernel<T, K>), dim3(grid_for(ntiles)), dim3(256), 0, stream, (const T*)in, (T*)out,
                       is, os, L, ntiles);
  } else {
    const uint64_t total = (uint64_t)batch << L;
    const int grid = (int)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
    hipLaunchKernelGGL(bitrev_small_kernel<T>, dim3(grid > 0 ? grid : 1), dim3(256), 0, stream, (const T*)in, (T*)out,
                       is, os, L, total);
  }
  return hipGetLastError();
}

hipError_t launch_bitrev_permute(int word_bits, const void* in, void* out, uint64_t in_stride, uint64_t out_stride,
                                 uint32_t L, uint32_t batch, hipStream_t stream) {
  // (doubles are moved as 64-bit patterns)
  if (word_bits == 32) return launch_bitrev_t<uint32_t>(in, out, in_stride, out_stride, L, batch, stream);
  return launch_bitrev_t<uint64_t>(in, out, in_stride, out_stride, L, batch, stream);
}

// ----------------------------------------------------------------------------- small utilities
__global__ void fill_u32_kernel(uint32_t* x, uint64_t n, uint32_t value) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    x[i] = value;
}

hipError_t launch_fill_u32(uint32_t* x, uint64_t n, uint32_t value, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const int grid = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid), dim3(256), 0, stream, x, n, value);
  return hipGetLastError();
}

__global__ void widen_u16_kernel(const uint16_t* __restrict__ in, uint32_t* __restrict__ out, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = in[i];
}

hipError_t launch_widen_u16(const uint16_t* in, uint32_t* out, uint64_t n, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const int grid = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(widen_u16_kernel, dim3(grid), dim3(256), 0, stream, in, out, n);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------- validation
template <typename T>
__global__ void range_check_kernel(const T* __restrict__ x, uint64_t n, uint64_t stride, uint64_t total, T p,
                                   uint32_t* flag) {
  bool bad = false;
  for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < total; g += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t vec = g / n, i = g % n;
    bad |= x[vec * stride + i] >= p;
  }
  if (bad) atomicOr(flag, 1u);
}

hipError_t launch_range_check(int word_bits, const void* x, uint64_t n, uint64_t stride, uint32_t batch, uint64_t p,
                              uint32_t* flag, hipStream_t stream) {
  const uint64_t total = n * batch;
  if (total == 0) return hipSuccess;
  const int grid = (int)((total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096);
  if (word_bits == 32)
    hipLaunchKernelGGL(range_check_kernel<uint32_t>, dim3(grid), dim3(256), 0, stream, (const uint32_t*)x, n, stride,
                       total, (uint32_t)p, flag);
  else
    hipLaunchKernelGGL(range_check_kernel<uint64_t>, dim3(grid), dim3(256), 0, stream, (const uint64_t*)x, n, stride,
                       total, p, flag);
  return hipGetLastError();
}

}  // namespace nttgpu
