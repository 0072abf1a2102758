// Latency path of ONE product (section 5.2 with Algorithm 1, n1 = 2^d): the 2^d
// sub-problems of length S = 2^M run on 2^d workgroups at once instead of one after
// the other in a single workgroup, and a second, short kernel recombines them.
//
// Workgroup h forms the folds f_h[j] = sum_k x[j + k S] psi_h^k, psi_h = w_(2^d)^([h]_d)
// of both operands (the first d forward stages restricted to block h), transforms
// them with the wave-local machinery, multiplies entry-wise (Montgomery, with the
// scale 2^bits/N applied to b's fold), inverse-transforms and writes the partial
// result to the workspace.  The recombination applies the last d inverse stages
// across the 2^d partials position by position and writes the canonical product.
#include "kernels.hpp"
#include "ntt_wave.hpp"

namespace nttgpu {

// psi^k for psi = w_(2^D)^(e0), from the universal table: w_(2^D)^e for
// e < 2^(D-1) is t[2^(D-1) + [e]_(D-1)], the upper half of the circle its negation.
template <typename T, int D>
__device__ __forceinline__ TwPair<T> root_pow(gcptr<TwPair<T>> t, uint32_t e, T p) {
  constexpr uint32_t half = 1u << (D - 1);
  e &= (1u << D) - 1;
  const uint32_t i = D == 1 ? 0u : (__brev(e & (half - 1)) >> (32 - (D - 1)));
  TwPair<T> x = ldtw<T>(t + (half + i));
  if (e >= half) {
    x.w = p - x.w;
    x.ws = ~x.ws;  // floor((p - w) 2^bits / p) = 2^bits - 1 - floor(w 2^bits / p) for 0 < w < p
  }
  return x;
}

template <typename T, int LAZY, int NT, int M, int D>
__device__ void split_sub(const SplitArgs& A, T* sa, T* sb, const Arith<T>& ar) {
  constexpr int S = 1 << M;
  constexpr int K = 1 << D;  // fold terms at most
  const uint32_t h = blockIdx.x;
  const gcptr<PolyConst<T>> pc = gconst<PolyConst<T>>(uni(A.cst));
  const gcptr<TwPair<T>> tw = gconst<TwPair<T>>(uni(A.tw));
  const gcptr<TwPair<T>> twi = gconst<TwPair<T>>(uni(A.twi));
  const gcptr<T> a = gconst<T>(uni(A.a));
  const gcptr<T> b = gconst<T>(uni(A.b));
  const uint64_t la = A.la, lb = A.lb;
  // psi_h^k, and sigma (the Montgomery scale 2^bits / N: fb[0][0] of the plan)
  const uint32_t eh = __brev(h) >> (32 - D);
  const TwPair<T> sigma = uni(ldtw<T>(&pc->fb[0][0]));
  TwPair<T> fa[K];
#pragma unroll
  for (int k = 0; k < K; ++k) fa[k] = uni(root_pow<T, D>(tw, (uint32_t)k * eh, ar.p));
  const int tid = opaque_tid();
  // folds into LDS, natural position order (FB positions' loads in flight together)
  constexpr int FB = 4;
#pragma unroll 1
  for (int j0 = tid; j0 < S; j0 += NT * FB) {
    T xa[FB][K], xb[FB][K];
#pragma unroll
    for (int f = 0; f < FB; ++f)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint64_t idx = (uint64_t)(j0 + f * NT) + (uint64_t)k * S;
        const bool in = j0 + f * NT < S;
        xa[f][k] = (in && idx < la) ? a[idx] : (T)0;
        xb[f][k] = (in && idx < lb) ? b[idx] : (T)0;
      }
#pragma unroll
    for (int f = 0; f < FB; ++f) {
      const int j = j0 + f * NT;
      if (j >= S) break;
      T sa_ = xa[f][0], sb_ = xb[f][0];
#pragma unroll
      for (int k = 1; k < K; ++k) {
        sa_ = ar.red1(sa_ + ar.red1(ar.shoup_u(xa[f][k], fa[k].w, fa[k].ws)));
        sb_ = ar.red1(sb_ + ar.red1(ar.shoup_u(xb[f][k], fa[k].w, fa[k].ws)));
      }
      sa[lidx(j)] = sa_;
      sb[lidx(j)] = ar.red1(ar.shoup_u(sb_, sigma.w, sigma.ws));  // b's fold times sigma
    }
  }
  __syncthreads();
  T* const sv2[2] = {sa, sb};
  fwd_G<T, LAZY, NT, 2, M>(ar, sv2, D, h, tw);
  if ((opaque_tid() >> 6) < (1 << (M - 10))) {
    T x[2][16];
    fwd_W<T, LAZY, 2, M>(ar, sv2, D, h, tw, x);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      T xa = x[0][i], yb = x[1][i];
      if constexpr (LAZY == kLazy) {
        xa = ar.red1(ar.red2(xa));  // xa < p, yb < 4p: xa yb < 2^bits p
      } else {  // xa < p, yb < 2p: xa yb < 2p^2 < 2^bits p (Function 13's bound)
        xa = ar.red1(xa);
        if constexpr (LAZY == kBand) yb = ar.red1(yb);  // Function 16 needs xa yb < 2^50 p
      }
      T z = ar.mont(xa, yb);  // (0, 2p)
      if constexpr (LAZY != kLazy) z = ar.red1(z);
      x[0][i] = z;
    }
    inv_W<T, LAZY, M>(ar, sa, D, h, twi, x[0]);
  }
  inv_G<T, LAZY, NT, M>(ar, sa, D, h, twi);
  const gptr<T> park = gmut<T>(uni(A.park)) + (size_t)h * S;
  for (int j = opaque_tid(); j < S; j += NT) park[j] = sa[lidx(j)];
}

template <typename T, int NT, int M, int D>
__global__ __launch_bounds__(NT) void polymul_split_kernel(SplitArgs A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sa = (T*)smem_raw;
  T* sb = sa + lds_words(1 << M);
  const gcptr<PolyConst<T>> pc = gconst<PolyConst<T>>(uni(A.cst));
  Arith<T> ar;
  ar.p = uni(pc->p);
  ar.p2 = uni(pc->p2);
  ar.pinv = uni(pc->pinv);
  if (uni(pc->lazy)) split_sub<T, true, NT, M, D>(A, sa, sb, ar);
  else split_sub<T, false, NT, M, D>(A, sa, sb, ar);
}

// The last D inverse stages across the 2^D partials (inverse of the fold's
// first D forward stages): stage t = D-1 .. 0 pairs partials (i, i + 2^(D-1-t)) of
// block `blk` with twiddle TWI[2^t + blk]; outputs k go to c[j + k S].
template <typename T, int LAZY, int D>
__device__ __forceinline__ void recombine_one(const SplitArgs& A, const Arith<T>& ar, uint64_t j, int M) {
  constexpr int K = 1 << D;
  const uint64_t S = 1ull << M;
  const gcptr<T> park = gconst<T>(A.park);
  const gcptr<TwPair<T>> twi = gconst<TwPair<T>>(A.twi);
  T u[K];
  const int lam = (int)A.lam;
#pragma unroll
  for (int k = 0; k < K; ++k) u[k] = k < lam ? park[(uint64_t)k * S + j] : (T)0;
  // TFT truncation: the partials h >= lam (not computed) are the combinations of the
  // computed ones that make the coefficients k >= lam vanish
  if constexpr (D >= 2) {
    if (lam < K) {
      const gcptr<PolyConst<T>> pc = gconst<PolyConst<T>>(A.cst);
#pragma unroll
      for (int r = 0; r < K / 2 - 1; ++r) {
        const int row = lam + r;
        if (row >= K) break;
        T acc = 0;
#pragma unroll
        for (int cidx = 0; cidx < K - 1; ++cidx) {
          if (cidx >= lam) break;
          const TwPair<T> f = uni(ldtw<T>(D == 2 ? &pc->tft2[cidx] : &pc->tft3[lam - 5][r][cidx]));
          acc = ar.red1(acc + ar.red1(ar.shoup_u(u[cidx], f.w, f.ws)));
        }
        u[row] = acc;
      }
    }
  }
#pragma unroll
  for (int t = D - 1; t >= 0; --t) {
    const int half = 1 << (D - 1 - t);
#pragma unroll
    for (int blk = 0; blk < (1 << t); ++blk) {
      const TwPair<T> w = uni(ldtw<T>(twi + ((1 << t) + blk)));
#pragma unroll
      for (int i = 0; i < half; ++i) gs_bfly<LAZY, true>(ar, u[blk * 2 * half + i], u[blk * 2 * half + i + half], w);
    }
  }
  const gptr<T> c = gmut<T>(A.c);
  const uint64_t lc = A.la + A.lb - 1;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint64_t o = j + (uint64_t)k * S;
    if (o < lc) c[o] = canon_from_inv<LAZY>(ar, u[k]);
  }
}

template <typename T, int D>
__global__ __launch_bounds__(256) void split_recombine_kernel(SplitArgs A, int M) {
  const gcptr<PolyConst<T>> pc = gconst<PolyConst<T>>(uni(A.cst));
  Arith<T> ar;
  ar.p = uni(pc->p);
  ar.p2 = uni(pc->p2);
  ar.pinv = uni(pc->pinv);
  const bool lazy = uni(pc->lazy) != 0;
  const uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= (1ull << M)) return;
  if (lazy) recombine_one<T, true, D>(A, ar, j, M);
  else recombine_one<T, false, D>(A, ar, j, M);
}

template <typename T, int M, int D>
static hipError_t launch_split_md(const SplitArgs& a, hipStream_t stream) {
  constexpr int NT = 64 << (M - 10);
  const size_t lds = 2 * (size_t)lds_words(1 << M) * sizeof(T);
  auto k = polymul_split_kernel<T, NT, M, D>;
  hipError_t e = allow_dynamic_lds((const void*)k, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(a.lam), dim3(NT), lds, stream, a);
  hipLaunchKernelGGL((split_recombine_kernel<T, D>), dim3(((1u << M) + 255) / 256), dim3(256), 0, stream, a, M);
  return hipGetLastError();
}

template <typename T, int M>
static hipError_t launch_split_m(const SplitArgs& a, int d, hipStream_t stream) {
  switch (d) {
    case 1: return launch_split_md<T, M, 1>(a, stream);
    case 2: return launch_split_md<T, M, 2>(a, stream);
    case 3: return launch_split_md<T, M, 3>(a, stream);
  }
  return hipErrorInvalidValue;
}

bool split_supported(int word_bits, int log2n, int d) {
  // (the launch computes the sub-problems h < lam only, lam = ceil(lc / 2^(log2n - d)))
  const int M = log2n - d;
  if (d < 1 || d > 3) return false;
  return M >= 10 && M <= (word_bits == 32 ? 13 : 12);
}

hipError_t launch_split(int word_bits, const SplitArgs& a, int log2n, int d, hipStream_t stream) {
  if (!split_supported(word_bits, log2n, d)) return hipErrorInvalidValue;
  const int M = log2n - d;
  if (word_bits == 32) {
    switch (M) {
      case 10: return launch_split_m<uint32_t, 10>(a, d, stream);
      case 11: return launch_split_m<uint32_t, 11>(a, d, stream);
      case 12: return launch_split_m<uint32_t, 12>(a, d, stream);
      case 13: return launch_split_m<uint32_t, 13>(a, d, stream);
    }
  } else {
    switch (M) {
      case 10: return launch_split_m<uint64_t, 10>(a, d, stream);
      case 11: return launch_split_m<uint64_t, 11>(a, d, stream);
      case 12: return launch_split_m<uint64_t, 12>(a, d, stream);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace nttgpu
