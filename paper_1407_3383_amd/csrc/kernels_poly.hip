// Fused polynomial product kernels (section 5.2): fold, two forward transforms,
// entry-wise product, inverse transform and recombination, all inside one
// workgroup, for transform lengths up to 2^16 (32-bit) / 2^15 (64-bit) residues.
//
// A product of transform length N = 2^(d+m) runs as 2^d sub-problems of length
// 2^m = S that fit in LDS (two operands of S words each).  Sub-problem h starts
// from the fold f_h[j] = sum_k x[j + k S] psi_h^k (the first d forward stages,
// restricted to block h; psi_h = w_{2^d}^([h]_d)), is transformed, multiplied and
// inverse-transformed in LDS, and its result is parked in registers.  The last d
// inverse stages then combine the 2^d partial results register-to-register (each
// thread holds the same positions j of every partial) and the linear product is
// written out.  One workgroup serves one product at a time; a launch loops over a
// descriptor list, so products of any prime and any length in the size class share
// one launch (section 2.2, Remark 6: several moduli in one vector launch).
#include "kernels.hpp"

namespace nttgpu {

template <typename T, bool LAZY, int NT, int LOGS, int MAXD>
__device__ void polymul_item(const FusedItem& it, T* sa, T* sb) {
  const PolyConst<T>* __restrict__ pc = (const PolyConst<T>*)it.cst;
  Arith<T> ar;
  ar.p = pc->p;
  ar.p2 = pc->p2;
  ar.pinv = pc->pinv;
  const TwPair<T>* __restrict__ tw = (const TwPair<T>*)it.tw;
  const TwPair<T>* __restrict__ twi = (const TwPair<T>*)it.twi;
  const T* __restrict__ a = (const T*)it.a;
  const T* __restrict__ b = (const T*)it.b;
  T* __restrict__ c = (T*)it.c;
  const int L = (int)it.log2n;
  const int m = L < LOGS ? L : LOGS;
  const int d = L - m;
  const int S = 1 << m;
  const int nsub = 1 << d;
  const uint64_t la = it.la, lb = it.lb, lc = la + lb - 1;
  constexpr int EPT = (1 << LOGS) / NT;
  T P0[MAXD > 0 ? EPT : 1], P1[MAXD > 1 ? EPT : 1], P2[MAXD > 1 ? EPT : 1];

  for (int h = 0; h < nsub; ++h) {
    // Fold of both operands (zero padding: indices >= la, lb read as 0); the
    // Montgomery scale 2^bits/N is applied to b here so that the entry-wise
    // Montgomery product yields a^ b^ / N.
    for (int j = threadIdx.x; j < S; j += NT) {
      T fa = 0, fb = 0;
      for (int k = 0; k < nsub; ++k) {
        const uint64_t idx = (uint64_t)j + (uint64_t)k * S;
        if (idx < la) {
          const T x = a[idx];
          const T t = k == 0 ? x : ar.red1(ar.shoup(x, pc->fa[h][k].w, pc->fa[h][k].ws));
          fa = ar.red1(fa + t);
        }
        if (idx < lb) {
          const T t = ar.red1(ar.shoup(b[idx], pc->fb[h][k].w, pc->fb[h][k].ws));
          fb = ar.red1(fb + t);
        }
      }
      sa[lidx(j)] = fa;
      sb[lidx(j)] = fb;
    }
    __syncthreads();
    fwd_lds<T, LAZY, NT, true>(ar, sa, sb, m, d, (uint32_t)h, tw);
    for (int j = threadIdx.x; j < S; j += NT) {
      T x = sa[lidx(j)], y = sb[lidx(j)];
      if constexpr (LAZY) {
        x = ar.red1(ar.red2(x));  // x < p, y < 4p: x y < 2^bits p
      } else {
        x = ar.red1(x);
        y = ar.red1(y);
      }
      T z = ar.mont(x, y);  // (0, 2p)
      if constexpr (!LAZY) z = ar.red1(z);
      sa[lidx(j)] = z;
    }
    __syncthreads();
    inv_lds<T, LAZY, NT>(ar, sa, m, d, (uint32_t)h, twi);
    if (h + 1 < nsub) {
      if constexpr (MAXD > 0) {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          const T v = sa[lidx((int)threadIdx.x + k * NT)];
          if (h == 0) P0[k] = v;
          else if (h == 1) P1[k] = v;
          else P2[k] = v;
        }
      }
    } else {
      // Recombination: inverse global stages d-1 .. 0 across the partial results.
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const int j = (int)threadIdx.x + k * NT;
        if (j < S) {
          T v0 = sa[lidx(j)];
          if (d == 0) {
            if ((uint64_t)j < lc) c[j] = canon_from_inv<LAZY>(ar, v0);
          } else if (d == 1) {
            if constexpr (MAXD > 0) {
              T x = P0[k];
              gs_bfly<LAZY>(ar, x, v0, twi[1]);
              if ((uint64_t)j < lc) c[j] = canon_from_inv<LAZY>(ar, x);
              if ((uint64_t)j + S < lc) c[j + S] = canon_from_inv<LAZY>(ar, v0);
            }
          } else {
            if constexpr (MAXD > 1) {
              T x0 = P0[k], x1 = P1[k], x2 = P2[k], x3 = v0;
              const TwPair<T> w1 = twi[1], w2 = twi[2], w3 = twi[3];
              gs_bfly<LAZY>(ar, x0, x1, w2);
              gs_bfly<LAZY>(ar, x2, x3, w3);
              gs_bfly<LAZY>(ar, x0, x2, w1);
              gs_bfly<LAZY>(ar, x1, x3, w1);
              const uint64_t jj = (uint64_t)j;
              if (jj < lc) c[jj] = canon_from_inv<LAZY>(ar, x0);
              if (jj + S < lc) c[jj + S] = canon_from_inv<LAZY>(ar, x1);
              if (jj + 2 * (uint64_t)S < lc) c[jj + 2 * (uint64_t)S] = canon_from_inv<LAZY>(ar, x2);
              if (jj + 3 * (uint64_t)S < lc) c[jj + 3 * (uint64_t)S] = canon_from_inv<LAZY>(ar, x3);
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

// Persistent over the item list: workgroup w serves items w, w + G, w + 2G, ...
template <typename T, int NT, int LOGS, int MAXD>
__global__ __launch_bounds__(NT) void polymul_fused_kernel(FusedBatch batch) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sa = (T*)smem_raw;
  T* sb = sa + lds_words(1 << LOGS);
  for (int i = blockIdx.x; i < batch.count; i += gridDim.x) {
    const FusedItem it = batch.items ? batch.items[i] : batch.single;
    const PolyConst<T>* pc = (const PolyConst<T>*)it.cst;
    if (pc->lazy) polymul_item<T, true, NT, LOGS, MAXD>(it, sa, sb);
    else polymul_item<T, false, NT, LOGS, MAXD>(it, sa, sb);
  }
}

template <typename T, int NT, int LOGS, int MAXD>
static hipError_t launch_fused_cls(const FusedBatch& batch, int grid, hipStream_t stream) {
  const size_t lds = 2 * (size_t)lds_words(1 << LOGS) * sizeof(T);
  auto k = polymul_fused_kernel<T, NT, LOGS, MAXD>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(grid), dim3(NT), lds, stream, batch);
  return hipGetLastError();
}

// Size classes: the class fixes the workgroup size and the LDS sub-problem size.
int fused_class(int word_bits, int log2n) {
  if (word_bits == 32) {
    if (log2n <= 10) return 0;
    if (log2n <= 12) return 1;
    if (log2n <= 13) return 2;
    if (log2n <= 16) return 3;
    return -1;
  }
  if (log2n <= 10) return 0;
  if (log2n <= 12) return 1;
  if (log2n <= 15) return 3;
  return -1;
}

int fused_max_log2n(int word_bits) { return word_bits == 32 ? 16 : 15; }

hipError_t launch_fused(int word_bits, int cls, const FusedBatch& batch, int grid, hipStream_t stream) {
  if (word_bits == 32) {
    switch (cls) {
      case 0: return launch_fused_cls<uint32_t, 64, 10, 0>(batch, grid, stream);
      case 1: return launch_fused_cls<uint32_t, 256, 12, 0>(batch, grid, stream);
      case 2: return launch_fused_cls<uint32_t, 512, 13, 0>(batch, grid, stream);
      case 3: return launch_fused_cls<uint32_t, 1024, 14, 2>(batch, grid, stream);
    }
  } else {
    switch (cls) {
      case 0: return launch_fused_cls<uint64_t, 64, 10, 0>(batch, grid, stream);
      case 1: return launch_fused_cls<uint64_t, 256, 12, 0>(batch, grid, stream);
      case 3: return launch_fused_cls<uint64_t, 1024, 13, 2>(batch, grid, stream);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace nttgpu
