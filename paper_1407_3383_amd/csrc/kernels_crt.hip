// Integer product tail (section 5.3): Chinese remaindering of the three residue
// products and carry propagation of C(2^16) into 32-bit limbs.
//
// Garner's mixed-radix form per coefficient k:
//   x1 = r1, x2 = (r2 - x1) p1^-1 mod p2, x3 = (r3 - x1 - x2 p1) (p1 p2)^-1 mod p3,
//   v_k = x1 + p1 x2 + p1 p2 x3,
// computed exactly in 64 bits (the host only launches when every coefficient is
// below 2^64).  The number C = sum_k v_k 2^(16 k) is then normalised in three steps:
//   1. column sums over 16-bit positions m: s_m = sum_i digit_i(v_(m-i)) < 2^18,
//      and t_m = (s_m mod 2^16) + floor(s_(m-1) / 2^16) <= 2^16 + 3, so every carry
//      left is 0 or 1: position m generates one (t_m >= 2^16), propagates the one
//      it receives (t_m = 2^16 - 1) or kills it (otherwise);
//   2. the carry into a block is decided by the nearest block below it that does not
//      propagate: a prefix maximum of keys 2 (b + 1) + generate over such blocks;
//   3. inside a block the same prefix maximum over positions gives each position's
//      carry in, and pairs of 16-bit limbs are packed.
#include "kernels.hpp"

namespace nttgpu {

constexpr int kCrtNT = 256;
constexpr int kCrtPPT = 8;                   // positions per thread
constexpr int kCrtBlock = kCrtNT * kCrtPPT;  // positions per workgroup
constexpr int kCrtHalo = 4;                  // coefficients below the block that reach into it

int crt_block_positions() { return kCrtBlock; }

// Function 8 with the final correction left out: [0, 2p) for any 32-bit x.
__device__ __forceinline__ uint32_t shoup_lazy(uint32_t x, uint32_t w, uint32_t ws, uint32_t p) {
  return x * w - __umulhi(x, ws) * p;
}
__device__ __forceinline__ uint32_t red(uint32_t x, uint32_t p) { return min(x, x - p); }

// v_k from the three residues; no reduction of x1 or x2 is needed first, because
// every Shoup input below stays under 2^32:
//   r2 + 3 p2 - x1          with x1 < p1 < 3 p2
//   r3 + 8 p3 - x1 - u      with x1 < p1 < 6 p3 and u = x2 p1 mod p3 in [0, 2 p3)
__device__ __forceinline__ uint64_t garner(const CrtArgs& A, uint32_t r1, uint32_t r2, uint32_t r3) {
  const uint32_t x1 = r1;
  const uint32_t x2 = red(shoup_lazy(r2 + 3u * A.p2 - x1, A.c12, A.c12s, A.p2), A.p2);
  const uint32_t u = shoup_lazy(x2, A.p1m3, A.p1m3s, A.p3);
  const uint32_t x3 = red(shoup_lazy(r3 + 8u * A.p3 - x1 - u, A.c123, A.c123s, A.p3), A.p3);
  return (uint64_t)x1 + (uint64_t)A.p1 * x2 + A.p1p2 * (uint64_t)x3;
}

__device__ __forceinline__ uint32_t digit(uint64_t v, int i) { return (uint32_t)(v >> (16 * i)) & 0xFFFFu; }

// Inclusive prefix maximum across a wave.
__device__ __forceinline__ uint32_t wave_scan_max(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)x, off, 64);
    if (lane >= off) x = max(x, y);
  }
  return x;
}
__device__ __forceinline__ uint32_t wave_max(uint32_t x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, off, 64));
  return x;
}

// Key of a non-propagating run ending at local position j: 2 (j + 1) + generate.
__device__ __forceinline__ uint32_t pos_key(uint32_t t, uint32_t j) {
  return t == 0xFFFFu ? 0u : 2u * (j + 1u) + (t >= 0x10000u ? 1u : 0u);
}

// Phase 1: Garner values of the block's coefficients (plus the 4-coefficient halo
// below it) staged once in LDS, column sums t_m for the block's positions (stored
// for all positions of the block: they are 0 above the product), block status.
__global__ __launch_bounds__(kCrtNT) void crt_phase1_kernel(CrtArgs A) {
  __shared__ uint64_t v[kCrtBlock + kCrtHalo];
  __shared__ uint32_t wmax[kCrtNT / 64];
  const uint64_t mb = (uint64_t)blockIdx.x * kCrtBlock;
  gcptr<uint32_t> r1 = gconst<uint32_t>(A.r1);
  gcptr<uint32_t> r2 = gconst<uint32_t>(A.r2);
  gcptr<uint32_t> r3 = gconst<uint32_t>(A.r3);
  // local index j <-> coefficient mb - 4 + j
  for (int j = threadIdx.x; j < kCrtBlock + kCrtHalo; j += kCrtNT) {
    const int64_t k = (int64_t)mb - kCrtHalo + j;
    uint64_t x = 0;
    if (k >= 0 && (uint64_t)k < A.lc) x = garner(A, r1[k], r2[k], r3[k]);
    v[j] = x;
  }
  __syncthreads();
  uint32_t key = 0;
  gptr<uint32_t> t = gmut<uint32_t>(A.t);
#pragma unroll
  for (int q = 0; q < kCrtPPT; ++q) {
    const int lp = threadIdx.x + kCrtNT * q;  // position mb + lp uses v at local lp .. lp + 4
    const uint64_t v0 = v[lp], v1 = v[lp + 1], v2 = v[lp + 2], v3 = v[lp + 3], v4 = v[lp + 4];
    const uint32_t s = digit(v4, 0) + digit(v3, 1) + digit(v2, 2) + digit(v1, 3);       // s_m
    const uint32_t sp = digit(v3, 0) + digit(v2, 1) + digit(v1, 2) + digit(v0, 3);      // s_(m-1)
    const uint32_t tm = (s & 0xFFFFu) + (sp >> 16);
    t[mb + lp] = tm;
    key = max(key, pos_key(tm, (uint32_t)lp));
  }
  key = wave_max(key);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = key;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t k = 0;
#pragma unroll
    for (int w = 0; w < kCrtNT / 64; ++w) k = max(k, wmax[w]);
    // 0 kill, 1 generate, 2 propagate
    gmut<uint32_t>(A.blk)[blockIdx.x] = k == 0 ? 2u : (k & 1u);
  }
}

// Phase 2 (one workgroup): block statuses -> carry into each block.
__global__ __launch_bounds__(1024) void crt_phase2_kernel(CrtArgs A, uint32_t nblk) {
  __shared__ uint32_t wsum[16];
  gptr<uint32_t> blk = gmut<uint32_t>(A.blk) + (uint64_t)blockIdx.y * A.bstride;
  const uint32_t per = (nblk + 1023) / 1024;  // at most 8: the host caps nblk at 8192
  const uint32_t b0 = threadIdx.x * per;
  uint32_t st[8];
  uint32_t key = 0;
#pragma unroll
  for (uint32_t i = 0; i < 8; ++i) {
    st[i] = 2u;
    if (i < per && b0 + i < nblk) {
      st[i] = blk[b0 + i];
      if (st[i] != 2u) key = 2u * (b0 + i + 1u) + st[i];
    }
  }
  const uint32_t incl = wave_scan_max(key);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t below = 0;
  for (int i = 0; i < w; ++i) below = max(below, wsum[i]);
  const uint32_t up = (uint32_t)__shfl_up((int)incl, 1, 64);
  uint32_t excl = max(below, lane > 0 ? up : 0u);
#pragma unroll
  for (uint32_t i = 0; i < 8; ++i) {
    if (i < per && b0 + i < nblk) {
      blk[b0 + i] = excl & 1u;  // carry in: generate bit of the nearest non-propagating block below
      if (st[i] != 2u) excl = 2u * (b0 + i + 1u) + st[i];
    }
  }
}

// Phase 3: carry into each position from the in-block prefix maximum and the block's
// carry in, then 16-bit limbs packed in pairs.
__global__ __launch_bounds__(kCrtNT) void crt_phase3_kernel(CrtArgs A) {
  __shared__ uint32_t wsum[kCrtNT / 64];
  const uint64_t mb = (uint64_t)blockIdx.x * kCrtBlock;
  const uint32_t lp0 = threadIdx.x * kCrtPPT;
  const uint4* tv = (const uint4*)(A.t + mb + lp0);  // the workspace holds whole blocks
  const uint4 ta = tv[0], tb = tv[1];
  const uint32_t t[kCrtPPT] = {ta.x, ta.y, ta.z, ta.w, tb.x, tb.y, tb.z, tb.w};
  uint32_t key = 0;
#pragma unroll
  for (int q = 0; q < kCrtPPT; ++q) key = max(key, pos_key(t[q], lp0 + q));
  const uint32_t incl = wave_scan_max(key);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t below = 0;
  for (int i = 0; i < w; ++i) below = max(below, wsum[i]);
  const uint32_t up = (uint32_t)__shfl_up((int)incl, 1, 64);
  const uint32_t excl = max(below, lane > 0 ? up : 0u);
  uint32_t carry = excl == 0 ? gconst<uint32_t>(A.blk)[blockIdx.x] : (excl & 1u);
  uint32_t limb[kCrtPPT];
#pragma unroll
  for (int q = 0; q < kCrtPPT; ++q) {
    const uint32_t x = t[q] + carry;
    limb[q] = x & 0xFFFFu;
    carry = x >> 16;
  }
  gptr<uint32_t> c = gmut<uint32_t>(A.c);
#pragma unroll
  for (int q = 0; q < kCrtPPT; q += 2) {
    const uint64_t m = mb + lp0 + q;
    if (m < A.npos) c[m >> 1] = limb[q] | (limb[q + 1] << 16);
  }
}

hipError_t launch_crt_carry(const CrtArgs& a, hipStream_t stream) {
  const uint64_t nblk = (a.npos + kCrtBlock - 1) / kCrtBlock;
  if (nblk == 0) return hipSuccess;
  if (nblk > 8192) return hipErrorInvalidValue;
  hipLaunchKernelGGL(crt_phase1_kernel, dim3((unsigned)nblk), dim3(kCrtNT), 0, stream, a);
  hipLaunchKernelGGL(crt_phase2_kernel, dim3(1), dim3(1024), 0, stream, a, (uint32_t)nblk);
  hipLaunchKernelGGL(crt_phase3_kernel, dim3((unsigned)nblk), dim3(kCrtNT), 0, stream, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ 32-bit chunks
// The same tail for chunks of h = 32 bits (section 5.3's choice of h for these
// primes): v_k < p1 p2 p3 < 2^87 takes three 32-bit digits, the column sum of
// position m is s_m = d0(v_m) + d1(v_(m-1)) + d2(v_(m-2)) < 3 2^32, and
// t_m = (s_m mod 2^32) + floor(s_(m-1) / 2^32) <= 2^32 + 1 leaves carries of 0 or 1
// again, resolved by the same prefix maxima; the limbs are t_m + carry mod 2^32.
constexpr int kCrt32Halo = 3;  // s_(m-1) reaches v_(m-3)

namespace {

// v = x1 + p1 x2 + p1 p2 x3 as (lo 64 bits, hi 32 bits).
__device__ __forceinline__ void garner96(const CrtArgs& A, uint32_t r1, uint32_t r2, uint32_t r3, uint64_t& lo,
                                         uint32_t& hi) {
  const uint32_t x1 = r1;
  const uint32_t x2 = red(shoup_lazy(r2 + 3u * A.p2 - x1, A.c12, A.c12s, A.p2), A.p2);
  const uint32_t u = shoup_lazy(x2, A.p1m3, A.p1m3s, A.p3);
  const uint32_t x3 = red(shoup_lazy(r3 + 8u * A.p3 - x1 - u, A.c123, A.c123s, A.p3), A.p3);
  const uint64_t s = (uint64_t)x1 + (uint64_t)A.p1 * x2;  // < 2^60
  const uint64_t bl = A.p1p2 * (uint64_t)x3;
  const uint64_t bh = __umul64hi(A.p1p2, (uint64_t)x3);
  lo = s + bl;
  hi = (uint32_t)(bh + (lo < s ? 1u : 0u));
}

__device__ __forceinline__ uint32_t key32(uint64_t t, uint32_t j) {
  return t == 0xFFFFFFFFull ? 0u : 2u * (j + 1u) + (t >= (1ull << 32) ? 1u : 0u);
}

}  // namespace

__global__ __launch_bounds__(kCrtNT) void crt32_phase1_kernel(CrtArgs A) {
  __shared__ uint64_t vlo[kCrtBlock + kCrt32Halo];
  __shared__ uint32_t vhi[kCrtBlock + kCrt32Halo];
  __shared__ uint32_t wmax[kCrtNT / 64];
  const uint64_t mb = (uint64_t)blockIdx.x * kCrtBlock;
  const uint64_t e = blockIdx.y;
  gcptr<uint32_t> r1 = gconst<uint32_t>(A.r1) + e * A.rstride;
  gcptr<uint32_t> r2 = gconst<uint32_t>(A.r2) + e * A.rstride;
  gcptr<uint32_t> r3 = gconst<uint32_t>(A.r3) + e * A.rstride;
  for (int j = threadIdx.x; j < kCrtBlock + kCrt32Halo; j += kCrtNT) {
    const int64_t k = (int64_t)mb - kCrt32Halo + j;
    uint64_t lo = 0;
    uint32_t hi = 0;
    if (k >= 0 && (uint64_t)k < A.lc) garner96(A, r1[k], r2[k], r3[k], lo, hi);
    vlo[j] = lo;
    vhi[j] = hi;
  }
  __syncthreads();
  uint32_t key = 0;
  gptr<uint64_t> t = gmut<uint64_t>(A.t) + e * A.tstride;
#pragma unroll
  for (int q = 0; q < kCrtPPT; ++q) {
    const int lp = threadIdx.x + kCrtNT * q;  // position mb + lp: v_(m-i) at local lp + 3 - i
    const uint64_t s = (vlo[lp + 3] & 0xFFFFFFFFull) + (vlo[lp + 2] >> 32) + (uint64_t)vhi[lp + 1];   // s_m
    const uint64_t sp = (vlo[lp + 2] & 0xFFFFFFFFull) + (vlo[lp + 1] >> 32) + (uint64_t)vhi[lp];     // s_(m-1)
    const uint64_t tm = (s & 0xFFFFFFFFull) + (sp >> 32);
    t[mb + lp] = tm;
    key = max(key, key32(tm, (uint32_t)lp));
  }
  key = wave_max(key);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = key;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t k = 0;
#pragma unroll
    for (int w = 0; w < kCrtNT / 64; ++w) k = max(k, wmax[w]);
    gmut<uint32_t>(A.blk)[e * A.bstride + blockIdx.x] = k == 0 ? 2u : (k & 1u);
  }
}

__global__ __launch_bounds__(kCrtNT) void crt32_phase3_kernel(CrtArgs A) {
  __shared__ uint32_t wsum[kCrtNT / 64];
  const uint64_t mb = (uint64_t)blockIdx.x * kCrtBlock;
  const uint64_t e = blockIdx.y;
  const uint32_t lp0 = threadIdx.x * kCrtPPT;
  const uint64_t* tv = (const uint64_t*)A.t + e * A.tstride + mb + lp0;  // the workspace holds whole blocks
  uint64_t t[kCrtPPT];
#pragma unroll
  for (int q = 0; q < kCrtPPT; ++q) t[q] = tv[q];
  uint32_t key = 0;
#pragma unroll
  for (int q = 0; q < kCrtPPT; ++q) key = max(key, key32(t[q], lp0 + q));
  const uint32_t incl = wave_scan_max(key);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t below = 0;
  for (int i = 0; i < w; ++i) below = max(below, wsum[i]);
  const uint32_t up = (uint32_t)__shfl_up((int)incl, 1, 64);
  const uint32_t excl = max(below, lane > 0 ? up : 0u);
  uint64_t carry = excl == 0 ? gconst<uint32_t>(A.blk)[e * A.bstride + blockIdx.x] : (excl & 1u);
  gptr<uint32_t> c = gmut<uint32_t>(A.c) + e * A.cstride;
#pragma unroll
  for (int q = 0; q < kCrtPPT; ++q) {
    const uint64_t x = t[q] + carry;
    const uint64_t m = mb + lp0 + q;
    if (m < A.npos) c[m] = (uint32_t)x;
    carry = x >> 32;
  }
}

hipError_t launch_crt32_carry(const CrtArgs& a, hipStream_t stream) {
  const uint64_t nblk = (a.npos + kCrtBlock - 1) / kCrtBlock;
  if (nblk == 0) return hipSuccess;
  if (nblk > 8192) return hipErrorInvalidValue;
  const uint32_t batch = a.batch > 1 ? a.batch : 1u;
  if (batch > 65535) return hipErrorInvalidValue;
  if (batch > 1 && (a.tstride < nblk * kCrtBlock || a.bstride < nblk || a.cstride < a.npos || a.rstride < a.lc))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(crt32_phase1_kernel, dim3((unsigned)nblk, batch), dim3(kCrtNT), 0, stream, a);
  hipLaunchKernelGGL(crt_phase2_kernel, dim3(1, batch), dim3(1024), 0, stream, a, (uint32_t)nblk);
  hipLaunchKernelGGL(crt32_phase3_kernel, dim3((unsigned)nblk, batch), dim3(kCrtNT), 0, stream, a);
  return hipGetLastError();
}

// out[i] = in[i] mod p for 32-bit words: Function 8 with y = 1 (psi = floor(2^32 / p))
// gives [0, 2p) for any word, one min finishes.
__global__ void reduce_mod_kernel(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, uint64_t n, uint32_t p,
                                  uint32_t psi) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t x = in[i];
    out[i] = red(x - __umulhi(x, psi) * p, p);
  }
}

hipError_t launch_reduce_mod(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t p, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint32_t psi = (uint32_t)((1ull << 32) / p);
  const int grid = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(reduce_mod_kernel, dim3(grid), dim3(256), 0, stream, in, out, n, p, psi);
  return hipGetLastError();
}

}  // namespace nttgpu
