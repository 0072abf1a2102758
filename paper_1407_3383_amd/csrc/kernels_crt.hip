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
//      left is 0 or 1 (generate: t_m >= 2^16, propagate: t_m = 2^16 - 1);
//   2. a scan of the per-block (generate, propagate) pairs gives each block's carry in;
//   3. each block scans its own positions and packs pairs of 16-bit limbs.
#include "kernels.hpp"

namespace nttgpu {

constexpr int kCrtNT = 256;
constexpr int kCrtPPT = 8;                        // positions per thread
constexpr int kCrtBlock = kCrtNT * kCrtPPT;       // positions per workgroup

int crt_block_positions() { return kCrtBlock; }

__device__ __forceinline__ uint32_t shoup32(uint32_t x, uint32_t w, uint32_t ws, uint32_t p) {
  uint32_t q = __umulhi(x, ws);
  uint32_t r = x * w - q * p;
  return min(r, r - p);
}

__device__ __forceinline__ uint64_t garner(const CrtArgs& A, uint64_t k) {
  if (k >= A.lc) return 0;
  const uint32_t p1 = A.p1, p2 = A.p2, p3 = A.p3;
  const uint32_t x1 = A.r1[k];
  uint32_t x1m2 = x1;  // x1 < p1 < 4 p2 reduced below p2
  while (x1m2 >= p2) x1m2 -= p2;
  uint32_t d2 = A.r2[k] + p2 - x1m2;
  d2 = min(d2, d2 - p2);
  const uint32_t x2 = shoup32(d2, A.c12, A.c12s, p2);
  uint32_t x1m3 = x1;
  while (x1m3 >= p3) x1m3 -= p3;
  uint32_t x2m3 = x2;
  while (x2m3 >= p3) x2m3 -= p3;
  const uint32_t t = shoup32(x2m3, A.p1m3, A.p1m3s, p3);  // x2 p1 mod p3
  uint32_t d3 = A.r3[k] + p3 - x1m3;
  d3 = min(d3, d3 - p3);
  d3 = d3 + p3 - t;
  d3 = min(d3, d3 - p3);
  const uint32_t x3 = shoup32(d3, A.c123, A.c123s, p3);
  return (uint64_t)x1 + (uint64_t)p1 * x2 + A.p1p2 * (uint64_t)x3;
}

// s_m for m in [m0 - 1, m0 + PPT): needs v_(m0-4) .. v_(m0+PPT-1).
__device__ __forceinline__ void column_sums(const CrtArgs& A, uint64_t m0, uint32_t (&t)[kCrtPPT]) {
  uint64_t v[kCrtPPT + 4];
#pragma unroll
  for (int i = 0; i < kCrtPPT + 4; ++i) {
    const int64_t k = (int64_t)m0 - 4 + i;
    v[i] = k >= 0 ? garner(A, (uint64_t)k) : 0;
  }
  uint32_t s[kCrtPPT + 1];
#pragma unroll
  for (int q = 0; q <= kCrtPPT; ++q) {
    // position m = m0 - 1 + q  ->  v index (m - i) - (m0 - 4) = q + 3 - i
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) acc += (uint32_t)((v[q + 3 - i] >> (16 * i)) & 0xFFFF);
    s[q] = (m0 == 0 && q == 0) ? 0u : acc;
  }
#pragma unroll
  for (int q = 0; q < kCrtPPT; ++q) t[q] = (s[q + 1] & 0xFFFF) + (s[q] >> 16);
}

// Carry status of a run: 0 = kill (carry out 0), 1 = generate (1), 2 = propagate.
__device__ __forceinline__ uint32_t gp_of(uint32_t t) { return t >= 0x10000u ? 1u : (t == 0xFFFFu ? 2u : 0u); }
__device__ __forceinline__ uint32_t gp_combine(uint32_t lo, uint32_t hi) { return hi == 2u ? lo : hi; }

__global__ __launch_bounds__(kCrtNT) void crt_phase1_kernel(CrtArgs A) {
  __shared__ uint32_t red[kCrtNT];
  const uint64_t m0 = (uint64_t)blockIdx.x * kCrtBlock + (uint64_t)threadIdx.x * kCrtPPT;
  uint32_t t[kCrtPPT];
  column_sums(A, m0, t);
  uint32_t g = 2u;
#pragma unroll
  for (int q = 0; q < kCrtPPT; ++q) {
    const uint64_t m = m0 + q;
    if (m < A.npos) {
      A.t[m] = t[q];
      g = gp_combine(g, gp_of(t[q]));
    }
  }
  red[threadIdx.x] = g;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 2u;
    for (int i = 0; i < kCrtNT; ++i) acc = gp_combine(acc, red[i]);
    A.blk[blockIdx.x] = acc;
  }
}

// One workgroup turns the per-block statuses into carry-in bits (exclusive scan).
__global__ __launch_bounds__(1024) void crt_phase2_kernel(CrtArgs A, uint32_t nblk) {
  __shared__ uint32_t sh[1024];
  const uint32_t per = (nblk + 1023) / 1024;
  const uint32_t b0 = threadIdx.x * per;
  uint32_t acc = 2u;
  for (uint32_t i = 0; i < per; ++i)
    if (b0 + i < nblk) acc = gp_combine(acc, A.blk[b0 + i]);
  sh[threadIdx.x] = acc;
  __syncthreads();
  // inclusive Hillis-Steele scan of the thread summaries
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = sh[threadIdx.x];
    uint32_t lo = threadIdx.x >= (uint32_t)off ? sh[threadIdx.x - off] : 2u;
    __syncthreads();
    sh[threadIdx.x] = gp_combine(lo, v);
    __syncthreads();
  }
  uint32_t carry = threadIdx.x == 0 ? 0u : (sh[threadIdx.x - 1] == 1u ? 1u : 0u);
  __syncthreads();
  for (uint32_t i = 0; i < per; ++i) {
    if (b0 + i < nblk) {
      const uint32_t st = A.blk[b0 + i];
      A.blk[b0 + i] = carry;
      carry = st == 2u ? carry : (st == 1u ? 1u : 0u);
    }
  }
}

__global__ __launch_bounds__(kCrtNT) void crt_phase3_kernel(CrtArgs A) {
  __shared__ uint32_t sh[kCrtNT];
  const uint64_t m0 = (uint64_t)blockIdx.x * kCrtBlock + (uint64_t)threadIdx.x * kCrtPPT;
  uint32_t t[kCrtPPT];
  uint32_t g = 2u;
#pragma unroll
  for (int q = 0; q < kCrtPPT; ++q) {
    const uint64_t m = m0 + q;
    t[q] = m < A.npos ? A.t[m] : 0u;
    g = gp_combine(g, gp_of(t[q]));
  }
  sh[threadIdx.x] = g;
  __syncthreads();
  for (int off = 1; off < kCrtNT; off <<= 1) {
    uint32_t v = sh[threadIdx.x];
    uint32_t lo = threadIdx.x >= (uint32_t)off ? sh[threadIdx.x - off] : 2u;
    __syncthreads();
    sh[threadIdx.x] = gp_combine(lo, v);
    __syncthreads();
  }
  const uint32_t cin_blk = A.blk[blockIdx.x];
  uint32_t carry;
  if (threadIdx.x == 0) {
    carry = cin_blk;
  } else {
    const uint32_t st = sh[threadIdx.x - 1];
    carry = st == 2u ? cin_blk : (st == 1u ? 1u : 0u);
  }
  uint32_t limb16[kCrtPPT];
#pragma unroll
  for (int q = 0; q < kCrtPPT; ++q) {
    const uint32_t x = t[q] + carry;
    limb16[q] = x & 0xFFFFu;
    carry = x >> 16;
  }
#pragma unroll
  for (int q = 0; q < kCrtPPT; q += 2) {
    const uint64_t m = m0 + q;
    if (m < A.npos) A.c[m >> 1] = limb16[q] | (limb16[q + 1] << 16);
  }
}

hipError_t launch_crt_carry(const CrtArgs& a, hipStream_t stream) {
  const uint64_t nblk = (a.npos + kCrtBlock - 1) / kCrtBlock;
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(crt_phase1_kernel, dim3((unsigned)nblk), dim3(kCrtNT), 0, stream, a);
  hipLaunchKernelGGL(crt_phase2_kernel, dim3(1), dim3(1024), 0, stream, a, (uint32_t)nblk);
  hipLaunchKernelGGL(crt_phase3_kernel, dim3((unsigned)nblk), dim3(kCrtNT), 0, stream, a);
  return hipGetLastError();
}

}  // namespace nttgpu
