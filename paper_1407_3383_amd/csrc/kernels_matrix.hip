// Polynomial matrix product (section 5.2): after the forward transforms of every entry
// of A and B, the product at each frequency k is an n x n matrix product over F_p,
// C^(k) = A^(k) B^(k); the inverse transforms of C's entries then give C = A B.
//
// freq_matmul_kernel: one workgroup owns KB consecutive frequencies.  It stages those
// frequencies of every entry of A and B in LDS (entry-major, KB words per entry), then
// each work item -- one frequency and one 4 x 4 tile of C -- accumulates its 16 sums of
// n products in 64-bit registers (one v_mad_u64_u32 per product).  A tile takes rows
// ib + S t and columns jb + S t (S = ceil(n / 4)), so that neighbouring tiles in a wave
// read neighbouring entries of B (different LDS banks) and the same entries of A (one
// broadcast).  Every `fold` products the sums are folded, s = hi 2^32 + lo ->
// hi (2^32 mod p) + lo < p 2^32, which keeps them below 2^64; at the end one Montgomery
// reduction (Function 13, m = 32) and one product by a constant K (Function 8) give
// s 2^-32 K mod p: K = 2^32 / N when the inverse transforms do not scale by 1/N, and
// K = 2^32 when they do.  C may alias A: a workgroup writes only the frequencies it has
// already staged.
#include "kernels.hpp"

namespace nttgpu {

namespace {

constexpr int kMatThreads = 256;

__global__ __launch_bounds__(kMatThreads) void freq_matmul_kernel(MatArgs M) {
  extern __shared__ __align__(16) uint32_t mat_lds[];
  const uint32_t n = M.n, KB = M.kb, n2 = n * n;
  const uint64_t N = M.N;
  const uint64_t k0 = (uint64_t)blockIdx.x * KB;
  uint32_t* As = mat_lds;
  uint32_t* Bs = mat_lds + (size_t)n2 * KB;
  const uint32_t tid = threadIdx.x;
  if (KB >= 4) {
    const uint32_t q = KB >> 2;
    for (uint32_t idx = tid; idx < n2 * q; idx += kMatThreads) {
      const uint32_t e = idx / q, c = (idx - e * q) << 2;
      const uint64_t g = (uint64_t)e * N + k0 + c;
      *(uint4*)(As + (size_t)e * KB + c) = *(const uint4*)(M.A + g);
      *(uint4*)(Bs + (size_t)e * KB + c) = *(const uint4*)(M.B + g);
    }
  } else {
    for (uint32_t idx = tid; idx < n2 * KB; idx += kMatThreads) {
      const uint32_t e = idx / KB, c = idx - e * KB;
      const uint64_t g = (uint64_t)e * N + k0 + c;
      As[idx] = M.A[g];
      Bs[idx] = M.B[g];
    }
  }
  __syncthreads();
  const uint32_t p = M.p, S = (n + 3) >> 2;
  const uint32_t items = S * S * KB;
  for (uint32_t w = tid; w < items; w += kMatThreads) {
    const uint32_t t = w / KB, kk = w - t * KB;
    const uint32_t ib = t / S, jb = t - ib * S;
    uint64_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = 0;
    for (uint32_t l0 = 0; l0 < n; l0 += M.fold) {
      const uint32_t l1 = min(n, l0 + M.fold);
#pragma unroll 2
      for (uint32_t l = l0; l < l1; ++l) {
        uint32_t x[4], y[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const uint32_t i = ib + S * a;
          x[a] = i < n ? As[(size_t)(i * n + l) * KB + kk] : 0u;
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const uint32_t j = jb + S * b;
          y[b] = j < n ? Bs[(size_t)(l * n + j) * KB + kk] : 0u;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] += (uint64_t)x[a] * y[b];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = (uint64_t)(uint32_t)(acc[a][b] >> 32) * M.r32 + (uint32_t)acc[a][b];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const uint32_t i = ib + S * a;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint32_t j = jb + S * b;
        if (i < n && j < n) {
          const uint64_t s = acc[a][b];
          const uint32_t m = (uint32_t)s * M.pinv;
          uint32_t r = (uint32_t)(s >> 32) - __umulhi(m, p) + p;  // s 2^-32 mod p, in (0, 2p)
          r = min(r, r - p);
          const uint32_t q = __umulhi(r, M.kws);
          r = r * M.kw - q * p;  // r K mod p, in [0, 2p)
          r = min(r, r - p);
          M.C[(uint64_t)(i * n + j) * N + k0 + kk] = r;
        }
      }
    }
  }
}

__global__ void copy_rows_kernel(uint32_t* dst, uint64_t dst_stride, uint64_t dst_len, const uint32_t* src,
                                 uint64_t src_stride, uint64_t src_len, uint32_t rows) {
  const uint64_t total = (uint64_t)rows * dst_len;
  for (uint64_t idx = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t r = idx / dst_len, t = idx - r * dst_len;
    dst[r * dst_stride + t] = t < src_len ? src[r * src_stride + t] : 0u;
  }
}

}  // namespace

uint32_t freq_matmul_block(uint32_t n, uint64_t N) {
  if (n == 0 || n > kMatMaxN) return 0;
  uint32_t kb = 256;
  while (kb > 1 && (uint64_t)n * n * kb > 8192) kb >>= 1;
  while ((uint64_t)kb > N) kb >>= 1;
  return kb;
}

hipError_t launch_freq_matmul(const MatArgs& a, hipStream_t stream) {
  if (a.n == 0 || a.n > kMatMaxN || a.kb == 0 || (a.N % a.kb) != 0 || a.fold == 0) return hipErrorInvalidValue;
  if (a.kb >= 4 && (((uintptr_t)a.A | (uintptr_t)a.B) & 15u)) return hipErrorInvalidValue;
  const size_t lds = 2 * (size_t)a.n * a.n * a.kb * sizeof(uint32_t);
  hipError_t e = allow_dynamic_lds((const void*)freq_matmul_kernel, lds);
  if (e != hipSuccess) return e;
  const uint64_t grid = a.N / a.kb;
  if (grid > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(freq_matmul_kernel, dim3((uint32_t)grid), dim3(kMatThreads), lds, stream, a);
  return hipGetLastError();
}

hipError_t launch_copy_rows(uint32_t* dst, uint64_t dst_stride, uint64_t dst_len, const uint32_t* src,
                            uint64_t src_stride, uint64_t src_len, uint32_t rows, hipStream_t stream) {
  const uint64_t total = (uint64_t)rows * dst_len;
  if (total == 0) return hipSuccess;
  const uint64_t blocks = (total + 255) / 256;
  const uint32_t grid = (uint32_t)(blocks < 8192 ? blocks : 8192);
  hipLaunchKernelGGL(copy_rows_kernel, dim3(grid), dim3(256), 0, stream, dst, dst_stride, dst_len, src, src_stride,
                     src_len, rows);
  return hipGetLastError();
}

}  // namespace nttgpu
