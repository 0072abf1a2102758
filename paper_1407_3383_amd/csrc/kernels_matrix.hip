// Polynomial matrix product (section 5.2): after the forward transforms of every entry
// of A and B, the product at each frequency k is an n x n matrix product over F_p,
// C^(k) = A^(k) B^(k); the inverse transforms of C's entries then give C = A B.
//
// freq_matmul_kernel: one workgroup owns KB consecutive frequencies.  It stages those
// frequencies of every entry of A (by rows) and B (by columns) in LDS, then each work
// item -- one frequency and one 4 x 4 tile of C -- accumulates its 16 sums of n
// products in 64-bit registers (one v_mad_u64_u32 per product).  A tile takes rows
// ib + S t and columns jb + S t (S = ceil(n / 4)), so that neighbouring tiles in a wave
// read neighbouring columns of B (different LDS banks, by the row padding) and the same
// row of A (one broadcast).  Every `fold` products the sums are folded, s = hi 2^32 + lo ->
// hi (2^32 mod p) + lo < p 2^32, which keeps them below 2^64; at the end one Montgomery
// reduction (Function 13, m = 32) and one product by a constant K (Function 8) give
// s 2^-32 K mod p: K = 2^32 / N when the inverse transforms do not scale by 1/N, and
// K = 2^32 when they do.  C may alias A: a workgroup writes only the frequencies it has
// already staged.
#include "kernels.hpp"

namespace nttgpu {

namespace {

constexpr int kMatThreads = 512;

// LDS layout, RS = (n + 1) KB words per matrix row: As[i RS + l KB + kk] = A[i][l] and
// Bt[j RS + l KB + kk] = B[l][j] at frequency k0 + kk.  Consecutive l are KB words
// apart in both (immediate offsets once the l loop is unrolled); the KB padding words
// per row put neighbouring rows of a wave's tiles on different banks.
template <int KB>
__global__ __launch_bounds__(kMatThreads) void freq_matmul_kernel(MatArgs M) {
  extern __shared__ __align__(16) uint32_t mat_lds[];
  const uint32_t n = M.n, n2 = n * n, RS = (n + 1) * KB;
  const uint64_t N = M.N;
  // consecutive frequency slices on one XCD (workgroups are dealt to the 8 XCDs in
  // turn): the slices of one 128-byte line are then fetched into one L2
  const uint32_t G = gridDim.x, bid = blockIdx.x;
  const uint32_t slice = (G & 7u) == 0 ? (bid & 7u) * (G >> 3) + (bid >> 3) : bid;
  const uint64_t k0 = (uint64_t)slice * KB;
  uint32_t* As = mat_lds;
  uint32_t* Bt = mat_lds + (size_t)n * RS;
  const uint32_t tid = threadIdx.x;
  if constexpr (KB >= 4) {
    constexpr uint32_t q = KB / 4;
    for (uint32_t idx = tid; idx < n2 * q; idx += kMatThreads) {
      const uint32_t e = idx / q, c = (idx - e * q) * 4;
      const uint32_t r = e / n, s = e - r * n;  // entry (r, s)
      const uint64_t g = (uint64_t)e * N + k0 + c;
      *(uint4*)(As + r * RS + s * KB + c) = *(const uint4*)(M.A + g);  // A[r][s]: row r, l = s
      *(uint4*)(Bt + s * RS + r * KB + c) = *(const uint4*)(M.B + g);  // B[r][s]: column s, l = r
    }
  } else {
    for (uint32_t idx = tid; idx < n2 * KB; idx += kMatThreads) {
      const uint32_t e = idx / KB, c = idx - e * KB;
      const uint32_t r = e / n, s = e - r * n;
      const uint64_t g = (uint64_t)e * N + k0 + c;
      As[r * RS + s * KB + c] = M.A[g];
      Bt[s * RS + r * KB + c] = M.B[g];
    }
  }
  __syncthreads();
  const uint32_t p = M.p, S = (n + 3) >> 2;
  const uint32_t items = S * S * KB;
  for (uint32_t w = tid; w < items; w += kMatThreads) {
    const uint32_t t = w / KB, kk = w - t * KB;
    const uint32_t ib = t / S, jb = t - ib * S;
    // rows ib + S a and columns jb + S b; those beyond n read row / column n - 1 and
    // are not stored
    const uint32_t* pa[4];
    const uint32_t* pb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) pa[a] = As + min(ib + S * a, n - 1) * RS + kk;
#pragma unroll
    for (int b = 0; b < 4; ++b) pb[b] = Bt + min(jb + S * b, n - 1) * RS + kk;
    uint64_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = 0;
    for (uint32_t l0 = 0; l0 < n; l0 += M.fold) {
      const uint32_t l1 = min(n, l0 + M.fold);
#pragma unroll 4
      for (uint32_t l = l0; l < l1; ++l) {
        uint32_t x[4], y[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) x[a] = pa[a][l * KB];
#pragma unroll
        for (int b = 0; b < 4; ++b) y[b] = pb[b][l * KB];
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

// p != 0: words reduced modulo p on the way (Function 8 with y = 1, psi = floor(2^32 / p),
// gives [0, 2p) for any 32-bit word; one min finishes).
__global__ void copy_rows_kernel(uint32_t* dst, uint64_t dst_stride, uint64_t dst_len, const uint32_t* src,
                                 uint64_t src_stride, uint64_t src_len, uint32_t rows, uint32_t p, uint32_t psi) {
  const uint64_t total = (uint64_t)rows * dst_len;
  for (uint64_t idx = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t r = idx / dst_len, t = idx - r * dst_len;
    uint32_t v = t < src_len ? src[r * src_stride + t] : 0u;
    if (p) {
      v = v - __umulhi(v, psi) * p;
      v = min(v, v - p);
    }
    dst[r * dst_stride + t] = v;
  }
}

}  // namespace

uint32_t freq_matmul_block(uint32_t n, uint64_t N) {
  if (n == 0 || n > kMatMaxN) return 0;
  uint32_t kb = 256;
  // n (n + 1) KB words per operand, at most 8448 (33 KiB): two operands in 68 KiB of
  // LDS, two workgroups per CU; KB = 8 at n = 32, 16 at n = 16 (measured best)
  while (kb > 1 && (uint64_t)n * (n + 1) * kb > 8448) kb >>= 1;
  while ((uint64_t)kb > N) kb >>= 1;
  return kb;
}

template <int KB>
static hipError_t launch_freq_matmul_kb(const MatArgs& a, hipStream_t stream) {
  const size_t lds = 2 * (size_t)a.n * (a.n + 1) * KB * sizeof(uint32_t);
  auto k = freq_matmul_kernel<KB>;
  hipError_t e = allow_dynamic_lds((const void*)k, lds);
  if (e != hipSuccess) return e;
  const uint64_t grid = a.N / KB;
  if (grid > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3((uint32_t)grid), dim3(kMatThreads), lds, stream, a);
  return hipGetLastError();
}

hipError_t launch_freq_matmul(const MatArgs& a, hipStream_t stream) {
  if (a.n == 0 || a.n > kMatMaxN || a.kb == 0 || (a.N % a.kb) != 0 || a.fold == 0) return hipErrorInvalidValue;
  if (a.kb >= 4 && (((uintptr_t)a.A | (uintptr_t)a.B) & 15u)) return hipErrorInvalidValue;
  switch (a.kb) {
    case 1: return launch_freq_matmul_kb<1>(a, stream);
    case 2: return launch_freq_matmul_kb<2>(a, stream);
    case 4: return launch_freq_matmul_kb<4>(a, stream);
    case 8: return launch_freq_matmul_kb<8>(a, stream);
    case 16: return launch_freq_matmul_kb<16>(a, stream);
    case 32: return launch_freq_matmul_kb<32>(a, stream);
    case 64: return launch_freq_matmul_kb<64>(a, stream);
    case 128: return launch_freq_matmul_kb<128>(a, stream);
    case 256: return launch_freq_matmul_kb<256>(a, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_copy_rows(uint32_t* dst, uint64_t dst_stride, uint64_t dst_len, const uint32_t* src,
                            uint64_t src_stride, uint64_t src_len, uint32_t rows, hipStream_t stream,
                            uint32_t reduce_p) {
  const uint64_t total = (uint64_t)rows * dst_len;
  if (total == 0) return hipSuccess;
  if (reduce_p >= (1u << 31)) return hipErrorInvalidValue;
  const uint32_t psi = reduce_p ? (uint32_t)((1ull << 32) / reduce_p) : 0u;
  const uint64_t blocks = (total + 255) / 256;
  const uint32_t grid = (uint32_t)(blocks < 8192 ? blocks : 8192);
  hipLaunchKernelGGL(copy_rows_kernel, dim3(grid), dim3(256), 0, stream, dst, dst_stride, dst_len, src, src_stride,
                     src_len, rows, reduce_p, psi);
  return hipGetLastError();
}

}  // namespace nttgpu
