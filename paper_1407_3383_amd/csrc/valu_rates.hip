// Issue-rate probes for the vector ALU instructions the transform kernels are built
// from, and for the kernels' own butterflies run on registers alone.  Each thread
// runs 8 independent dependency chains (enough to cover the instruction latencies
// with several waves per SIMD) of one instruction, written as inline assembly so
// that the compiler can neither merge nor drop them; the chains' values are written
// out once at the end.  The rate follows from the count of instructions issued and
// the kernel's duration: lane-operations per second = threads * iterations * 16 * 8
// / time.  Butterfly probes run the library's own CT / GS butterflies (arith.hpp)
// on 8 register pairs per thread with a twiddle held in scalar registers, and count
// butterflies.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "arith.hpp"

using namespace nttgpu;

namespace {

enum {
  OP_ADD = 0, OP_SUB, OP_ADD3, OP_MIN, OP_MUL_LO, OP_MUL_HI, OP_MAD64, OP_CNDMASK, OP_FMA_F64, OP_XOR,
  OP_LSHL_ADD, OP_CT31, OP_CT_LAZY, OP_GS31, OP_GS_LAZY, OP_DPP_MOV, OP_PERMLANE32_SWAP, OP_DS_BPERMUTE, OP_COUNT
};

template <int OP>
__device__ __forceinline__ void step(uint32_t& x, uint32_t c, uint32_t d) {
  if constexpr (OP == OP_ADD) asm volatile("v_add_u32 %0, %0, %1" : "+v"(x) : "v"(c));
  else if constexpr (OP == OP_SUB) asm volatile("v_sub_u32 %0, %0, %1" : "+v"(x) : "v"(c));
  else if constexpr (OP == OP_ADD3) asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(x) : "v"(c), "v"(d));
  else if constexpr (OP == OP_MIN) asm volatile("v_min_u32 %0, %0, %1" : "+v"(x) : "v"(c));
  else if constexpr (OP == OP_MUL_LO) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x) : "v"(c));
  else if constexpr (OP == OP_MUL_HI) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(x) : "v"(c));
  else if constexpr (OP == OP_XOR) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(x) : "v"(c));
  else if constexpr (OP == OP_LSHL_ADD) asm volatile("v_lshl_add_u32 %0, %0, 1, %1" : "+v"(x) : "v"(c));
  else if constexpr (OP == OP_CNDMASK) asm volatile("v_cndmask_b32 %0, %0, %1, vcc" : "+v"(x) : "v"(c));
}

template <int OP>
__global__ __launch_bounds__(256) void rate_kernel(uint32_t* out, int iters, uint32_t seed) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t c = seed | 1u, d = seed >> 3;
  uint32_t x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = tid * 8u + (uint32_t)k;
  if constexpr (OP == OP_CNDMASK) asm volatile("v_cmp_gt_u32 vcc, %0, %1" : : "v"(x[0]), "v"(c) : "vcc");
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
      for (int k = 0; k < 8; ++k) step<OP>(x[k], c, d);
  }
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) r ^= x[k];
  out[tid] = r;
}

// 32x32 -> 64-bit multiply-add chains (the fixed-multiplicand product's two
// instructions): 64-bit accumulators.
__global__ __launch_bounds__(256) void rate_mad64_kernel(uint32_t* out, int iters, uint32_t seed) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t c = seed | 1u;
  uint64_t x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = tid * 8u + (uint32_t)k;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
      for (int k = 0; k < 8; ++k)
        asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(x[k]) : "v"((uint32_t)x[k]), "v"(c) : "vcc");
  }
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) r ^= (uint32_t)x[k] ^ (uint32_t)(x[k] >> 32);
  out[tid] = r;
}

__global__ __launch_bounds__(256) void rate_fma64_kernel(uint32_t* out, int iters, uint32_t seed) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const double c = 1.0 + 1.0 / (double)(seed | 1u), d = 1.0 / 3.0;
  double x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = (double)(tid * 8u + (uint32_t)k);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
      for (int k = 0; k < 8; ++k) asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(x[k]) : "v"(c), "v"(d));
  }
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) r ^= (uint32_t)__double_as_longlong(x[k]);
  out[tid] = r;
}

// Cross-lane moves, the alternatives to an exchange through LDS between the wave-local
// rounds: a DPP row shift (v_mov_b32 with row_shr:1, a VALU instruction), gfx950's
// v_permlane32_swap (swaps the upper half-wave of one register with the lower of
// another: one instruction per register pair) and ds_bpermute (a lane gather through
// the LDS crossbar, issued on the LDS pipe).  Built-ins, so that the compiler places the
// wait states DPP needs.  8 chains per thread; per iteration 128 moves (64 swaps).
template <int OP>
__global__ __launch_bounds__(256) void rate_xlane_kernel(uint32_t* out, int iters) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int addr = (int)(((threadIdx.x & 63u) ^ 1u) << 2);  // neighbouring lane
  uint32_t x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = tid * 8u + (uint32_t)k;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if constexpr (OP == OP_DPP_MOV) {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = __builtin_amdgcn_update_dpp(0u, x[k], 0x111, 0xf, 0xf, false);
      } else if constexpr (OP == OP_PERMLANE32_SWAP) {
#pragma unroll
        for (int k = 0; k < 8; k += 2) {
          const auto r = __builtin_amdgcn_permlane32_swap(x[k], x[k + 1], false, false);
          x[k] = r[0];
          x[k + 1] = r[1];
        }
      } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)x[k]);
      }
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) r ^= x[k];
  out[tid] = r;
}

// The library's butterflies on registers: 8 pairs per thread, 16 butterflies per
// pair and iteration, twiddle in scalar registers (the UNI forms).
template <bool GS, int LAZY>
__global__ __launch_bounds__(256) void rate_bfly_kernel(uint32_t* out, int iters, uint32_t p, uint32_t pinv,
                                                        uint32_t w, uint32_t ws) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  Arith<uint32_t> ar;
  ar.p = uni(p);
  ar.p2 = uni(2 * p);
  ar.pinv = uni(pinv);
  TwPair<uint32_t> tw;
  tw.w = uni(w);
  tw.ws = uni(ws);
  uint32_t X[8], Y[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    X[k] = (tid * 16u + (uint32_t)k) % p;
    Y[k] = (tid * 16u + 8u + (uint32_t)k) % p;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 16; ++u)
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if constexpr (GS) gs_bfly<LAZY, true>(ar, X[k], Y[k], tw);
        else ct_bfly<LAZY, true>(ar, X[k], Y[k], tw);
      }
  }
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) r ^= X[k] ^ Y[k];
  out[tid] = r;
}

}  // namespace

extern "C" {

// Launches probe `op` on `grid` workgroups of 256 threads, `iters` iterations of 128
// operations (or butterflies) per thread; `out` holds grid * 256 words.  For the
// butterfly probes p (< 2^31), p^-1 mod 2^32 and the twiddle pair (w, floor(w 2^32 / p))
// are arguments.  Returns 0 or a HIP error code.
int valu_rate_launch(int op, int grid, int iters, void* out, uint64_t p, uint32_t pinv, uint32_t w, uint32_t ws,
                     void* stream) {
  hipStream_t s = (hipStream_t)stream;
  uint32_t* o = (uint32_t*)out;
  const dim3 g(grid), b(256);
  const uint32_t seed = 0x9e3779b9u;
  switch (op) {
    case OP_ADD: hipLaunchKernelGGL(rate_kernel<OP_ADD>, g, b, 0, s, o, iters, seed); break;
    case OP_SUB: hipLaunchKernelGGL(rate_kernel<OP_SUB>, g, b, 0, s, o, iters, seed); break;
    case OP_ADD3: hipLaunchKernelGGL(rate_kernel<OP_ADD3>, g, b, 0, s, o, iters, seed); break;
    case OP_MIN: hipLaunchKernelGGL(rate_kernel<OP_MIN>, g, b, 0, s, o, iters, seed); break;
    case OP_MUL_LO: hipLaunchKernelGGL(rate_kernel<OP_MUL_LO>, g, b, 0, s, o, iters, seed); break;
    case OP_MUL_HI: hipLaunchKernelGGL(rate_kernel<OP_MUL_HI>, g, b, 0, s, o, iters, seed); break;
    case OP_MAD64: hipLaunchKernelGGL(rate_mad64_kernel, g, b, 0, s, o, iters, seed); break;
    case OP_CNDMASK: hipLaunchKernelGGL(rate_kernel<OP_CNDMASK>, g, b, 0, s, o, iters, seed); break;
    case OP_FMA_F64: hipLaunchKernelGGL(rate_fma64_kernel, g, b, 0, s, o, iters, seed); break;
    case OP_XOR: hipLaunchKernelGGL(rate_kernel<OP_XOR>, g, b, 0, s, o, iters, seed); break;
    case OP_LSHL_ADD: hipLaunchKernelGGL(rate_kernel<OP_LSHL_ADD>, g, b, 0, s, o, iters, seed); break;
    case OP_CT31:
      hipLaunchKernelGGL((rate_bfly_kernel<false, false>), g, b, 0, s, o, iters, (uint32_t)p, pinv, w, ws);
      break;
    case OP_CT_LAZY:
      hipLaunchKernelGGL((rate_bfly_kernel<false, true>), g, b, 0, s, o, iters, (uint32_t)p, pinv, w, ws);
      break;
    case OP_GS31:
      hipLaunchKernelGGL((rate_bfly_kernel<true, false>), g, b, 0, s, o, iters, (uint32_t)p, pinv, w, ws);
      break;
    case OP_GS_LAZY:
      hipLaunchKernelGGL((rate_bfly_kernel<true, true>), g, b, 0, s, o, iters, (uint32_t)p, pinv, w, ws);
      break;
    case OP_DPP_MOV: hipLaunchKernelGGL(rate_xlane_kernel<OP_DPP_MOV>, g, b, 0, s, o, iters); break;
    case OP_PERMLANE32_SWAP: hipLaunchKernelGGL(rate_xlane_kernel<OP_PERMLANE32_SWAP>, g, b, 0, s, o, iters); break;
    case OP_DS_BPERMUTE: hipLaunchKernelGGL(rate_xlane_kernel<OP_DS_BPERMUTE>, g, b, 0, s, o, iters); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

int valu_rate_op_count(void) { return OP_COUNT; }

}  // extern "C"
