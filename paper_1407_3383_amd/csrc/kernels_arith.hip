// Element-wise evaluation of the device modular primitives (section 2: Function 8's
// fixed-multiplicand product without its final correction, Montgomery's product of
// Function 13, the min-trick reductions of Function 2; section 3: Function 16 over
// doubles) and of the two butterflies built from them, on arrays: the arithmetic
// alone, as every transform kernel uses it, for tests against the oracle.
#include <type_traits>

#include "arith.hpp"
#include "arith_apply.hpp"

namespace nttgpu {

namespace {

template <typename T, int OP, int LAZY>
__global__ __launch_bounds__(256) void arith_apply_kernel(ArithArgs A, Arith<T> ar) {
  const T* x = (const T*)A.x;
  const T* y = (const T*)A.y;
  const T* ys = (const T*)A.ys;
  T* out = (T*)A.out;
  TwPair<T> tw;
  tw.w = (T)A.tw;
  tw.ws = (T)A.tws;
  if constexpr (std::is_same<T, double>::value) {
    tw.w = A.twd;
    tw.ws = 0.0;
  }
  tw = uni(tw);  // a twiddle that is the same in every lane (the scalar-operand forms)
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < A.n; i += (uint64_t)gridDim.x * blockDim.x) {
    if constexpr (OP == NTT_ARITH_SHOUP) {
      out[i] = ar.shoup(x[i], y[i], std::is_same<T, double>::value ? (T)0 : ys[i]);
    } else if constexpr (OP == NTT_ARITH_MONT) {
      out[i] = ar.mont(x[i], y[i]);
    } else if constexpr (OP == NTT_ARITH_RED1) {
      out[i] = ar.red1(x[i]);
    } else if constexpr (OP == NTT_ARITH_RED2) {
      out[i] = ar.red2(x[i]);
    } else if constexpr (OP == NTT_ARITH_CT) {
      T X = x[i], Y = y[i];
      ct_bfly<LAZY, true>(ar, X, Y, tw);
      out[i] = X;
      out[A.n + i] = Y;
    } else {
      T X = x[i], Y = y[i];
      gs_bfly<LAZY, true>(ar, X, Y, tw);
      out[i] = X;
      out[A.n + i] = Y;
    }
  }
}

template <typename T, int OP>
hipError_t launch_op(const ArithArgs& a, const Arith<T>& ar, int mode, hipStream_t stream) {
  const uint64_t blocks = (a.n + 255) / 256;
  const uint32_t grid = (uint32_t)(blocks < 4096 ? blocks : 4096);
  if (mode == kLazy) {
    hipLaunchKernelGGL((arith_apply_kernel<T, OP, kLazy>), dim3(grid), dim3(256), 0, stream, a, ar);
  } else if constexpr (std::is_same<T, double>::value) {
    if (mode == kBand) hipLaunchKernelGGL((arith_apply_kernel<T, OP, kBand>), dim3(grid), dim3(256), 0, stream, a, ar);
    else hipLaunchKernelGGL((arith_apply_kernel<T, OP, kSafe>), dim3(grid), dim3(256), 0, stream, a, ar);
  } else {
    hipLaunchKernelGGL((arith_apply_kernel<T, OP, kSafe>), dim3(grid), dim3(256), 0, stream, a, ar);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_word(const ArithArgs& a, const Arith<T>& ar, int lazy, hipStream_t stream) {
  switch (a.op) {
    case NTT_ARITH_SHOUP: return launch_op<T, NTT_ARITH_SHOUP>(a, ar, lazy, stream);
    case NTT_ARITH_MONT: return launch_op<T, NTT_ARITH_MONT>(a, ar, lazy, stream);
    case NTT_ARITH_RED1: return launch_op<T, NTT_ARITH_RED1>(a, ar, lazy, stream);
    case NTT_ARITH_RED2: return launch_op<T, NTT_ARITH_RED2>(a, ar, lazy, stream);
    case NTT_ARITH_CT: return launch_op<T, NTT_ARITH_CT>(a, ar, lazy, stream);
    case NTT_ARITH_GS: return launch_op<T, NTT_ARITH_GS>(a, ar, lazy, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_arith_apply(const ArithArgs& a, hipStream_t stream) {
  if (a.n == 0) return hipSuccess;
  if (a.word == 32) {
    Arith<uint32_t> ar;
    ar.p = (uint32_t)a.p;
    ar.p2 = (uint32_t)(2 * a.p);
    ar.pinv = (uint32_t)a.pinv;
    return launch_word<uint32_t>(a, ar, a.p < (1ull << 30) ? kLazy : kSafe, stream);
  }
  if (a.word == 64) {
    Arith<uint64_t> ar;
    ar.p = a.p;
    ar.p2 = 2 * a.p;
    ar.pinv = a.pinv;
    return launch_word<uint64_t>(a, ar, kLazy, stream);
  }
  Arith<double> ar;
  ar.p = (double)a.p;
  ar.p2 = 2.0 * (double)a.p;
  ar.pinv = 1.0 / (double)a.p;
  return launch_word<double>(a, ar, a.p < (1ull << 48) ? kLazy : a.p < (1ull << 49) ? kSafe : kBand, stream);
}

}  // namespace nttgpu
