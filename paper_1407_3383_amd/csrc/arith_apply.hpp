// Element-wise evaluation of the device modular primitives (tests of the arithmetic
// alone; see ntt_arith_apply in include/ntt_mi355x.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ntt_mi355x.h"

namespace nttgpu {

// op NTT_ARITH_*; word 32 / 64 (unsigned words) or 0 (doubles, Function 16).
struct ArithArgs {
  const void* x;
  const void* y;
  const void* ys;     // Shoup companions of y (unsigned words, op SHOUP)
  void* out;          // n words (2 n for the butterflies: X' then Y')
  uint64_t n;
  uint64_t p, pinv;   // pinv = p^-1 mod 2^word (unsigned words)
  uint64_t tw, tws;   // butterfly twiddle and companion (unsigned words)
  double twd;         // butterfly twiddle (doubles)
  int op, word;
};
hipError_t launch_arith_apply(const ArithArgs& a, hipStream_t stream);

}  // namespace nttgpu
