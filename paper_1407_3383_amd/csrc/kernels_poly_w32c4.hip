// Fused product kernel for 32-bit words and transform length 2^16 as two sub-problems
// of 2^15 words (one operand's sub-problem in LDS, the other's transform in registers;
// one partial parked in the workspace).
#include "polymul_fused.hpp"

namespace nttgpu {

hipError_t launch_fused_w32_c4(const FusedBatch& batch, int grid, hipStream_t stream) {
  return launch_fused_cls<uint32_t, 1024, 15, 16, 1, 1>(batch, grid, stream);
}

}  // namespace nttgpu
