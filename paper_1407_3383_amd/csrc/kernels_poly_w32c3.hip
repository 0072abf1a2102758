// Fused product kernel for 32-bit words and transform lengths 2^14 .. 2^16 (up to
// four sub-problems of 2^14 words per product, partials parked in the workspace).
#include "polymul_fused.hpp"

namespace nttgpu {

hipError_t launch_fused_w32_c3(const FusedBatch& batch, int grid, hipStream_t stream) {
  return launch_fused_cls<uint32_t, 1024, 14, 14, 2, 1>(batch, grid, stream);
}

}  // namespace nttgpu
