// Fused product kernels for 32-bit words, transform lengths up to 2^13 (one
// sub-problem per product, held in LDS).
#include "polymul_fused.hpp"

namespace nttgpu {

hipError_t launch_fused_w32_small(int cls, const FusedBatch& batch, int grid, hipStream_t stream) {
  switch (cls) {
    case 0: return launch_fused_cls<uint32_t, 64, 10, 0, 0, 0>(batch, grid, stream);
    case 1: return launch_fused_cls<uint32_t, 256, 12, 11, 0, 0>(batch, grid, stream);
    case 2: return launch_fused_cls<uint32_t, 512, 13, 13, 0, 0>(batch, grid, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace nttgpu
