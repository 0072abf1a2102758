// Fused product kernels for 64-bit words (p < 2^62) and for residues held in doubles
// (section 3, p < 2^49): transform lengths up to 2^15.
#include "polymul_fused.hpp"

namespace nttgpu {

hipError_t launch_fused_w64(int cls, const FusedBatch& batch, int grid, hipStream_t stream) {
  switch (cls) {
    case 0: return launch_fused_cls<uint64_t, 64, 10, 0, 0, 0>(batch, grid, stream);
    case 1: return launch_fused_cls<uint64_t, 256, 12, 11, 0, 0>(batch, grid, stream);
    case 3: return launch_fused_cls<uint64_t, 512, 13, 13, 2, 0>(batch, grid, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace nttgpu
