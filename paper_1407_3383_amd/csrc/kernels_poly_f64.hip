// The fused product kernels over residues held in doubles (section 3, Function 16
// through Arith<double>; the classes and grids of the 64-bit word size), and their
// variants for primes 2^49 <= p < 2^50 (band).
#include "polymul_fused.hpp"

namespace nttgpu {

hipError_t launch_fused_f64(int cls, bool band, const FusedBatch& batch, int grid, hipStream_t stream) {
  if (band) {
    switch (cls) {
      case 0: return launch_fused_cls<double, 64, 10, 0, 0, 0, true>(batch, grid, stream);
      case 1: return launch_fused_cls<double, 256, 12, 11, 0, 0, true>(batch, grid, stream);
      case 3: return launch_fused_cls<double, 512, 13, 13, 2, 0, true>(batch, grid, stream);
    }
    return hipErrorInvalidValue;
  }
  switch (cls) {
    case 0: return launch_fused_cls<double, 64, 10, 0, 0, 0>(batch, grid, stream);
    case 1: return launch_fused_cls<double, 256, 12, 11, 0, 0>(batch, grid, stream);
    case 3: return launch_fused_cls<double, 512, 13, 13, 2, 0>(batch, grid, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace nttgpu
