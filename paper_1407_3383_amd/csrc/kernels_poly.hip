// Fused polynomial product kernels (section 5.2): size classes, workspace and grid
// of a fused launch, and the dispatch to the translation units that instantiate the
// kernels of polymul_fused.hpp (one per word type and class group).
#include "polymul_fused.hpp"

namespace nttgpu {

// Size classes: the class fixes the workgroup size and the LDS sub-problem size.
int fused_class(int word_bits, int log2n) {
  if (word_bits == 32) {
    if (log2n <= 10) return 0;
    if (log2n <= 12) return 1;
    if (log2n <= 13) return 2;
    if (log2n <= 16) return 3;
    return -1;
  }
  if (log2n <= 10) return 0;
  if (log2n <= 12) return 1;
  if (log2n <= 15) return 3;
  return -1;
}

int fused_max_log2n(int word_bits) { return word_bits == 32 ? 16 : 15; }

// Words of workspace per workgroup that parks partial results (classes 3 and 4).
size_t fused_park_words(int word_bits, int cls) {
  if (word_bits != 32) return 0;
  if (cls == 3) return 3 * ((size_t)1 << 14);
  if (cls == 4) return (size_t)1 << 15;
  return 0;
}

// Workgroups of a class-3 or class-4 launch (its items loop over this many workgroups).
int fused_grid(int word_bits, int cls, size_t count, int cus) {
  (void)word_bits;
  if (cls == 3 || cls == 4) return (int)std::min<size_t>(count, (size_t)cus);
  return (int)std::min<size_t>(count, (size_t)1 << 20);
}

hipError_t launch_fused(int word_bits, int cls, const FusedBatch& batch, int grid, hipStream_t stream) {
  if (word_bits == 32) {
    if (cls == 3) return launch_fused_w32_c3(batch, grid, stream);
    if (cls == 4) return launch_fused_w32_c4(batch, grid, stream);
    return launch_fused_w32_small(cls, batch, grid, stream);
  }
  return launch_fused_w64(cls, batch, grid, stream);
}

}  // namespace nttgpu
