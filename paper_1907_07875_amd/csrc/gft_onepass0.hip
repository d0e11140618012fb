// One-pass large-signal GFT for gfx950: FP32 blocks (16x16x4 FP32 MFMAs; the kernel is in onepass_core.hpp).
#include "launch.hpp"
#include "onepass_core.hpp"

namespace gft {

int onepass_occupancy_f32(const OnePass &P, bool in16) { return onepass::occupancy_prec<0>(P.src_mode, in16); }

hipError_t launch_onepass_f32(const OnePass &P, const void *in, void *out, int64_t S, bool in16, bool out16,
                              int grid, hipStream_t st) {
  return onepass::launch_prec<0>(P, in, out, S, in16, out16, grid, st);
}

}  // namespace gft
