// One-pass large-signal GFT for gfx950: BF16 blocks, and the launch entry points (the
// kernel is in onepass_core.hpp; FP32 and split-BF16 blocks are instantiated in
// gft_onepass0.hip and gft_onepass3.hip).
#include "launch.hpp"
#include "onepass_core.hpp"

namespace gft {

int onepass_rows(int precision) {
  return 16 * (precision == 3 ? onepass::OnePassShape<3, 1>::MT : onepass::OnePassShape<1, 1>::MT);
}

int onepass_occupancy(const OnePass &P, int precision, bool in16) {
  if (precision == 3) return onepass_occupancy_split(P, in16);
  if (precision == 0) return onepass_occupancy_f32(P, in16);
  return onepass::occupancy_prec<1>(P.src_mode, in16);
}

hipError_t launch_onepass(const OnePass &P, int precision, const void *in, void *out, int64_t S, bool in16,
                          bool out16, int grid, hipStream_t st) {
  if (S <= 0) return hipSuccess;
  const int64_t panels = (S + onepass_rows(precision) - 1) / onepass_rows(precision);
  if (grid <= 0 || grid > panels) grid = (int)(panels < (1 << 30) ? panels : (1 << 30));
  if (precision == 3) return launch_onepass_split(P, in, out, S, in16, out16, grid, st);
  if (precision == 0) return launch_onepass_f32(P, in, out, S, in16, out16, grid, st);
  if (precision != 1) return hipErrorInvalidValue;
  return onepass::launch_prec<1>(P, in, out, S, in16, out16, grid, st);
}

}  // namespace gft
