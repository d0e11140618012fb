// Mixed batch kernel with BF16 storage of signals and coefficients: the lds_core.hpp
// kernel instantiated for BF16 input and output, in a translation unit of its own so that
// it compiles beside the FP32-storage kernels.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.hpp"
#include "lds_core.hpp"

namespace gft {

template <int PREC>
static hipError_t launch_batch16_p(int dir, const DevProgram *progs, const UProgram *uprogs, int G,
                                   const int64_t *sig_off, int64_t total_elems, const void *in, void *out,
                                   size_t lds, int grid, int reg_groups, int cost16, hipStream_t stream) {
  return dir == 0 ? launch_batch_pd<PREC, 0, true>(progs, uprogs, G, sig_off, total_elems, in, out, lds, grid, reg_groups, cost16, stream)
                  : launch_batch_pd<PREC, 1, true>(progs, uprogs, G, sig_off, total_elems, in, out, lds, grid, reg_groups, cost16, stream);
}

hipError_t launch_apply_batch_io16(int prec, int dir, const DevProgram *progs, const UProgram *uprogs, int G,
                                   const int64_t *sig_off, int64_t total_elems, const void *in, void *out,
                                   size_t lds, int grid, int reg_groups, int cost16, hipStream_t stream) {
  switch (prec) {
    case kFP32: return launch_batch16_p<kFP32>(dir, progs, uprogs, G, sig_off, total_elems, in, out, lds, grid, reg_groups, cost16, stream);
    case kBF16: return launch_batch16_p<kBF16>(dir, progs, uprogs, G, sig_off, total_elems, in, out, lds, grid, reg_groups, cost16, stream);
    case kFP16: return launch_batch16_p<kFP16>(dir, progs, uprogs, G, sig_off, total_elems, in, out, lds, grid, reg_groups, cost16, stream);
    case kSPLIT: return launch_batch16_p<kSPLIT>(dir, progs, uprogs, G, sig_off, total_elems, in, out, lds, grid, reg_groups, cost16, stream);
    default: return hipErrorInvalidValue;
  }
}

int batch_occupancy_io16(int prec, size_t lds) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (prec) {
    case kFP32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gft_apply_batch<kFP32, 0, true>, kThreads, lds); break;
    case kBF16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gft_apply_batch<kBF16, 0, true>, kThreads, lds); break;
    case kFP16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gft_apply_batch<kFP16, 0, true>, kThreads, lds); break;
    case kSPLIT: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gft_apply_batch<kSPLIT, 0, true>, kThreads, lds); break;
    default: break;
  }
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

}  // namespace gft
