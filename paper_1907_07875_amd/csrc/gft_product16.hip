// Separable engine, BF16 storage of signals and coefficients (dense factors): the
// product_core.hpp kernel with tile pattern 2, in a translation unit of its own so that it
// compiles beside the FP32-storage kernels.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "product_core.hpp"

namespace gft {

hipError_t launch_product_io16(const PProgram &P, const void *in, void *out, int64_t nsig,
                               hipStream_t stream, int num_cus, int grid_cap) {
  return dispatch_product<true>(P, in, out, nsig, stream, num_cus, grid_cap, nullptr);
}

int product_occupancy_io16(const PProgram &P) {
  int occ = 1;
  if (dispatch_product<true>(P, nullptr, nullptr, 0, nullptr, -1, 0, &occ) != hipSuccess) return 1;
  return occ;
}

}  // namespace gft
