// Kernel launch entry points (defined in gft_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_program.hpp"

namespace gft {

// Persistent fused apply of one program to S signals; grid = min(tiles, grid_cap).
hipError_t launch_apply(const DevProgram &P, const float *in, float *out, int64_t S,
                        hipStream_t stream, int grid_cap);

// Resident workgroups per CU of the apply kernel for this program's LDS footprint.
int apply_occupancy(const DevProgram &P);

// Register-butterfly engine (uniform hypercube plans).
bool butterfly_supported(int S, int M);
hipError_t launch_butterfly(const UProgram &P, const float *in, float *out, int64_t nsig,
                            hipStream_t stream, int num_cus);

}  // namespace gft
