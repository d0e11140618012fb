// Kernel launch entry points (defined in gft_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_program.hpp"

namespace gft {

// Persistent fused apply of one program to S signals; grid = min(tiles, grid_cap).
hipError_t launch_apply(const DevProgram &P, const void *in, void *out, int64_t S,
                        hipStream_t stream, int grid_cap, bool in16, bool out16);

// Resident workgroups per CU of the apply kernel for this program's LDS footprint.
int apply_occupancy(const DevProgram &P);

// Mixed batch: G programs (device array `progs`) in one persistent launch; graphs with a
// register-butterfly program (device array `uprogs`, entry S = 0 for the others; or null)
// run on the first reg_groups workgroups' waves, the rest on the LDS programs.
size_t batch_lds_bytes(int G, size_t max_program_lds, bool reg_phase);
int batch_occupancy(int prec, size_t lds, bool io16);
// BF16 storage (gft_batch16.hip).
int batch_occupancy_io16(int prec, size_t lds);
hipError_t launch_apply_batch_io16(int prec, int dir, const DevProgram *progs, const UProgram *uprogs, int G,
                                   const int64_t *sig_off, int64_t total_elems, const void *in, void *out,
                                   size_t lds, int grid, int reg_groups, int cost16, hipStream_t stream);
bool batch_butterfly_supported(int prec, const UProgram &U);
// cost16: register-phase fixed cost per signal in sixteenths of the padded slot count;
// io16: signals and coefficients stored in BF16 (else FP32).
hipError_t launch_apply_batch(int prec, int dir, bool io16, const DevProgram *progs, const UProgram *uprogs,
                              int G, const int64_t *sig_off, int64_t total_elems, const void *in,
                              void *out, size_t lds, int grid, int reg_groups, int cost16,
                              hipStream_t stream);

// Large-signal engine.
// Signal rows per LDS tile of a stage/gather pass: as many as fill about tile_kb KB (0: the
// built-in 40 KB), 1 to 16.
int permute_rows(const PermPass &P, int tile_kb = 0);
// in16 / out16: BF16 input rows / BF16 output rows (else FP32).
hipError_t launch_permute_stages(const PermPass &P, const void *in, bool in16, void *out, bool out16,
                                 int64_t S, int num_cus, hipStream_t stream, int tile_kb = 0);
int64_t block_gemm_grid(const int32_t *sizes, int nblocks, int64_t S);
// prec: 0 FP32, 1 BF16 (A and matrices stored in BF16), 3 split BF16 (FP32 storage)
// omap non-null: column c of block b is written to column omap[b.omap + c] of C (row
// stride ldy) instead of the workspace (the output permutation fused into the epilogue);
// out16 (with omap only): C holds BF16 values.
hipError_t launch_block_gemm(int prec, const LBlock *blocks, int nblocks, const void *mats,
                             const void *A, void *C, bool out16, int64_t S, int ld, int64_t grid,
                             const int32_t *omap, int ldy, hipStream_t stream);

// One-pass form of the large-signal engine (OnePass; precision GFT_BF16 or GFT_SPLIT_BF16).
// grid: most workgroups (0: one per row panel), each taking panels of onepass_rows()
// signals in turn.
int onepass_rows(int precision);
int onepass_occupancy(const OnePass &P, int precision, bool in16);   // resident workgroups per CU
hipError_t launch_onepass(const OnePass &P, int precision, const void *in, void *out, int64_t S, bool in16,
                          bool out16, int grid, hipStream_t stream);
// FP32 instances (gft_onepass0.hip)
int onepass_occupancy_f32(const OnePass &P, bool in16);
hipError_t launch_onepass_f32(const OnePass &P, const void *in, void *out, int64_t S, bool in16, bool out16,
                              int grid, hipStream_t st);
// split-BF16 instances (gft_onepass3.hip)
int onepass_occupancy_split(const OnePass &P, bool in16);
hipError_t launch_onepass_split(const OnePass &P, const void *in, void *out, int64_t S, bool in16, bool out16,
                                int grid, hipStream_t stream);

// Static scratch of the allocation-free apply: kScratchBytes per GPU, in the code object.
// large_scratch_setup(dev) runs with device `dev` current (at plan preparation), looks up
// the array's address on that device once and keeps it; large_scratch(dev) returns it
// (null before set-up).
constexpr size_t kScratchBytes = (size_t)64 << 20;
hipError_t large_scratch_setup(int dev);
void *large_scratch(int dev);

// Register-butterfly engine (uniform hypercube plans).
bool butterfly_supported(const UProgram &P);   // a kernel is compiled for its shape
// in16 / out16: the input / output array holds BF16 values (else FP32).
// grid_cap: most workgroups launched (0: every resident workgroup, occupancy x CUs).
hipError_t launch_butterfly(const UProgram &P, const void *in, void *out, int64_t nsig,
                            hipStream_t stream, int num_cus, bool in16, bool out16, int grid_cap = 0);
int butterfly_occupancy(const UProgram &P, bool in16, bool out16);   // resident workgroups per CU

// Product-graph engine: factor sizes padded to 16, 32 or 64 (0 above 64).
int product_pad(int n);
hipError_t launch_product(const PProgram &P, const float *in, float *out, int64_t nsig,
                          hipStream_t stream, int num_cus, int grid_cap = 0);
int product_occupancy(const PProgram &P);   // resident workgroups per CU
// BF16 storage (tile_pattern 2), gft_product16.hip.
hipError_t launch_product_io16(const PProgram &P, const void *in, void *out, int64_t nsig,
                               hipStream_t stream, int num_cus, int grid_cap);
int product_occupancy_io16(const PProgram &P);

// Streaming copy of `bytes` (a multiple of 16) between 16-byte aligned, non-overlapping
// device buffers (gft_copy.hip).
hipError_t launch_stream_copy(const void *in, void *out, int64_t bytes, hipStream_t stream,
                              int num_cus);

}  // namespace gft
