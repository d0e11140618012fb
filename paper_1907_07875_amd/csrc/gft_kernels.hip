// Fused GFT kernels for gfx950 (CDNA4).
//
// One engine runs every plan: a tile of T = 16*mt signals (signal-major, contiguous in
// HBM) is read with 16-byte coalesced loads into an LDS tile [T][stride]; the Haar stages
// (eq. B_phi, unscaled add/sub plus sqrt(2) on V_Z) run in place in LDS; the dense leaf
// blocks run as [T x K] * [K x N] products on v_mfma_f32_16x16x4_f32 with operands
// gathered from LDS and results scattered to a second LDS tile in output order; the
// tile is written back with 16-byte coalesced stores.  The inverse program runs blocks
// first and stages after.  The kernel is persistent: each workgroup walks tiles
// blockIdx.x, blockIdx.x + gridDim.x, ...
#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.hpp"
#include "lds_core.hpp"

namespace gft {

// ---------------------------------------------------------------------------- launch

template <int MT, int PREC, bool IN16, bool OUT16>
static hipError_t launch_mt_io(const DevProgram &P, const void *in, void *out, int64_t S,
                               hipStream_t stream, int grid_cap) {
  const size_t lds = program_lds_bytes(P);
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)gft_apply<MT, PREC, IN16, OUT16>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int64_t T = 16 * MT;
  const int64_t tiles = (S + T - 1) / T;
  int grid = (int)(tiles < grid_cap ? tiles : grid_cap);
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((gft_apply<MT, PREC, IN16, OUT16>), dim3(grid), dim3(kThreads), lds, stream,
                     P, in, out, S);
  return hipGetLastError();
}

template <int MT, int PREC>
static hipError_t launch_mt(const DevProgram &P, const void *in, void *out, int64_t S,
                            hipStream_t stream, int grid_cap, bool in16, bool out16) {
  if (in16)
    return out16 ? launch_mt_io<MT, PREC, true, true>(P, in, out, S, stream, grid_cap)
                 : launch_mt_io<MT, PREC, true, false>(P, in, out, S, stream, grid_cap);
  return out16 ? launch_mt_io<MT, PREC, false, true>(P, in, out, S, stream, grid_cap)
               : launch_mt_io<MT, PREC, false, false>(P, in, out, S, stream, grid_cap);
}

template <int PREC>
static int occupancy_p(const DevProgram &P) {
  const size_t lds = program_lds_bytes(P);
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (P.mt) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gft_apply<1, PREC, false, false>, kThreads, lds); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gft_apply<2, PREC, false, false>, kThreads, lds); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gft_apply<4, PREC, false, false>, kThreads, lds); break;
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gft_apply<8, PREC, false, false>, kThreads, lds); break;
    default: break;
  }
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

int apply_occupancy(const DevProgram &P) {
  switch (P.prec) {
    case kFP32: return occupancy_p<kFP32>(P);
    case kBF16: return occupancy_p<kBF16>(P);
    case kFP16: return occupancy_p<kFP16>(P);
    case kSPLIT: return occupancy_p<kSPLIT>(P);
    default: return 1;
  }
}

template <int PREC>
static hipError_t launch_p(const DevProgram &P, const void *in, void *out, int64_t S,
                           hipStream_t stream, int grid_cap, bool in16, bool out16) {
  switch (P.mt) {
    case 1: return launch_mt<1, PREC>(P, in, out, S, stream, grid_cap, in16, out16);
    case 2: return launch_mt<2, PREC>(P, in, out, S, stream, grid_cap, in16, out16);
    case 4: return launch_mt<4, PREC>(P, in, out, S, stream, grid_cap, in16, out16);
    case 8: return launch_mt<8, PREC>(P, in, out, S, stream, grid_cap, in16, out16);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_apply(const DevProgram &P, const void *in, void *out, int64_t S,
                        hipStream_t stream, int grid_cap, bool in16, bool out16) {
  switch (P.prec) {
    case kFP32: return launch_p<kFP32>(P, in, out, S, stream, grid_cap, in16, out16);
    case kBF16: return launch_p<kBF16>(P, in, out, S, stream, grid_cap, in16, out16);
    case kFP16: return launch_p<kFP16>(P, in, out, S, stream, grid_cap, in16, out16);
    case kSPLIT: return launch_p<kSPLIT>(P, in, out, S, stream, grid_cap, in16, out16);
    default: return hipErrorInvalidValue;
  }
}

size_t batch_lds_bytes(int G, size_t max_program_lds, bool reg_phase) {
  // three int64 prefix arrays of G + 1 entries (rounded to even), then the program area,
  // which the register phase uses as four wave tile regions
  const size_t reg = reg_phase ? 4 * sizeof(float) * (size_t)kBatchTileWords : 0;
  return 3 * 8 * (size_t)((G + 2) & ~1) + (max_program_lds > reg ? max_program_lds : reg);
}

template <int PREC>
static hipError_t launch_batch_p(int dir, const DevProgram *progs, const UProgram *uprogs, int G,
                                 const int64_t *sig_off, int64_t total_elems, const void *in,
                                 void *out, size_t lds, int grid, int reg_groups, int cost16,
                                 hipStream_t stream) {
  return dir == 0 ? launch_batch_pd<PREC, 0, false>(progs, uprogs, G, sig_off, total_elems, in, out, lds, grid, reg_groups, cost16, stream)
                  : launch_batch_pd<PREC, 1, false>(progs, uprogs, G, sig_off, total_elems, in, out, lds, grid, reg_groups, cost16, stream);
}

int batch_occupancy(int prec, size_t lds, bool io16) {
  if (io16) return batch_occupancy_io16(prec, lds);
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define GFT_OCC(p) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gft_apply_batch<p, 0, false>, kThreads, lds)
  switch (prec) {
    case kFP32: GFT_OCC(kFP32); break;
    case kBF16: GFT_OCC(kBF16); break;
    case kFP16: GFT_OCC(kFP16); break;
    case kSPLIT: GFT_OCC(kSPLIT); break;
    default: break;
  }
#undef GFT_OCC
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

bool batch_butterfly_supported(int prec, const UProgram &U) {
  if (prec == kFP32)
    return (U.S == 1 && (U.M == 16 || U.M == 32 || (U.M == 48 && U.gen))) || (U.S == 2 && (U.M == 16 || (U.M == 32 && U.gen)));
  if (prec == kBF16) return U.gen && U.S == 1 && (U.M == 16 || U.M == 32);
  return false;
}

hipError_t launch_apply_batch(int prec, int dir, bool io16, const DevProgram *progs, const UProgram *uprogs,
                              int G, const int64_t *sig_off, int64_t total_elems, const void *in,
                              void *out, size_t lds, int grid, int reg_groups, int cost16,
                              hipStream_t stream) {
  if (cost16 < 1 || cost16 > 64) return hipErrorInvalidValue;
  if (io16)
    return launch_apply_batch_io16(prec, dir, progs, uprogs, G, sig_off, total_elems, in, out, lds, grid,
                                   reg_groups, cost16, stream);
  switch (prec) {
    case kFP32: return launch_batch_p<kFP32>(dir, progs, uprogs, G, sig_off, total_elems, in, out, lds, grid, reg_groups, cost16, stream);
    case kBF16: return launch_batch_p<kBF16>(dir, progs, uprogs, G, sig_off, total_elems, in, out, lds, grid, reg_groups, cost16, stream);
    case kFP16: return launch_batch_p<kFP16>(dir, progs, uprogs, G, sig_off, total_elems, in, out, lds, grid, reg_groups, cost16, stream);
    case kSPLIT: return launch_batch_p<kSPLIT>(dir, progs, uprogs, G, sig_off, total_elems, in, out, lds, grid, reg_groups, cost16, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gft
