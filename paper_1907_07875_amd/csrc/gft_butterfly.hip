// Register-butterfly GFT kernel for one graph (gfx950): the tile loop of butterfly_core.hpp
// over a grid-stride range of 16-signal tiles.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "butterfly_core.hpp"
#include "device_program.hpp"

namespace gft {

namespace {
constexpr int kWaves = 4;
}  // namespace

template <int S, int M, int DIR, bool IN16, bool OUT16, bool GEN, bool BF>
__global__ __launch_bounds__(64 * kWaves) void gft_butterfly_f32(UProgram P, const void *in,
                                                                 void *out, int64_t nsig) {
  constexpr int TW = bfly::tile_words<S, M>();
  __shared__ __attribute__((aligned(16))) float lds_all[kWaves * TW];
  const int wave = threadIdx.x >> 6;
  bfly::butterfly_tiles<S, M, DIR, IN16, OUT16, GEN, BF>(
      P, in, out, nsig, (int64_t)blockIdx.x * kWaves + wave, (nsig + 15) / 16,
      (int64_t)gridDim.x * kWaves, lds_all + wave * TW);
}

// ---------------------------------------------------------------------------- launch

// grid_cap > 0: launch at most that many workgroups (the tile loop strides over the rest);
// 0: every resident workgroup (occupancy x CUs).  num_cus < 0: only report the occupancy
// (returned through *occ_out) without launching.
template <int S, int M, int DIR, bool IN16, bool OUT16, bool GEN, bool BF>
static hipError_t launch_bf(const UProgram &P, const void *in, void *out, int64_t nsig,
                            hipStream_t stream, int num_cus, int grid_cap, int *occ_out) {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, gft_butterfly_f32<S, M, DIR, IN16, OUT16, GEN, BF>,
                                                   64 * kWaves, 0) != hipSuccess || occ < 1)
    occ = 1;
  if (occ_out) *occ_out = occ;
  if (num_cus < 0) return hipSuccess;
  const int64_t ntiles = (nsig + 15) / 16;
  const int64_t want = (ntiles + kWaves - 1) / kWaves;
  const int64_t cap = grid_cap > 0 ? grid_cap : (int64_t)occ * (num_cus > 0 ? num_cus : 1);
  const int grid = (int)(want < cap ? want : cap);
  hipLaunchKernelGGL((gft_butterfly_f32<S, M, DIR, IN16, OUT16, GEN, BF>), dim3(grid > 0 ? grid : 1),
                     dim3(64 * kWaves), 0, stream, P, in, out, nsig);
  return hipGetLastError();
}

template <int S, int M, int DIR, bool GEN, bool BF>
static hipError_t launch_bf_io(const UProgram &P, const void *in, void *out, int64_t nsig,
                               hipStream_t stream, int num_cus, bool in16, bool out16, int grid_cap,
                               int *occ_out) {
  if (in16)
    return out16 ? launch_bf<S, M, DIR, true, true, GEN, BF>(P, in, out, nsig, stream, num_cus, grid_cap, occ_out)
                 : launch_bf<S, M, DIR, true, false, GEN, BF>(P, in, out, nsig, stream, num_cus, grid_cap, occ_out);
  return out16 ? launch_bf<S, M, DIR, false, true, GEN, BF>(P, in, out, nsig, stream, num_cus, grid_cap, occ_out)
               : launch_bf<S, M, DIR, false, false, GEN, BF>(P, in, out, nsig, stream, num_cus, grid_cap, occ_out);
}

bool butterfly_supported(const UProgram &P) { return butterfly_shape_compiled(P.S, P.M, P.gen != 0); }

static hipError_t dispatch_bf(const UProgram &P, const void *in, void *out, int64_t nsig,
                              hipStream_t stream, int num_cus, bool in16, bool out16, int grid_cap,
                              int *occ_out) {
#define GFT_BF_CASE(s, m, pad, bf)                                                                   \
  if (P.S == s && P.M == m && (P.gen != 0) == pad && (P.prec != 0) == bf)                           \
    return P.dir == 0                                                                                \
               ? launch_bf_io<s, m, 0, pad, bf>(P, in, out, nsig, stream, num_cus, in16, out16, grid_cap, occ_out) \
               : launch_bf_io<s, m, 1, pad, bf>(P, in, out, nsig, stream, num_cus, in16, out16, grid_cap, occ_out);
  GFT_BF_CASE(1, 16, false, false)
  GFT_BF_CASE(1, 32, false, false)
  GFT_BF_CASE(2, 16, false, false)
  GFT_BF_CASE(3, 16, false, false)
  GFT_BF_CASE(1, 16, true, false)
  GFT_BF_CASE(1, 32, true, false)
  GFT_BF_CASE(1, 16, true, true)
  GFT_BF_CASE(1, 32, true, true)
  GFT_BF_CASE(1, 48, true, false)
  GFT_BF_CASE(2, 16, true, false)
  GFT_BF_CASE(2, 32, true, false)
  GFT_BF_CASE(1, 48, true, true)
#undef GFT_BF_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_butterfly(const UProgram &P, const void *in, void *out, int64_t nsig,
                            hipStream_t stream, int num_cus, bool in16, bool out16, int grid_cap) {
  return dispatch_bf(P, in, out, nsig, stream, num_cus, in16, out16, grid_cap, nullptr);
}

int butterfly_occupancy(const UProgram &P, bool in16, bool out16) {
  int occ = 1;
  if (dispatch_bf(P, nullptr, nullptr, 0, nullptr, -1, in16, out16, 0, &occ) != hipSuccess) return 1;
  return occ;
}

}  // namespace gft
