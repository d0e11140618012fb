// Streaming copy (gfx950): the reference for what a kernel that only moves its data through
// HBM reaches on this part, quoted beside the GFT kernels' rooflines.  Each thread moves
// four 16-byte groups per grid-stride step with non-temporal loads and stores, the same
// access kind the transform kernels use for signal data.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace gft {

namespace {
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyThreads = 256, kCopyUnroll = 4;

__global__ __launch_bounds__(kCopyThreads) void stream_copy(const u32x4 *__restrict__ in,
                                                             u32x4 *__restrict__ out, int64_t n16) {
  const int64_t step = (int64_t)gridDim.x * kCopyThreads * kCopyUnroll;
  for (int64_t base = (int64_t)blockIdx.x * kCopyThreads * kCopyUnroll + threadIdx.x; base < n16;
       base += step) {
    u32x4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const int64_t i = base + (int64_t)u * kCopyThreads;
      v[u] = i < n16 ? __builtin_nontemporal_load(in + i) : u32x4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const int64_t i = base + (int64_t)u * kCopyThreads;
      if (i < n16) __builtin_nontemporal_store(v[u], out + i);
    }
  }
}
}  // namespace

// bytes: a multiple of 16; in, out: 16-byte aligned, not overlapping (checked by the caller).
// 64 workgroups per CU at most (the fastest grid measured for large copies).
hipError_t launch_stream_copy(const void *in, void *out, int64_t bytes, hipStream_t stream,
                              int num_cus) {
  const int64_t n16 = bytes / 16;
  const int64_t per = (int64_t)kCopyThreads * kCopyUnroll;
  const int64_t want = (n16 + per - 1) / per;
  const int64_t cap = (int64_t)64 * (num_cus > 0 ? num_cus : 1);
  const int grid = (int)(want < cap ? want : cap);
  hipLaunchKernelGGL(stream_copy, dim3(grid > 0 ? grid : 1), dim3(kCopyThreads), 0, stream,
                     static_cast<const u32x4 *>(in), static_cast<u32x4 *>(out), n16);
  return hipGetLastError();
}

}  // namespace gft
