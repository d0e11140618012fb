// Large-signal GFT engine for gfx950: permutation/stage pass and grouped leaf-block GEMM.
//
// For signals too long to stage a tile of 16 in LDS (n in the thousands) and for large leaf
// blocks (hundreds of nodes), the leaf products are real contractions [S x b] * [b x b]:
// they run as MFMA GEMM tiles over a block-contiguous workspace, with the Haar stages and
// the output-order permutation in separate streaming passes.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_program.hpp"

namespace gft {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;
constexpr float kSqrt2f = 1.41421356237309504880f;

__device__ __forceinline__ uint32_t bf16_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ bf16x4 pack_bf16(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  const u32x2 w = {a | (b << 16), c | (d << 16)};
  return __builtin_bit_cast(bf16x4, w);
}

}  // namespace

// ---------------------------------------------------------------------------- pass 1/3

// Rows of `rows` signals per tile: tile[r][j] = in[r * ld_in + (scatter-inverse) ...].
// The pass is given in gather form on both sides:
//   load:  tile[r][j] = gin[j] < 0 ? 0 : in[r * ld_in + gin[j]]        (j < n_tile)
//   store: out[r * ld_out + c] = gout[c] < 0 ? 0 : tile[r][gout[c]]    (c < out_cols)
// (gin / gout null = identity).  With no stages the tile is skipped altogether: each
// output element gathers its input directly (a row is a few KB, so the gathered reads stay
// in L2 while writes are coalesced).
__global__ __launch_bounds__(kThreads) void gft_permute_stages(PermPass P, const float *in,
                                                               float *out, int64_t S,
                                                               int rows, int stride) {
  const int tid = threadIdx.x;
  if (P.num_stages == 0) {
    const int64_t total = S * (int64_t)P.out_cols;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + tid; e < total; e += (int64_t)gridDim.x * kThreads) {
      const int64_t r = e / P.out_cols;
      const int c = (int)(e - r * P.out_cols);
      const int src = P.gather ? P.gather[c] : c;
      out[r * P.ld_out + c] = src >= 0 ? in[r * P.ld_in + src] : 0.0f;
    }
    return;
  }
  extern __shared__ float tile[];
  const int64_t ntiles = (S + rows - 1) / rows;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t r0 = t * rows;
    const int nr = (int)((S - r0) < rows ? (S - r0) : rows);
    for (int idx = tid; idx < nr * P.n_tile; idx += kThreads) {
      const int r = idx / P.n_tile, j = idx - r * P.n_tile;
      const int src = P.scatter ? P.scatter[j] : j;
      tile[r * stride + j] = src >= 0 ? in[(r0 + r) * (int64_t)P.ld_in + src] : 0.0f;
    }
    __syncthreads();
    for (int s = 0; s < P.num_stages; ++s) {
      const int off = P.stages[2 * s], cnt = P.stages[2 * s + 1];
      for (int idx = tid; idx < nr * cnt; idx += kThreads) {
        const int r = idx / cnt, u = idx - r * cnt;
        const int i = P.ops[2 * (off + u)], j = P.ops[2 * (off + u) + 1];
        float *row = tile + r * stride;
        if (j >= 0) {
          const float a = row[i], b = row[j];
          row[i] = a + b;
          row[j] = a - b;
        } else {
          row[i] *= kSqrt2f;
        }
      }
      __syncthreads();
    }
    for (int idx = tid; idx < nr * P.out_cols; idx += kThreads) {
      const int r = idx / P.out_cols, c = idx - r * P.out_cols;
      const int g = P.gather ? P.gather[c] : c;
      out[(r0 + r) * (int64_t)P.ld_out + c] = g >= 0 ? tile[r * stride + g] : 0.0f;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------- pass 2

// Grouped GEMM over leaf blocks: C[:, col_b + j] = sum_k A[:, col_b + k] * M_b[k][j].
// Workgroup tile 128 signals x 128 columns, K step 16, four waves of 64 x 64 each
// (4 x 4 MFMA 16x16 tiles).  A and B tiles are prefetched into registers while the
// previous tile is multiplied out of LDS (A stored k-major so that MFMA operand reads are
// conflict-free); the prefetch is unconditional (the last tile is re-read) because loads
// under a branch are waited for inside it.  PREC: 0 = FP32 (16x16x4 f32), 1 = BF16, 3 = split BF16 hi+lo (16x16x16
// bf16; three products for split).
constexpr int kBM = 128, kBN = 128, kBK = 16, kPad = 4;

template <int PREC>
__global__ __launch_bounds__(kThreads) void gft_block_gemm(const LBlock *__restrict__ blocks,
                                                           int nblocks, const float *mats,
                                                           const float *A, float *C, int64_t S,
                                                           int ld) {
  __shared__ __attribute__((aligned(16))) float As[kBK][kBM + kPad];
  __shared__ __attribute__((aligned(16))) float Bs[kBK][kBN + kPad];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, g = lane >> 4, r = lane & 15;
  const int wm = wave >> 1, wn = wave & 1;
  // locate (block, m tile, n tile) of this workgroup
  const int64_t mtiles = (S + kBM - 1) / kBM;
  int64_t id = blockIdx.x;
  int b = 0;
  for (; b < nblocks; ++b) {
    const int64_t nt = (blocks[b].size + kBN - 1) / kBN;
    if (id < mtiles * nt) break;
    id -= mtiles * nt;
  }
  if (b >= nblocks) return;
  const LBlock blk = blocks[b];
  const int ntb = (blk.size + kBN - 1) / kBN;
  const int64_t row0 = (id / ntb) * kBM;
  const int col0 = (int)(id % ntb) * kBN;
  const int K = blk.size;
  const float *Ab = A + blk.col;
  const float *Bm = mats + blk.mat;

  // register prefetch of one K tile: A 128x16 (2 float4 per thread), B 16x128 (2 float4)
  floatx4 ra[2], rb[2];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int idx = tid + kThreads * i;
      const int m = idx >> 2, kq = (idx & 3) * 4;
      int64_t row = row0 + m;
      row = row < S ? row : S - 1;                         // clamped: never stored
      const int k = k0 + kq;
      floatx4 v = *reinterpret_cast<const floatx4 *>(Ab + row * ld + (k < K ? k : 0));
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (k + j >= K) v[j] = 0.0f;
      ra[i] = v;
      const int kb = idx >> 5, nq = (idx & 31) * 4;
      const int kr = k0 + kb < K ? k0 + kb : K - 1;
      const int c = col0 + nq;
      floatx4 w = *reinterpret_cast<const floatx4 *>(Bm + (int64_t)kr * blk.ld + (c < blk.ld ? c : 0));
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (k0 + kb >= K || c + j >= K) w[j] = 0.0f;
      rb[i] = w;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int idx = tid + kThreads * i;
      const int m = idx >> 2, kq = (idx & 3) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) As[kq + j][m] = ra[i][j];
      const int kb = idx >> 5, nq = (idx & 31) * 4;
      *reinterpret_cast<floatx4 *>(&Bs[kb][nq]) = rb[i];
    }
  };

  floatx4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int nk = (K + kBK - 1) / kBK;
  load(0);
  for (int kt = 0; kt < nk; ++kt) {
    store();
    __syncthreads();
    load((kt + 1 < nk ? kt + 1 : kt) * kBK);   // unconditional: see the prefetch note
    if constexpr (PREC == 0) {
#pragma unroll
      for (int kk = 0; kk < kBK / 4; ++kk) {
        float a[4], bb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = As[4 * kk + g][wm * 64 + 16 * i + r];
#pragma unroll
        for (int j = 0; j < 4; ++j) bb[j] = Bs[4 * kk + g][wn * 64 + 16 * j + r];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], bb[j], acc[i][j], 0, 0, 0);
      }
    } else {
      // 16x16x16 bf16: lane (g, r) supplies A[r][4g + q] and B[4g + q][r], q < 4
      bf16x4 ahi[4], alo[4], bhi[4], blo[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        uint32_t h[4], l[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float x = As[4 * g + q][wm * 64 + 16 * i + r];
          h[q] = bf16_bits(x);
          l[q] = bf16_bits(x - __uint_as_float(h[q] << 16));
        }
        ahi[i] = pack_bf16(h[0], h[1], h[2], h[3]);
        alo[i] = pack_bf16(l[0], l[1], l[2], l[3]);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        uint32_t h[4], l[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float x = Bs[4 * g + q][wn * 64 + 16 * j + r];
          h[q] = bf16_bits(x);
          l[q] = bf16_bits(x - __uint_as_float(h[q] << 16));
        }
        bhi[j] = pack_bf16(h[0], h[1], h[2], h[3]);
        blo[j] = pack_bf16(l[0], l[1], l[2], l[3]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi[i], bhi[j], acc[i][j], 0, 0, 0);
          if constexpr (PREC == 3) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi[i], blo[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo[i], bhi[j], acc[i][j], 0, 0, 0);
          }
        }
    }
    __syncthreads();
  }
  // epilogue: lane (g, r) holds rows 4g + v, column r of each 16x16 tile
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = col0 + wn * 64 + 16 * j + r;
      if (c >= K) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + wm * 64 + 16 * i + 4 * g + v;
        if (row < S) C[row * ld + blk.col + c] = acc[i][j][v];
      }
    }
}

// ---------------------------------------------------------------------------- launch

hipError_t launch_permute_stages(const PermPass &P, const float *in, float *out, int64_t S,
                                 int rows, int stride, int grid, hipStream_t stream) {
  const size_t lds = P.num_stages ? (size_t)rows * stride * 4 : 0;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)gft_permute_stages,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(gft_permute_stages, dim3(grid), dim3(kThreads), lds, stream, P, in, out, S,
                     rows, stride);
  return hipGetLastError();
}

int64_t block_gemm_grid(const int32_t *sizes, int nblocks, int64_t S) {
  const int64_t mtiles = (S + kBM - 1) / kBM;
  int64_t tiles = 0;
  for (int b = 0; b < nblocks; ++b) tiles += mtiles * ((sizes[b] + kBN - 1) / kBN);
  return tiles;
}

hipError_t launch_block_gemm(int prec, const LBlock *blocks, int nblocks, const float *mats,
                             const float *A, float *C, int64_t S, int ld, int64_t grid,
                             hipStream_t stream) {
  if (grid <= 0) return hipSuccess;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  switch (prec) {
    case 0: hipLaunchKernelGGL(gft_block_gemm<0>, dim3((unsigned)grid), dim3(kThreads), 0, stream,
                               blocks, nblocks, mats, A, C, S, ld); break;
    case 1: hipLaunchKernelGGL(gft_block_gemm<1>, dim3((unsigned)grid), dim3(kThreads), 0, stream,
                               blocks, nblocks, mats, A, C, S, ld); break;
    case 3: hipLaunchKernelGGL(gft_block_gemm<3>, dim3((unsigned)grid), dim3(kThreads), 0, stream,
                               blocks, nblocks, mats, A, C, S, ld); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gft
