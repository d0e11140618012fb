// Device code of the LDS-program engines: the generic single-graph kernel and the mixed
// batch kernel (see gft_kernels.hip), shared by the FP32-storage translation unit and the
// BF16-storage batch one (gft_batch16.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "butterfly_core.hpp"
#include "device_program.hpp"
#include "program.hpp"

namespace gft {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 halfx4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// gft_precision values (include/gft.h)
constexpr int kFP32 = 0, kBF16 = 1, kFP16 = 2, kSPLIT = 3;

// FP32 -> BF16 bits, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float floatx2_t __attribute__((ext_vector_type(2)));
// Two values rounded to BF16 in one gfx950 conversion (v_cvt_pk_bf16_f32; nearest even,
// FP32 denormals preserved: as the bit arithmetic above for every value but NaN
// payloads): a in the low half, b in the high half.
__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(floatx2_t{a, b}, bf16x2_t));
}


constexpr int kThreads = 256;
constexpr float kSqrt2f = 1.41421356237309504880f;

// e / d from magic = ceil(2^32 / d) (0 encodes d == 1); exact while e * d < 2^32.
__device__ __forceinline__ uint32_t fdiv(uint32_t e, uint32_t magic) {
  return magic ? __umulhi(e, magic) : e;
}

struct LdsTables {
  const int32_t *stages;  // 4 words per stage
  const int32_t *ops;     // 2 words per op
  const int32_t *blocks;  // 8 words per block
  const int32_t *items;
  const int32_t *gidx;
  const int32_t *sidx;
};

__device__ __forceinline__ LdsTables carve(const DevProgram &P, const int32_t *base) {
  LdsTables t;
  t.stages = base;
  t.ops = t.stages + 4 * (P.num_pre + P.num_post);
  t.blocks = t.ops + 2 * P.total_ops;
  t.items = t.blocks + 8 * P.num_blocks;
  t.gidx = t.items + P.num_items;
  t.sidx = t.gidx + P.gidx_len;
  return t;
}

// Tile loads are split in two halves so the next tile's HBM reads overlap the current
// tile's compute: issue_tile() starts up to kPrefetch vector loads per thread into
// registers; commit_tile() writes them to LDS rows of `stride` floats, loads whatever
// did not fit in registers, and zero-fills rows at and beyond count / n up to `rows`.
// A vector is 4 consecutive values: a float4 (FP32 storage) or 4 BF16 in 8 bytes (B16).
constexpr int kPrefetch = 4;

typedef uint32_t u32x2v __attribute__((ext_vector_type(2)));
template <bool B16> struct IoVec { typedef floatx4 T; };
template <> struct IoVec<true> { typedef u32x2v T; };

__device__ __forceinline__ floatx4 widen(const floatx4 &v) { return v; }
__device__ __forceinline__ floatx4 widen(const u32x2v &w) {
  return floatx4{__uint_as_float(w[0] << 16), __uint_as_float(w[0] & 0xffff0000u),
                 __uint_as_float(w[1] << 16), __uint_as_float(w[1] & 0xffff0000u)};
}

template <bool B16>
__device__ __forceinline__ float load_one(const void *g, int64_t e) {
  if constexpr (B16) return __uint_as_float((uint32_t)static_cast<const uint16_t *>(g)[e] << 16);
  else return static_cast<const float *>(g)[e];
}

template <bool B16>
__device__ __forceinline__ const void *advance_ptr(const void *g, int64_t e) {
  return B16 ? (const void *)(static_cast<const uint16_t *>(g) + e) : (const void *)(static_cast<const float *>(g) + e);
}
template <bool B16>
__device__ __forceinline__ void *advance_ptr(void *g, int64_t e) {
  return B16 ? (void *)(static_cast<uint16_t *>(g) + e) : (void *)(static_cast<float *>(g) + e);
}

// The prefetch loads are unconditional so that they stay in flight across the compute of
// the previous tile (a guarded load is waited for inside its branch): lanes past the
// tile's last vector re-read it, and a tile with no whole vector reads `spare`, 16 bytes
// of valid device memory.  commit_tile() only stores the in-range ones.
template <bool B16>
__device__ __forceinline__ void issue_tile(const void *g, int count, const floatx4 *spare,
                                           typename IoVec<B16>::T (&pre)[kPrefetch]) {
  typedef typename IoVec<B16>::T V;
  const int nvec = count >> 2;
  const V *g4 = nvec > 0 ? static_cast<const V *>(g) : reinterpret_cast<const V *>(spare);
  const int last = nvec > 0 ? nvec - 1 : 0;
#pragma unroll
  for (int k = 0; k < kPrefetch; ++k) {
    const int v = threadIdx.x + k * kThreads;
    pre[k] = __builtin_nontemporal_load(g4 + (v < last ? v : last));   // streamed once
  }
}

// LDS element of tile element e (row e / n, column e mod n) for a float4 starting at e
// that is one aligned 16-byte access: stride == n (rows packed) or 4 | n (rows aligned,
// stride n + 4; a float4 never crosses a row).
__device__ __forceinline__ bool vec_lds(int n, int stride) { return stride == n || (n & 3) == 0; }
__device__ __forceinline__ uint32_t vec_index(uint32_t e, int n, int stride, uint32_t magic_n) {
  if (stride == n) return e;
  const uint32_t r = fdiv(e, magic_n);
  return r * (uint32_t)stride + (e - r * (uint32_t)n);
}

__device__ __forceinline__ void put4(float *lds, uint32_t e, const floatx4 &val, int n,
                                     int stride, uint32_t magic_n) {
  if (vec_lds(n, stride)) {
    *reinterpret_cast<floatx4 *>(lds + vec_index(e, n, stride, magic_n)) = val;
    return;
  }
  uint32_t r = fdiv(e, magic_n);
  uint32_t c = e - r * (uint32_t)n;
  const float q[4] = {val[0], val[1], val[2], val[3]};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    lds[r * stride + c] = q[k];
    if (++c == (uint32_t)n) {
      c = 0;
      ++r;
    }
  }
}

template <bool B16>
__device__ __forceinline__ void commit_tile(const void *g, int count, int rows, int n,
                                            int stride, uint32_t magic_n,
                                            const typename IoVec<B16>::T (&pre)[kPrefetch],
                                            float *lds) {
  typedef typename IoVec<B16>::T V;
  const int tid = threadIdx.x;
  const int nvec = count >> 2;
#pragma unroll
  for (int k = 0; k < kPrefetch; ++k) {
    const int v = tid + k * kThreads;
    if (v < nvec) put4(lds, 4u * (uint32_t)v, widen(pre[k]), n, stride, magic_n);
  }
  const V *g4 = static_cast<const V *>(g);
  for (int v = tid + kPrefetch * kThreads; v < nvec; v += kThreads)
    put4(lds, 4u * (uint32_t)v, widen(__builtin_nontemporal_load(g4 + v)), n, stride, magic_n);
  for (int e = 4 * nvec + tid; e < count; e += kThreads) {
    const uint32_t r = fdiv((uint32_t)e, magic_n);
    lds[r * stride + ((uint32_t)e - r * (uint32_t)n)] = load_one<B16>(g, e);
  }
  const int full = rows * n;
  for (int e = count + tid; e < full; e += kThreads) {
    const uint32_t r = fdiv((uint32_t)e, magic_n);
    lds[r * stride + ((uint32_t)e - r * (uint32_t)n)] = 0.0f;
  }
}

template <bool B16>
__device__ __forceinline__ void store_tile(const float *lds, int count, int n, int stride,
                                           uint32_t magic_n, void *g) {
  const int tid = threadIdx.x;
  const int nvec = count >> 2;
  const bool vec = vec_lds(n, stride);
  for (int v = tid; v < nvec; v += kThreads) {
    const uint32_t e = 4u * (uint32_t)v;
    float q[4];
    if (vec) {
      const floatx4 w = *reinterpret_cast<const floatx4 *>(lds + vec_index(e, n, stride, magic_n));
      q[0] = w[0];
      q[1] = w[1];
      q[2] = w[2];
      q[3] = w[3];
    } else {
      uint32_t r = fdiv(e, magic_n);
      uint32_t c = e - r * (uint32_t)n;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        q[k] = lds[r * stride + c];
        if (++c == (uint32_t)n) {
          c = 0;
          ++r;
        }
      }
    }
    if constexpr (B16)
      __builtin_nontemporal_store(u32x2v{bf16_pair(q[0], q[1]), bf16_pair(q[2], q[3])},
                                  static_cast<u32x2v *>(g) + v);
    else
      __builtin_nontemporal_store(floatx4{q[0], q[1], q[2], q[3]}, static_cast<floatx4 *>(g) + v);
  }
  for (int e = 4 * nvec + tid; e < count; e += kThreads) {
    const uint32_t r = fdiv((uint32_t)e, magic_n);
    const float x = lds[r * stride + ((uint32_t)e - r * (uint32_t)n)];
    if constexpr (B16) static_cast<uint16_t *>(g)[e] = (uint16_t)bf16_bits(x);
    else static_cast<float *>(g)[e] = x;
  }
}

// One butterfly stage over all T rows of an LDS tile (in place).
__device__ __forceinline__ void haar_stage(const int32_t *st, const int32_t *ops, int rows,
                                           int stride, float *lds) {
  const int off = st[0];
  const int cnt = st[1];
  const uint32_t magic = (uint32_t)st[2];
  const int items = rows * cnt;
  for (int idx = threadIdx.x; idx < items; idx += kThreads) {
    const uint32_t s = fdiv((uint32_t)idx, magic);
    const int u = idx - (int)s * cnt;
    const int i = ops[2 * (off + u)];
    const int j = ops[2 * (off + u) + 1];
    float *row = lds + s * stride;
    if (j >= 0) {
      const float a = row[i], b = row[j];
      row[i] = a + b;
      row[j] = a - b;
    } else {
      row[i] *= kSqrt2f;
    }
  }
}

// Dense leaf blocks: dst[:, sidx] = src[:, gidx] * M for every block.
// MFMA operand layouts (one 16x16 block; D in both: lane l receives D[4*(l/16) + v][l%16]):
//   16x16x4 f32:  lane l supplies A[l%16][l/16] and B[l/16][l%16];
//   16x16x16 bf16/f16: lane l supplies A[l%16][4*(l/16) + j] and B[4*(l/16) + j][l%16], j < 4.
// A = signal values gathered from LDS (rows = signals), B = block-matrix fragments.
// Split precision: x = x_hi + x_lo in BF16 for both operands, three products
// hi*hi + hi*lo + lo*hi accumulated in FP32.
template <int MT, int PREC>
__device__ __forceinline__ void block_products(const DevProgram &P, const LdsTables &t,
                                               const uint32_t *fragbase, const float *src,
                                               float *dst) {
  constexpr int WPL = PREC == kFP32 ? 1 : (PREC == kSPLIT ? 4 : 2);
  constexpr int KS = PREC == kFP32 ? 4 : 16;
  const int stride = P.stride;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4;
  const int r = lane & 15;
  for (int it = wave; it < P.num_items; it += kThreads / 64) {
    const int item = t.items[it];
    const int b = item >> 16;
    const int nt = item & 0xffff;
    const int32_t *B = t.blocks + 8 * b;
    const int size = B[0], kchunks = B[1], ntiles = B[2];
    const int32_t *gi = t.gidx + B[3];
    const uint32_t *frag = fragbase + B[5] + (nt * 64 + lane) * WPL;
    floatx4 acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < kchunks; ++kc) {
      const uint32_t *fw = frag + kc * ntiles * 64 * WPL;
      if constexpr (PREC == kFP32) {
        const float bm = __uint_as_float(fw[0]);
        const int col = gi[KS * kc + g];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          const float a = src[(16 * m + r) * stride + col];
          acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bm, acc[m], 0, 0, 0);
        }
      } else {
        const u32x2 bw = {fw[0], fw[1]};
        int col[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) col[j] = gi[KS * kc + 4 * g + j];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          const float *row = src + (16 * m + r) * stride;
          float x[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) x[j] = row[col[j]];
          if constexpr (PREC == kFP16) {
            const halfx4 a = {(_Float16)x[0], (_Float16)x[1], (_Float16)x[2], (_Float16)x[3]};
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, __builtin_bit_cast(halfx4, bw),
                                                           acc[m], 0, 0, 0);
          } else {
            const uint32_t w0 = bf16_pair(x[0], x[1]), w1 = bf16_pair(x[2], x[3]);
            const bf16x4 ahi = __builtin_bit_cast(bf16x4, u32x2{w0, w1});
            const bf16x4 bhi = __builtin_bit_cast(bf16x4, bw);
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bhi, acc[m], 0, 0, 0);
            if constexpr (PREC == kSPLIT) {
              const u32x2 lw = {bf16_pair(x[0] - __uint_as_float(w0 << 16), x[1] - __uint_as_float(w0 & 0xffff0000u)),
                                bf16_pair(x[2] - __uint_as_float(w1 << 16), x[3] - __uint_as_float(w1 & 0xffff0000u))};
              const bf16x4 alo = __builtin_bit_cast(bf16x4, lw);
              const u32x2 bwl = {fw[2], fw[3]};
              const bf16x4 blo = __builtin_bit_cast(bf16x4, bwl);
              acc[m] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, blo, acc[m], 0, 0, 0);
              acc[m] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bhi, acc[m], 0, 0, 0);
            }
          }
        }
      }
    }
    const int ncol = 16 * nt + r;
    if (ncol < size) {
      const int dcol = t.sidx[B[4] + ncol];
#pragma unroll
      for (int m = 0; m < MT; ++m) {
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[(16 * m + 4 * g + v) * stride + dcol] = acc[m][v];
      }
    }
  }
}

template <int MT, int PREC, bool IN16, bool OUT16>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(MT >= 8 ? 2 : 4))) void gft_apply(
    DevProgram P, const void *in, void *out, int64_t S) {
  extern __shared__ __attribute__((aligned(16))) int32_t smem[];
  constexpr int T = 16 * MT;
  const int n = P.n;
  const int stride = P.stride;
  for (int i = threadIdx.x; i < P.table_words; i += kThreads) smem[i] = P.table[i];
  const LdsTables t = carve(P, smem);
  uint32_t *lfrag = reinterpret_cast<uint32_t *>(smem + ((P.table_words + 3) & ~3));
  if (P.frag_lds)
    for (int i = threadIdx.x; i < P.frag_words; i += kThreads) lfrag[i] = P.frag[i];
  const uint32_t *fragbase = P.frag_lds ? lfrag : P.frag;
  float *buf0 = reinterpret_cast<float *>(lfrag + (P.frag_lds ? ((P.frag_words + 3) & ~3) : 0));
  float *buf1 = buf0 + T * stride;
  const int64_t num_tiles = (S + T - 1) / T;
  auto count_of = [&](int64_t tile) {
    const int64_t rem = S - tile * T;
    return (int)(rem < T ? rem : T) * n;
  };
  typename IoVec<IN16>::T pre[kPrefetch];
  int64_t tile = blockIdx.x;
  const floatx4 *spare = reinterpret_cast<const floatx4 *>(P.table);
  if (tile < num_tiles) issue_tile<IN16>(advance_ptr<IN16>(in, tile * T * n), count_of(tile), spare, pre);
  __syncthreads();
  for (; tile < num_tiles; tile += gridDim.x) {
    const int count = count_of(tile);
    commit_tile<IN16>(advance_ptr<IN16>(in, tile * T * n), count, T, n, stride, P.magic_n, pre, buf0);
    __syncthreads();
    // next tile's loads (the last tile re-reads itself rather than branch around the loads)
    const int64_t next = tile + gridDim.x < num_tiles ? tile + gridDim.x : num_tiles - 1;
    issue_tile<IN16>(advance_ptr<IN16>(in, next * T * n), count_of(next), spare, pre);
    for (int s = 0; s < P.num_pre; ++s) {
      haar_stage(t.stages + 4 * s, t.ops, T, stride, buf0);
      __syncthreads();
    }
    block_products<MT, PREC>(P, t, fragbase, buf0, buf1);
    __syncthreads();
    for (int s = P.num_pre; s < P.num_pre + P.num_post; ++s) {
      haar_stage(t.stages + 4 * s, t.ops, T, stride, buf1);
      __syncthreads();
    }
    store_tile<OUT16>(buf1, count, n, stride, P.magic_n, advance_ptr<OUT16>(out, tile * T * n));
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------- mixed batch

// One tile of T = 16*mt signals of one program, its loads already issued into `pre`:
// commit -> (issue the next tile's loads) -> pre stages -> blocks -> post stages -> store.
// The program's tables (and fragments, when LDS-resident) are already in LDS.
template <int MT, int PREC, bool IO16>
__device__ __forceinline__ void run_tile(const DevProgram &P, const LdsTables &t,
                                         const uint32_t *fragbase, const void *gin,
                                         void *gout, int count, float *buf0, float *buf1,
                                         typename IoVec<IO16>::T (&pre)[kPrefetch], const void *next_in,
                                         int next_count, const floatx4 *spare) {
  constexpr int T = 16 * MT;
  commit_tile<IO16>(gin, count, T, P.n, P.stride, P.magic_n, pre, buf0);
  __syncthreads();
  issue_tile<IO16>(next_in, next_count, spare, pre);
  for (int s = 0; s < P.num_pre; ++s) {
    haar_stage(t.stages + 4 * s, t.ops, T, P.stride, buf0);
    __syncthreads();
  }
  block_products<MT, PREC>(P, t, fragbase, buf0, buf1);
  __syncthreads();
  for (int s = P.num_pre; s < P.num_pre + P.num_post; ++s) {
    haar_stage(t.stages + 4 * s, t.ops, T, P.stride, buf1);
    __syncthreads();
  }
  store_tile<IO16>(buf1, count, P.n, P.stride, P.magic_n, gout);
  __syncthreads();
}

// Register-butterfly programs the batch kernel runs (FP32 blocks; BF16 blocks on the
// padded one-stage layout): S = 1 with M = 16, 32 or 48 (48: padded layout), S = 2 with
// M = 16 (uniform or padded) or 32 (padded).  The 48- and 32-slot padded forms run the lean
// tile loop (packed offsets, no next-tile prefetch), which keeps the kernel at 256 VGPRs;
// the two-stage 32-slot form still spills a little in its own path (measured: the batch
// is faster with it than with those grids on their LDS programs).
constexpr int kBatchTileWords = bfly::tile_words<2, 32>();   // the largest of these
// Held to two waves per SIMD by the largest forms, the FP32 kernel keeps HBM busy on the
// small forms by loading further ahead: 4 tiles for the one-stage 16-slot blocks, 3 for
// the 64-slot forms (measured on the mixed batch: 199 -> 193 us).  The BF16 kernel (three
// waves per SIMD) keeps one.
constexpr int kPfSmall = 4, kPfMid = 3;
template <int PREC, int DIR, bool IO>
__device__ __forceinline__ void batch_butterfly(const UProgram &U, const void *in, void *out,
                                                int64_t nsig, int64_t t0, int64_t t1, float *T) {
  if constexpr (PREC == kFP32) {
    if (U.S == 1 && U.M == 16) {
      if (U.gen) bfly::butterfly_tiles<1, 16, DIR, IO, IO, true, false, false, kPfSmall>(U, in, out, nsig, t0, t1, 1, T);
      else bfly::butterfly_tiles<1, 16, DIR, IO, IO, false, false, false, kPfSmall>(U, in, out, nsig, t0, t1, 1, T);
    } else if (U.S == 1 && U.M == 32) {
      if (U.gen) bfly::butterfly_tiles<1, 32, DIR, IO, IO, true, false, false, kPfMid>(U, in, out, nsig, t0, t1, 1, T);
      else bfly::butterfly_tiles<1, 32, DIR, IO, IO, false, false, false, kPfMid>(U, in, out, nsig, t0, t1, 1, T);
    } else if (U.S == 1 && U.M == 48 && U.gen) {
      bfly::butterfly_tiles<1, 48, DIR, IO, IO, true, false, true>(U, in, out, nsig, t0, t1, 1, T);
    } else if (U.S == 2 && U.M == 32 && U.gen) {
      bfly::butterfly_tiles<2, 32, DIR, IO, IO, true, false, true>(U, in, out, nsig, t0, t1, 1, T);
    } else if (U.S == 2 && U.M == 16) {
      if (U.gen) bfly::butterfly_tiles<2, 16, DIR, IO, IO, true, false, false, kPfMid>(U, in, out, nsig, t0, t1, 1, T);
      else bfly::butterfly_tiles<2, 16, DIR, IO, IO, false, false, false, kPfMid>(U, in, out, nsig, t0, t1, 1, T);
    }
  } else if constexpr (PREC == kBF16) {
    if (U.gen && U.S == 1 && U.M == 16)
      bfly::butterfly_tiles<1, 16, DIR, IO, IO, true, true>(U, in, out, nsig, t0, t1, 1, T);
    else if (U.gen && U.S == 1 && U.M == 32)
      bfly::butterfly_tiles<1, 32, DIR, IO, IO, true, true>(U, in, out, nsig, t0, t1, 1, T);
  }
}

// Cost of one signal in the register phase, in element-equivalents: a 16-signal tile takes
// about the longer of its HBM traffic (n values) and a fixed part that grows with the
// padded slot count N = M 2^S: cost16 N / 16 values' worth of traffic (measured per graph
// shape on this kernel: about 11; the plan-time tuner may pick another).
__device__ __forceinline__ int64_t reg_cost(const UProgram &U, int cost16) {
  const int fixed = (cost16 * (U.M << U.S)) / 16;
  return U.n > fixed ? U.n : fixed;
}

// Many graphs in one persistent launch.  Graph g owns signals [off[g], off[g+1]) and its
// data starts at element elem[g] = sum_{h<g} (off[h+1]-off[h]) * n_h of in/out; each
// workgroup first rebuilds elem[] in LDS from the device offsets (no host sync, no
// workspace), together with prefix sums over the graphs each engine serves: the cost
// (reg_cost per signal) of those with a register-butterfly program (uprogs[g].S > 0, or none
// when uprogs is null) and the elements of the rest.
//   Register phase: the waves of the first reg_groups workgroups split the first class's
//   cost into contiguous, equal shares; a wave runs the 16-signal tiles whose first signal's
//   cost offset lies in its share, graph by graph, through the butterfly tile loop.
//   LDS-program phase: every workgroup takes the tiles (16 * mt signals) of the other
//   graphs whose first element lies in its 1/gridDim share of their elements, and reloads
//   a program's tables into LDS only when it moves to another graph.
// Graphs whose data would end past total_elems are skipped.
template <int PREC, int DIR, bool IO16>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void gft_apply_batch(
    const DevProgram *__restrict__ progs, const UProgram *__restrict__ uprogs, int G,
    const int64_t *__restrict__ sig_off, int64_t total_elems, const void *in, void *out,
    int reg_groups, int cost16) {
  extern __shared__ __attribute__((aligned(16))) int32_t smem[];
  const int GP = (G + 2) & ~1;                                 // G + 1 rounded to even
  int64_t *elem = reinterpret_cast<int64_t *>(smem);           // all graphs
  int64_t *elemR = elem + GP;                                  // register-program graphs (cost)
  int64_t *elemL = elemR + GP;                                 // LDS-program graphs
  int32_t *area = smem + 6 * GP;                               // program area / tiles
  // per-thread partial sums over contiguous chunks of graphs, an exclusive scan of the
  // kThreads partials (inclusive scans inside each wave by shuffles, then the wave totals),
  // and a second pass writing the prefix arrays
  __shared__ int64_t wsum[3][kThreads / 64];
  const int per = (G + kThreads - 1) / kThreads;
  const int g0 = threadIdx.x * per, g1 = g0 + per < G ? g0 + per : G;
  // elements of graph g, and its register-phase cost (0 for the LDS-program class)
  auto elems = [&](int g, int64_t &cost) -> int64_t {
    const int64_t ns = sig_off[g + 1] - sig_off[g];
    const int64_t s = ns > 0 ? ns : 0;
    cost = (uprogs != nullptr && uprogs[g].S > 0) ? s * reg_cost(uprogs[g], cost16) : 0;
    return s * (int64_t)progs[g].n;
  };
  int64_t accA = 0, accR = 0, accL = 0;
  for (int g = g0; g < g1; ++g) {
    int64_t c;
    const int64_t e = elems(g, c);
    accA += e;
    accR += c;
    if (c == 0) accL += e;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t incA = accA, incR = accR, incL = accL;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t oA = __shfl_up(incA, d, 64), oR = __shfl_up(incR, d, 64), oL = __shfl_up(incL, d, 64);
    if (lane >= d) {
      incA += oA;
      incR += oR;
      incL += oL;
    }
  }
  if (lane == 63) {
    wsum[0][wave] = incA;
    wsum[1][wave] = incR;
    wsum[2][wave] = incL;
  }
  __syncthreads();
  int64_t baseA = 0, baseR = 0, baseL = 0;
  for (int w = 0; w < wave; ++w) {
    baseA += wsum[0][w];
    baseR += wsum[1][w];
    baseL += wsum[2][w];
  }
  accA = baseA + incA - accA;                                  // exclusive prefixes
  accR = baseR + incR - accR;
  accL = baseL + incL - accL;
  for (int g = g0; g < g1; ++g) {
    elem[g] = accA;
    elemR[g] = accR;
    elemL[g] = accL;
    int64_t c;
    const int64_t e = elems(g, c);
    accA += e;
    accR += c;
    if (c == 0) accL += e;
  }
  if (threadIdx.x == kThreads - 1) {
    elem[G] = accA;
    elemR[G] = accR;
    elemL[G] = accL;
  }
  __syncthreads();

  // ---- register phase
  if (uprogs != nullptr && (int)blockIdx.x < reg_groups) {
    const int64_t ER = elemR[G];
    const int64_t W = (int64_t)reg_groups * 4;
    const int64_t w = (int64_t)blockIdx.x * 4 + wave;
    const int64_t e0 = (int64_t)(((__int128)ER * w) / W);
    const int64_t e1 = (int64_t)(((__int128)ER * (w + 1)) / W);
    if (e0 < e1) {
      // graph holding cost offset e0 of the class: last g with elemR[g] <= e0
      int lo = 0, hi = G;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (elemR[mid] <= e0) lo = mid;
        else hi = mid;
      }
      float *T = reinterpret_cast<float *>(area) + wave * kBatchTileWords;
      for (int g = lo; g < G && elemR[g] < e1; ++g) {
        const int64_t gb = elemR[g], ge = elemR[g + 1];
        if (ge <= gb || elem[g + 1] > total_elems) continue;
        const UProgram U = uprogs[g];
        const int64_t cs = reg_cost(U, cost16), te = 16 * cs;  // cost per signal, per tile
        const int64_t t0 = e0 > gb ? (e0 - gb + te - 1) / te : 0;
        const int64_t t1 = ((e1 < ge ? e1 : ge) - gb + te - 1) / te;
        if (t0 < t1)
          batch_butterfly<PREC, DIR, IO16>(U, advance_ptr<IO16>(in, elem[g]), advance_ptr<IO16>(out, elem[g]),
                                           (ge - gb) / cs, t0, t1, T);
      }
    }
  }
  __syncthreads();   // the LDS-program phase reuses the tile regions

  // ---- LDS-program phase
  const int64_t E = elemL[G];
  const int64_t W = gridDim.x;
  const int64_t e0 = (int64_t)(((__int128)E * blockIdx.x) / W);
  const int64_t e1 = (int64_t)(((__int128)E * (blockIdx.x + 1)) / W);
  if (e0 >= e1) return;
  // graph holding element e0 of the class: last g with elemL[g] <= e0
  int lo = 0, hi = G;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (elemL[mid] <= e0) lo = mid;
    else hi = mid;
  }
  // The tiles this workgroup owns (first element in [e0, e1) of the class), in order:
  // (g, t) pairs.  advance() moves (g, t) to the next owned tile at or after it and returns
  // false when there is none; graphs that are empty, of the other class, or end past
  // total_elems are skipped.
  auto advance = [&](int &g, int64_t &t) -> bool {
    while (g < G) {
      const int64_t gbeg = elemL[g], gend = elemL[g + 1];
      if (gend <= gbeg || elem[g + 1] > total_elems) {
        ++g;
        t = 0;
        if (elemL[g < G ? g : G] >= e1) return false;
        continue;
      }
      const int64_t tile_elems = (int64_t)16 * progs[g].mt * progs[g].n;
      if (t < 0) t = (e0 - gbeg + tile_elems - 1) / tile_elems;   // first tile starting >= e0
      const int64_t start = gbeg + t * tile_elems;
      if (start >= gend) {   // this graph has no tile left for us: the next one may
        ++g;
        t = 0;
        continue;
      }
      return start < e1;
    }
    return false;
  };
  // element offset in in/out and element count of tile t of graph g
  auto span = [&](int g, int64_t t, int64_t &start) -> int {
    const int64_t tile_elems = (int64_t)16 * progs[g].mt * progs[g].n;
    start = elem[g] + t * tile_elems;
    const int64_t rem = elem[g + 1] - start;
    return (int)(rem < tile_elems ? rem : tile_elems);
  };
  int g = lo;
  int64_t t = -1;
  if (!advance(g, t)) return;
  const floatx4 *spare = reinterpret_cast<const floatx4 *>(progs[0].table);
  typename IoVec<IO16>::T pre[kPrefetch];
  int64_t start;
  int count = span(g, t, start);
  issue_tile<IO16>(advance_ptr<IO16>(in, start), count, spare, pre);
  int loaded = -1;
  DevProgram P{};
  LdsTables tabs{};
  const uint32_t *fragbase = nullptr;
  float *buf0 = nullptr, *buf1 = nullptr;
  for (;;) {
    if (loaded != g) {
      P = progs[g];
      for (int i = threadIdx.x; i < P.table_words; i += kThreads) area[i] = P.table[i];
      tabs = carve(P, area);
      uint32_t *lfrag = reinterpret_cast<uint32_t *>(area + ((P.table_words + 3) & ~3));
      if (P.frag_lds)
        for (int i = threadIdx.x; i < P.frag_words; i += kThreads) lfrag[i] = P.frag[i];
      fragbase = P.frag_lds ? lfrag : P.frag;
      buf0 = reinterpret_cast<float *>(lfrag + (P.frag_lds ? ((P.frag_words + 3) & ~3) : 0));
      buf1 = buf0 + 16 * P.mt * P.stride;
      loaded = g;
      __syncthreads();
    }
    // the next owned tile, whose loads run while this one is computed (the last tile
    // re-reads itself rather than branch around the loads)
    int ng = g;
    int64_t nt = t + 1;
    const bool more = advance(ng, nt);
    int64_t nstart = start;
    const int ncount = more ? span(ng, nt, nstart) : count;
    const void *gi = advance_ptr<IO16>(in, start), *gn = advance_ptr<IO16>(in, nstart);
    void *go = advance_ptr<IO16>(out, start);
    switch (P.mt) {
      case 1: run_tile<1, PREC, IO16>(P, tabs, fragbase, gi, go, count, buf0, buf1, pre, gn, ncount, spare); break;
      case 2: run_tile<2, PREC, IO16>(P, tabs, fragbase, gi, go, count, buf0, buf1, pre, gn, ncount, spare); break;
      case 4: run_tile<4, PREC, IO16>(P, tabs, fragbase, gi, go, count, buf0, buf1, pre, gn, ncount, spare); break;
      default: run_tile<8, PREC, IO16>(P, tabs, fragbase, gi, go, count, buf0, buf1, pre, gn, ncount, spare); break;
    }
    if (!more) break;
    g = ng;
    t = nt;
    start = nstart;
    count = ncount;
  }
}

// ---------------------------------------------------------------------------- batch launch

template <int PREC, int DIR, bool IO16>
static hipError_t launch_batch_pd(const DevProgram *progs, const UProgram *uprogs, int G,
                                  const int64_t *sig_off, int64_t total_elems, const void *in,
                                  void *out, size_t lds, int grid, int reg_groups, int cost16,
                                  hipStream_t stream) {
  if (lds + 24 * (kThreads / 64) > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)gft_apply_batch<PREC, DIR, IO16>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((gft_apply_batch<PREC, DIR, IO16>), dim3(grid), dim3(kThreads), lds, stream, progs,
                     uprogs, G, sig_off, total_elems, in, out, reg_groups, cost16);
  return hipGetLastError();
}

}  // namespace gft
