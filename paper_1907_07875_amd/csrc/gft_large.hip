// Large-signal GFT engine for gfx950: permutation/stage pass and grouped leaf-block GEMM.
//
// For signals too long to stage a tile of 16 in LDS (n in the thousands) and for large leaf
// blocks (hundreds of nodes), the leaf products are real contractions [S x b] * [b x b]:
// they run as MFMA GEMM tiles over a block-contiguous workspace, with the Haar stages and
// the output-order permutation in separate streaming passes.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "device_program.hpp"
#include "launch.hpp"

namespace gft {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

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

// One tile = `rows` consecutive signal rows.  Rows are contiguous in memory and in LDS
// (tile row stride = in_cols), so the load is a straight copy of rows x in_cols floats
// (float4 when in_cols is a multiple of 4).  Each Haar op is then applied to every row of
// the tile by one thread (the ops of a stage are disjoint), and the store gathers each
// output column from its tile column, threads owning columns (float4 stores when out_cols
// is a multiple of 4) so each index-table entry is read once per tile.  OUT16: the output
// is rounded to BF16 (round to nearest even): the workspace of BF16 leaf blocks, or BF16
// storage of the result.  IN16: the input rows hold BF16 values (BF16 storage), widened
// exactly into the FP32 tile.
template <bool IN16, bool OUT16>
__global__ __launch_bounds__(kThreads) void gft_permute_stages(PermPass P, const void *in_raw,
                                                               void *out_raw, int64_t S,
                                                               int rows) {
  extern __shared__ __attribute__((aligned(16))) float tile[];
  const int tid = threadIdx.x;
  const int ic = P.in_cols, oc = P.out_cols;
  const int64_t ntiles = (S + rows - 1) / rows;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t r0 = t * rows;
    const int nr = (int)((S - r0) < rows ? (S - r0) : rows);
    // load
    const float *src = static_cast<const float *>(in_raw) + r0 * ic;
    if constexpr (IN16) {
      const uint16_t *s16 = static_cast<const uint16_t *>(in_raw) + r0 * ic;
      if ((ic & 7) == 0) {
        const int tot = nr * (ic >> 3);
        const u32x4 *s8 = reinterpret_cast<const u32x4 *>(s16);
        for (int e = tid; e < tot; e += kThreads) {
          const u32x4 w = __builtin_nontemporal_load(s8 + e);
          floatx4 *t4 = reinterpret_cast<floatx4 *>(tile + 8 * e);
          t4[0] = floatx4{__uint_as_float(w[0] << 16), __uint_as_float(w[0] & 0xffff0000u),
                          __uint_as_float(w[1] << 16), __uint_as_float(w[1] & 0xffff0000u)};
          t4[1] = floatx4{__uint_as_float(w[2] << 16), __uint_as_float(w[2] & 0xffff0000u),
                          __uint_as_float(w[3] << 16), __uint_as_float(w[3] & 0xffff0000u)};
        }
      } else {
        const int tot = nr * ic;
        for (int e = tid; e < tot; e += kThreads) tile[e] = __uint_as_float((uint32_t)s16[e] << 16);
      }
    } else if ((ic & 3) == 0) {
      const int tot = nr * (ic >> 2);
      const floatx4 *s4 = reinterpret_cast<const floatx4 *>(src);
      floatx4 *t4 = reinterpret_cast<floatx4 *>(tile);
      int e = tid;
      for (; e + 3 * kThreads < tot; e += 4 * kThreads) {
        floatx4 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = __builtin_nontemporal_load(s4 + e + q * kThreads);
#pragma unroll
        for (int q = 0; q < 4; ++q) t4[e + q * kThreads] = v[q];
      }
      for (; e < tot; e += kThreads) t4[e] = __builtin_nontemporal_load(s4 + e);
    } else {
      const int tot = nr * ic;
      for (int e = tid; e < tot; e += kThreads) tile[e] = src[e];
    }
    __syncthreads();
    // Haar stages
    for (int s = 0; s < P.num_stages; ++s) {
      const int off = P.stages[2 * s], cnt = P.stages[2 * s + 1];
      for (int u = tid; u < cnt; u += kThreads) {
        const uint32_t op = P.ops[off + u];
        const int i = (int)(op & 0xffffu), j = (int)(op >> 16);
        if (j != 0xffff) {
          for (int r = 0; r < nr; ++r) {
            float *row = tile + r * ic;
            const float a = row[i], b = row[j];
            row[i] = a + b;
            row[j] = a - b;
          }
        } else {
          for (int r = 0; r < nr; ++r) tile[r * ic + i] *= kSqrt2f;
        }
      }
      __syncthreads();
    }
    // gather + store
    float *dst = static_cast<float *>(out_raw) + r0 * oc;
    uint16_t *dst16 = static_cast<uint16_t *>(out_raw) + r0 * oc;
    if ((oc & 3) == 0) {
      for (int c = 4 * tid; c < oc; c += 4 * kThreads) {
        int g[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) g[q] = P.gather ? P.gather[c + q] : c + q;
#pragma unroll 4
        for (int r = 0; r < nr; ++r) {
          floatx4 v;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float x = tile[r * ic + (g[q] >= 0 ? g[q] : 0)];
            v[q] = g[q] >= 0 ? x : 0.0f;
          }
          if constexpr (OUT16)
            __builtin_nontemporal_store(
                u32x2{bf16_bits(v[0]) | (bf16_bits(v[1]) << 16), bf16_bits(v[2]) | (bf16_bits(v[3]) << 16)},
                reinterpret_cast<u32x2 *>(dst16 + (int64_t)r * oc + c));
          else
            __builtin_nontemporal_store(v, reinterpret_cast<floatx4 *>(dst + (int64_t)r * oc + c));
        }
      }
    } else {
      for (int c = tid; c < oc; c += kThreads) {
        const int g = P.gather ? P.gather[c] : c;
        for (int r = 0; r < nr; ++r) {
          const float x = g >= 0 ? tile[r * ic + (g >= 0 ? g : 0)] : 0.0f;
          if constexpr (OUT16)
            dst16[(int64_t)r * oc + c] = (uint16_t)bf16_bits(x);
          else
            dst[(int64_t)r * oc + c] = x;
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------- pass 2

// Grouped GEMM over leaf blocks: C[:, col_b + j] = sum_k A[:, col_b + k] * M_b[k][j], M_b
// read from its stored transpose.  Workgroup tile 128 signals x 128 columns, four waves of
// 64 x 64 (4 x 4 MFMA 16x16 tiles).  Both operands sit in LDS with k contiguous per row
// (As[m][k], Bs[n][k], rows padded by 16 bytes).  The contraction sums over k, so the k that
// a lane supplies to each MFMA may be permuted as long as A and B agree: per 16 (FP32) or
// 32 (BF16) k, lane (g, r) takes the consecutive k = 4g .. 4g+3 (four 16x16x4 steps) or
// 8g .. 8g+7 (one 16x16x32 BF16 step, gfx950's double-rate form) and reads each fragment
// with one 16-byte LDS load.  BF16 operands are rounded once,
// when the tile is written to LDS (split BF16: hi and lo planes, three products).  LDS is
// double buffered, so one barrier per K step; the next global tile is loaded into registers
// (unconditionally: the last tile is re-read, since loads under a branch are waited for
// inside it) while the current one is multiplied.
//
// Tiles are numbered block by block, m tile by m tile, n tiles fastest.  Workgroup i runs
// on XCD i mod 8, so within each window of 64 workgroups the numbering is regrouped to give
// every XCD 8 consecutive tiles (those that share an A panel then share one L2) while the
// windows keep the work spread evenly over the XCDs, whatever the block sizes.
constexpr int kBM = 128, kBN = 128;

template <int PREC, int BK_> struct GemmCfg {
  static constexpr int BK = BK_;                            // K step
  static constexpr int row_bytes = BK * (PREC == 0 ? 4 : 2) + 16;  // LDS row, padded
  static constexpr int planes = PREC == 3 ? 2 : 1;          // split: hi + lo
  static constexpr int plane_bytes = kBM * row_bytes;       // one operand tile
  static constexpr int buf_bytes = 2 * planes * plane_bytes;
  static constexpr int lds_bytes = 2 * buf_bytes;           // double buffered
};

template <int PREC, int BK, bool OUT16>
__global__ __launch_bounds__(kThreads) void gft_block_gemm(const LBlock *__restrict__ blocks,
                                                           int nblocks, const void *mats_raw,
                                                           const void *A_raw, void *C_raw, int64_t S,
                                                           int ld, const int32_t *omap, int ldy) {
  using Cfg = GemmCfg<PREC, BK>;
  constexpr int kRowBytes = Cfg::row_bytes;
  constexpr int KS = PREC == 0 ? 4 : 8;                     // k per lane per fragment load
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, g = lane >> 4, r = lane & 15;
  const int wm = wave >> 1, wn = wave & 1;

  int64_t id = blockIdx.x;
  if (id < (int64_t)(gridDim.x & ~63u)) id = (id & ~63ll) + ((id & 7) << 3) + ((id >> 3) & 7);
  const int64_t mtiles = (S + kBM - 1) / kBM;
  int b = 0;
  int64_t row0;
  int col0;
  if (omap) {
    // output scattered to its final positions: the tiles of one m panel (every block, every
    // n tile) are consecutive, so the partial lines of its output rows meet in one L2
    int64_t per_m = 0;
    for (int q = 0; q < nblocks; ++q) per_m += (blocks[q].size + kBN - 1) / kBN;
    row0 = (id / per_m) * kBM;
    int64_t t = id % per_m;
    for (; b < nblocks; ++b) {
      const int64_t nt = (blocks[b].size + kBN - 1) / kBN;
      if (t < nt) break;
      t -= nt;
    }
    if (b >= nblocks || row0 >= S) return;
    col0 = (int)t * kBN;
  } else {
    for (; b < nblocks; ++b) {
      const int64_t nt = (blocks[b].size + kBN - 1) / kBN;
      if (id < mtiles * nt) break;
      id -= mtiles * nt;
    }
    if (b >= nblocks) return;
    const int ntb = (blocks[b].size + kBN - 1) / kBN;
    row0 = (id / ntb) * kBM;
    col0 = (int)(id % ntb) * kBN;
  }
  const LBlock blk = blocks[b];
  const int K = blk.size;

  // global -> registers.  FP32 storage (PREC 0, 3): NLD float4 of A (row m, k quad kq) and
  // of B^T (row m of the n tile); BF16 storage (PREC 1): NLD 16-byte groups of 8 k.
  constexpr int EPL = PREC == 1 ? 8 : 4;                   // elements per 16-byte load
  constexpr int NQ = BK / EPL, NLD = kBM * NQ / kThreads;  // loads per row, per thread
  typedef __attribute__((ext_vector_type(4))) uint32_t vec4;
  vec4 ra[NLD], rb[NLD];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      const int idx = tid + kThreads * i;
      const int m = idx / NQ, kq = (idx % NQ) * EPL;
      const int k = k0 + kq;
      const int kc = k < K ? k : 0;                        // rows are padded to 8: in bounds
      int64_t row = row0 + m;
      row = row < S ? row : S - 1;                         // clamped: never stored
      const int c = col0 + m;
      const int64_t boff = blk.mat + (int64_t)(c < K ? c : K - 1) * blk.ld + kc;
      vec4 v, w;
      if constexpr (PREC == 1) {
        v = *reinterpret_cast<const vec4 *>(static_cast<const uint16_t *>(A_raw) + row * ld + blk.col + kc);
        w = *reinterpret_cast<const vec4 *>(static_cast<const uint16_t *>(mats_raw) + boff);
#pragma unroll
        for (int h = 0; h < 4; ++h) {                      // word h holds k + 2h, k + 2h + 1
          const uint32_t mask = k + 2 * h >= K ? 0u : (k + 2 * h + 1 >= K ? 0xffffu : 0xffffffffu);
          v[h] &= mask;
          w[h] &= c < K ? mask : 0u;
        }
      } else {
        v = *reinterpret_cast<const vec4 *>(static_cast<const float *>(A_raw) + row * ld + blk.col + kc);
        w = *reinterpret_cast<const vec4 *>(static_cast<const float *>(mats_raw) + boff);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (k + j >= K) v[j] = 0u;
          if (k + j >= K || c >= K) w[j] = 0u;
        }
      }
      ra[i] = v;
      rb[i] = w;
    }
  };
  auto store = [&](int buf) {
    char *base = smem + buf * Cfg::buf_bytes;
#pragma unroll
    for (int i = 0; i < NLD; ++i) {
      const int idx = tid + kThreads * i;
      const int m = idx / NQ, kq = (idx % NQ) * EPL;
      if constexpr (PREC == 0) {
        *reinterpret_cast<vec4 *>(base + m * kRowBytes + kq * 4) = ra[i];
        *reinterpret_cast<vec4 *>(base + Cfg::plane_bytes + m * kRowBytes + kq * 4) = rb[i];
      } else if constexpr (PREC == 1) {
        *reinterpret_cast<vec4 *>(base + m * kRowBytes + kq * 2) = ra[i];
        *reinterpret_cast<vec4 *>(base + Cfg::plane_bytes + m * kRowBytes + kq * 2) = rb[i];
      } else {
        uint32_t ah[4], bh[4], al[4], bl[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float xa = __uint_as_float(ra[i][j]), xb = __uint_as_float(rb[i][j]);
          ah[j] = bf16_bits(xa);
          bh[j] = bf16_bits(xb);
          al[j] = bf16_bits(xa - __uint_as_float(ah[j] << 16));
          bl[j] = bf16_bits(xb - __uint_as_float(bh[j] << 16));
        }
        const int off = m * kRowBytes + kq * 2;
        *reinterpret_cast<u32x2 *>(base + off) = u32x2{ah[0] | (ah[1] << 16), ah[2] | (ah[3] << 16)};
        *reinterpret_cast<u32x2 *>(base + Cfg::plane_bytes + off) =
            u32x2{bh[0] | (bh[1] << 16), bh[2] | (bh[3] << 16)};
        *reinterpret_cast<u32x2 *>(base + 2 * Cfg::plane_bytes + off) =
            u32x2{al[0] | (al[1] << 16), al[2] | (al[3] << 16)};
        *reinterpret_cast<u32x2 *>(base + 3 * Cfg::plane_bytes + off) =
            u32x2{bl[0] | (bl[1] << 16), bl[2] | (bl[3] << 16)};
      }
    }
  };

  floatx4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int nk = (K + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    load((kt + 1 < nk ? kt + 1 : kt) * BK);    // unconditional: see the prefetch note
    const char *base = smem + (kt & 1) * Cfg::buf_bytes;
#pragma unroll
    for (int h = 0; h < BK / (4 * KS); ++h) {     // 16-byte fragments: k = 4*KS*h + KS*g + ...
      const int aoff = (wm * 64 + r) * kRowBytes + 16 * (4 * h + g);
      const int boff = Cfg::plane_bytes + (wn * 64 + r) * kRowBytes + 16 * (4 * h + g);
      if constexpr (PREC == 0) {
        floatx4 a4[4], b4[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a4[i] = *reinterpret_cast<const floatx4 *>(base + aoff + i * 16 * kRowBytes);
#pragma unroll
        for (int j = 0; j < 4; ++j) b4[j] = *reinterpret_cast<const floatx4 *>(base + boff + j * 16 * kRowBytes);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[i][kk], b4[j][kk], acc[i][j], 0, 0, 0);
      } else {
        u32x4 ah[4], bh[4], al[4], bl[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          ah[i] = *reinterpret_cast<const u32x4 *>(base + aoff + i * 16 * kRowBytes);
          if constexpr (PREC == 3) al[i] = *reinterpret_cast<const u32x4 *>(base + 2 * Cfg::plane_bytes + aoff + i * 16 * kRowBytes);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          bh[j] = *reinterpret_cast<const u32x4 *>(base + boff + j * 16 * kRowBytes);
          if constexpr (PREC == 3) bl[j] = *reinterpret_cast<const u32x4 *>(base + 2 * Cfg::plane_bytes + boff + j * 16 * kRowBytes);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const bf16x8 a = __builtin_bit_cast(bf16x8, ah[i]), bb = __builtin_bit_cast(bf16x8, bh[j]);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc[i][j], 0, 0, 0);
            if constexpr (PREC == 3) {
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, bl[j]), acc[i][j], 0, 0, 0);
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, al[i]), bb, acc[i][j], 0, 0, 0);
            }
          }
      }
    }
    store((kt + 1) & 1);     // the other buffer: last read before the previous barrier
    __syncthreads();
  }
  // epilogue: lane (g, r) holds rows 4g + v, column r of each 16x16 tile; column c goes to
  // the workspace (C, row stride ld) or, with omap, to output position omap[blk.omap + c]
  // of the final array (C, row stride ldy; OUT16: BF16 storage, rounded to nearest even)
  float *C = static_cast<float *>(C_raw);
  uint16_t *C16 = static_cast<uint16_t *>(C_raw);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = col0 + wn * 64 + 16 * j + r;
    if (c >= K) continue;
    const int64_t dcol = omap ? (int64_t)omap[blk.omap + c] : (int64_t)blk.col + c;
    const int64_t dld = omap ? ldy : ld;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + wm * 64 + 16 * i + 4 * g + v;
        if (row < S) {
          if constexpr (OUT16) C16[row * dld + dcol] = (uint16_t)bf16_bits(acc[i][j][v]);
          else C[row * dld + dcol] = acc[i][j][v];
        }
      }
  }
}

// ---------------------------------------------------------------------------- scratch

// Workspace of the allocation-free apply (gft_apply_noalloc): a fixed array in the code
// object, one copy per GPU the library runs on, held until the process ends.  Host code
// never passes `scratch` itself to a kernel (on the host the name is a stand-in, not a
// device address): large_scratch_setup() looks up each device's address once, and the
// kernels receive that address like any other workspace pointer.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

hipError_t large_scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[dev] = ptr;
  return hipSuccess;
}

void *large_scratch(int dev) {
  if (dev < 0 || dev >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[dev];
}

// ---------------------------------------------------------------------------- launch

int permute_rows(const PermPass &P, int tile_kb) {
  // about 40 KB of LDS per tile (four workgroups per CU) unless the tuner says otherwise,
  // 1 to 16 rows
  const int rows = ((tile_kb > 0 ? tile_kb : 40) * 1024) / (4 * P.in_cols);
  return rows < 1 ? 1 : (rows > 16 ? 16 : rows);
}

template <bool IN16, bool OUT16>
static hipError_t launch_perm_io(const PermPass &P, const void *in, void *out, int64_t S, int num_cus,
                                 hipStream_t stream, int tile_kb) {
  const int rows = permute_rows(P, tile_kb);
  const size_t lds = (size_t)rows * P.in_cols * 4;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)gft_permute_stages<IN16, OUT16>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int64_t tiles = (S + rows - 1) / rows;
  const int64_t cap = (int64_t)num_cus * 8;
  const int grid = (int)(tiles < cap ? tiles : cap);
  hipLaunchKernelGGL((gft_permute_stages<IN16, OUT16>), dim3(grid), dim3(kThreads), lds, stream, P, in,
                     out, S, rows);
  return hipGetLastError();
}

hipError_t launch_permute_stages(const PermPass &P, const void *in, bool in16, void *out, bool out16,
                                 int64_t S, int num_cus, hipStream_t stream, int tile_kb) {
  if (in16)
    return out16 ? launch_perm_io<true, true>(P, in, out, S, num_cus, stream, tile_kb)
                 : launch_perm_io<true, false>(P, in, out, S, num_cus, stream, tile_kb);
  return out16 ? launch_perm_io<false, true>(P, in, out, S, num_cus, stream, tile_kb)
               : launch_perm_io<false, false>(P, in, out, S, num_cus, stream, tile_kb);
}

int64_t block_gemm_grid(const int32_t *sizes, int nblocks, int64_t S) {
  const int64_t mtiles = (S + kBM - 1) / kBM;
  int64_t tiles = 0;
  for (int b = 0; b < nblocks; ++b) tiles += mtiles * ((sizes[b] + kBN - 1) / kBN);
  return tiles;
}

template <int PREC, int BK, bool OUT16>
static hipError_t launch_gemm_prec(const LBlock *blocks, int nblocks, const void *mats,
                                   const void *A, void *C, int64_t S, int ld, int64_t grid,
                                   const int32_t *omap, int ldy, hipStream_t stream) {
  const int lds = GemmCfg<PREC, BK>::lds_bytes;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)gft_block_gemm<PREC, BK, OUT16>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((gft_block_gemm<PREC, BK, OUT16>), dim3((unsigned)grid), dim3(kThreads), lds, stream,
                     blocks, nblocks, mats, A, C, S, ld, omap, ldy);
  return hipGetLastError();
}

hipError_t launch_block_gemm(int prec, const LBlock *blocks, int nblocks, const void *mats,
                             const void *A, void *C, bool out16, int64_t S, int ld, int64_t grid,
                             const int32_t *omap, int ldy, hipStream_t stream) {
  if (grid <= 0) return hipSuccess;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  if (out16 && !omap) return hipErrorInvalidValue;   // the workspace stays FP32
  if (out16) switch (prec) {
      case 0: return launch_gemm_prec<0, 16, true>(blocks, nblocks, mats, A, C, S, ld, grid, omap, ldy, stream);
      case 1: return launch_gemm_prec<1, 32, true>(blocks, nblocks, mats, A, C, S, ld, grid, omap, ldy, stream);
      case 3: return launch_gemm_prec<3, 32, true>(blocks, nblocks, mats, A, C, S, ld, grid, omap, ldy, stream);
      default: return hipErrorInvalidValue;
    }
  switch (prec) {
    case 0: return launch_gemm_prec<0, 16, false>(blocks, nblocks, mats, A, C, S, ld, grid, omap, ldy, stream);
    case 1: return launch_gemm_prec<1, 32, false>(blocks, nblocks, mats, A, C, S, ld, grid, omap, ldy, stream);
    case 3: return launch_gemm_prec<3, 32, false>(blocks, nblocks, mats, A, C, S, ld, grid, omap, ldy, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gft
