// Device code of the one-pass large-signal GFT (see OnePass in device_program.hpp); the
// FP32, BF16 and split-BF16 kernels are instantiated in translation units of their own.
//
// The three-pass form moves every signal through a workspace twice: the first pass writes
// the staged row, the GEMM reads it and writes the block outputs, the last pass gathers
// them into the output order.  For plans with at most one Haar stage before the blocks
// (the single decomposition G = G+ (+) G-, or none) and one or two leaf blocks that fit the
// columns of one workgroup, this kernel does all three in one visit of the signal:
//
//   * a workgroup owns 16*MT signal rows and every workspace column; its k loop runs over
//     32-wide k steps of the blocks (FP32 blocks: eight 16x16x4 products per k step, in
//     two halves of 16 k);
//   * staging: the inputs of a k step are loaded one or two steps ahead, while earlier
//     steps' MFMAs run (32-bit byte offsets from the panel's first row: no 64-bit address
//     arithmetic per value; as few loads as the plan's source pattern allows: one value per
//     entry where the first pass only copies, pairs of neighbours where two entries' sources
//     are adjacent); the first-pass values (x_i + x_phi(i), x_i - x_phi(i), sqrt(2) x_c of a
//     V_Z node, or a copy: a multiply and a fused multiply-add with the entry's
//     coefficients) are rounded to BF16 (split: a hi and a lo part; FP32 blocks: kept as
//     they are) into a double-buffered LDS tile, one barrier per k step;
//   * products: wave w holds the accumulators of its block's n-tiles for all the rows (up
//     to 8 tiles of 16 columns x MT tiles of 16 rows) and reads its B fragments straight
//     from global memory in MFMA operand order (the matrices are shared by every
//     workgroup and stay in L2), one k step ahead, each fragment reloaded right after its
//     last use;
//   * the last pass: 16-row slabs of the results are written to LDS at their workspace
//     columns, the last pass's Haar stages (the inverse's left stage, the forward's right
//     stage) run there, and the output rows leave in their final order as whole rows (the
//     gather table and the stages' operations are read from LDS copies).
//
// The built-in grid is persistent: one workgroup per CU takes panels in turn.
//
// Every value is computed with the same operations in the same order as in the three-pass
// form (FP32 stage arithmetic, the same BF16 rounding, the same MFMA sequence per k chunk
// and lane placement), so the two forms agree bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device_program.hpp"

namespace gft {
namespace onepass {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 512;
constexpr int kARow = 80;                 // LDS bytes of a staged row: 32 BF16 k + 16 of padding
constexpr int kARow32 = 144;              // the same for FP32 blocks: 32 FP32 k + 16 of padding
constexpr float kSqrt2f = 1.41421356237309504880f;
// Largest tables (at most 1024 workspace columns: two blocks of at most 32 k steps).
constexpr int kMaxEntries = 1088;
constexpr int kMaxOps3 = 2048;            // last-pass Haar operations
constexpr int kMaxN = 1024;               // row length
// Word 3 of a raw (unswizzled, stride 0) buffer resource on gfx9-family GPUs.
constexpr int kBufferWord3 = 0x00020000;

__device__ __forceinline__ uint32_t bf16_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
// Two values rounded to BF16 in one gfx950 conversion (v_cvt_pk_bf16_f32; nearest even,
// FP32 denormals preserved: as bf16_bits for every value but NaN payloads): a in the low
// half, b in the high half.
__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(floatx2{a, b}, bf16x2));
}

// Value `off` bytes past `base` (FP32, or BF16 widened exactly).
template <bool IN16>
__device__ __forceinline__ float load_in(const char *base, uint32_t off) {
  if constexpr (IN16) return __uint_as_float((uint32_t)(*reinterpret_cast<const uint16_t *>(base + off)) << 16);
  else return *reinterpret_cast<const float *>(base + off);
}

// The value `off` bytes past `base` and the one after it, with one aligned load.
template <bool IN16>
__device__ __forceinline__ void load_pair(const char *base, uint32_t off, float &a, float &b) {
  if constexpr (IN16) {
    const uint32_t w = *reinterpret_cast<const uint32_t *>(base + off);
    a = __uint_as_float(w << 16);
    b = __uint_as_float(w & 0xffff0000u);
  } else {
    const float2 v = *reinterpret_cast<const float2 *>(base + off);
    a = v.x;
    b = v.y;
  }
}

// First-pass value c1 x1 + c0 x0 of an entry (see OnePass::desc): the multiply and the
// fused add reproduce x_i + x_j, x_i - x_j, sqrt(2) x_c and copies exactly; c1 = 0 skips the
// add and c0 = 0 (padding) gives 0, whatever the inputs hold.
__device__ __forceinline__ float first_pass(float c0, float c1, float x0, float x1) {
  const float p = c0 * x0;
  const float v = c1 != 0.0f ? __builtin_fmaf(c1, x1, p) : p;
  return c0 != 0.0f ? v : 0.0f;
}

// Shapes: a panel of 64 rows (FP32 and BF16 blocks) or 48 rows (split blocks: two operand
// planes) per workgroup, one workgroup per CU (the accumulators of a panel fill half the
// register file); the inputs of a k step are loaded D steps ahead (a ring of D register
// sets): two with one source set, pairs, or two sets of one value per entry; one with two
// sets of two values (a second ring slot would spill; measured slower) and with FP32 blocks
// (a k step is 256 products per wave, long enough to cover the loads; two would spill).
template <int PREC, int NS> struct OnePassShape {
  static constexpr int MT = PREC == 3 ? 3 : 4;     // 16-row tiles per panel
  static constexpr int SR = 16;                    // result slab rows
  static constexpr int D = NS == 2 || PREC == 0 ? 1 : 2;
};

// PREC: GFT_FP32 (0), GFT_BF16 (1) or GFT_SPLIT_BF16 (3).  NS: how a k step's inputs are loaded
// (OnePass::src_mode: 1, one set for both blocks; 2, one set per block; 3, one load of two
// adjacent values per entry, the first for block 0, the second for block 1; 4, one set per
// block of one value per entry: every entry is a copy or a sqrt 2 scaling; 5, one set for
// both blocks, each lane's two entries loaded as two pairs of adjacent values, and the
// results written to the slab at their output columns).  IN16: the input rows hold BF16.
// out16: the output rows hold BF16.
template <int PREC, int NS, bool IN16>
__global__ __launch_bounds__(kThreads) void gft_onepass(OnePass P, const void *__restrict__ in,
                                                          void *__restrict__ out, int64_t S, int out16) {
  constexpr int MT = OnePassShape<PREC, NS>::MT;
  constexpr int D = OnePassShape<PREC, NS>::D;
  constexpr int BM = 16 * MT;
  constexpr int PL = PREC == 3 ? 2 : 1;                              // LDS operand planes
  constexpr int PLB = PREC == 1 ? 1 : 2;                             // fragments per (kc, nt)
  constexpr int AROW = PREC == 0 ? kARow32 : kARow;
  constexpr int kPlane = BM * AROW;
  constexpr int ESZ = IN16 ? 2 : 4;
  constexpr int SR = OnePassShape<PREC, NS>::SR;
  constexpr int ITEMS = (BM * 16 + kThreads - 1) / kThreads;         // (row, k pair) items
  constexpr int NX = NS == 2 || NS == 4 ? 2 : 1;                     // register sets per step
  __shared__ __attribute__((aligned(16))) int32_t sdesc[4 * kMaxEntries];
  __shared__ __attribute__((aligned(16))) char abuf[2 * 2 * PL * kPlane];
  __shared__ __attribute__((aligned(16))) float slab[SR * (1024 + 4)];
  __shared__ __attribute__((aligned(16))) int32_t sgather[kMaxN];
  constexpr bool DIRECT = NS == 5;                                   // results to output columns
  __shared__ int32_t somap[DIRECT ? kMaxN : 1];
  __shared__ uint32_t sops[kMaxOps3];
  const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, r = lane & 15, kp = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: per-wave fields in SGPRs
  const int nb = P.nblocks, n = P.n;
  constexpr int buf_bytes = 2 * PL * kPlane;                        // room for two blocks
  const int sstr = P.slab_stride;
  for (int i = tid; i < P.desc_words; i += kThreads) sdesc[i] = P.desc[i];
  if constexpr (DIRECT) {
    // the results go to their output columns; the columns no workspace column feeds stay zero
    for (int i = tid; i < P.ldw; i += kThreads) somap[i] = P.omap3[i];
    for (int i = tid; i < SR * sstr; i += kThreads) slab[i] = 0.0f;
  } else {
    for (int i = tid; i < n; i += kThreads) sgather[i] = P.gather3[i];
  }
  for (int i = tid; i < P.ops3_words; i += kThreads) sops[i] = P.ops3[i];
  __syncthreads();

  const int wb = P.wblk[wave], nt0 = P.wnt0[wave], wcnt = P.wcnt[wave];
  const int wbs = wb >= 0 ? wb : 0;
  const int wfo = P.frag_off[wbs], wntl = P.ntl[wbs], wK = P.K[wbs], wcol = P.col[wbs], wnk = P.nkc[wbs];
  // the B fragments (a table of at most a few MB: 32-bit offsets; every index below is
  // clamped to a valid fragment)
  const __amdgpu_buffer_rsrc_t frsrc =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(P.frag), (short)0, -1, kBufferWord3);
  const uint32_t flane = 16u * (uint32_t)lane;
  const int64_t npanels = (S + BM - 1) / BM;
  // (buffer loads: the fragment's byte offset is uniform and goes in a scalar register,
  // the lane's 16-byte slot is one shared vector register; global loads would hold a
  // 64-bit address per tile and step)
  auto frag_at = [&](int kc, int j, int pl) {
    const int nt = nt0 + (j < wcnt ? j : (wcnt > 0 ? wcnt - 1 : 0));   // always a valid tile
    const int off = ((wfo + kc * wntl + nt) * PLB + pl) * 1024;
    return __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(frsrc, flane, off, 0));
  };
  // the first k chunk's fragments; each panel's last k step loads them again for the next
  u32x4 bh[8], bl[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    bh[j] = frag_at(0, j, 0);
    if constexpr (PREC == 3) bl[j] = frag_at(0, j, 1);
  }

  // the input rows the staging loads read: panel p's first row (uniform) and each item's
  // row offset (rows past the last signal: clamped, never stored)
  const char *base = nullptr;
  uint32_t rowoff[ITEMS];
  auto set_panel = [&](int64_t p) {
    const int64_t r0 = p * BM;
    base = static_cast<const char *>(in) + r0 * n * ESZ;
    const int last = (S - r0 < BM ? (int)(S - r0) : BM) - 1;
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const int row = (tid >> 4) + 32 * it;
      rowoff[it] = (uint32_t)((row < last ? row : last) * n * ESZ);
    }
  };
  // ---- staging: inputs of k step kt into ring set q = kt mod D (loads only; consumed by
  // stage_store).  Steps past the end re-read the last step's inputs.
  float sx[D][NX][ITEMS][2][2];
  // split blocks: their registers have no room for the next panel's inputs during the last
  // pass (held there they spill, and the forward measured no faster)
  constexpr bool kPrefetchPanel = PREC != 3;

  for (int64_t panel = blockIdx.x; panel < npanels; panel += gridDim.x) {
    const int64_t row0 = panel * BM;
    auto stage_load = [&](int kt, float (&x)[NX][ITEMS][2][2]) {
      kt = kt < P.nk ? kt : P.nk - 1;
#pragma unroll
      for (int s = 0; s < NX; ++s) {
        // the block whose entries give this set's offsets: with one set, block 0 while it
        // has k steps left, then block 1; k steps past a block's end re-read its last one
        const int b = NX == 2 ? s : (kt < P.nkc[0] || nb == 1 ? 0 : 1);
        const int kk = kt < P.nkc[b] ? kt : P.nkc[b] - 1;
        const int32_t *d = sdesc + 4 * (P.desc_off[b] + 32 * kk + 2 * kp);
        const u32x4 d0 = *reinterpret_cast<const u32x4 *>(d), d1 = *reinterpret_cast<const u32x4 *>(d + 4);
#pragma unroll
        for (int it = 0; it < ITEMS; ++it)
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const u32x4 de = e == 0 ? d0 : d1;
            if constexpr (NS == 5) {
              // entries 2 kp and 2 kp + 1: their first sources are neighbours from the first
              // entry's, their second sources neighbours from the second entry's, downwards
              if (e == 0) {
                load_pair<IN16>(base, rowoff[it] + d0[0], x[s][it][0][0], x[s][it][1][0]);
                load_pair<IN16>(base, rowoff[it] + d1[1], x[s][it][1][1], x[s][it][0][1]);
              }
            } else if constexpr (NS == 3) {
              load_pair<IN16>(base, rowoff[it] + de[0], x[s][it][e][0], x[s][it][e][1]);
            } else if constexpr (NS == 4) {
              x[s][it][e][0] = load_in<IN16>(base, rowoff[it] + de[0]);
            } else {
              x[s][it][e][0] = load_in<IN16>(base, rowoff[it] + de[0]);
              x[s][it][e][1] = load_in<IN16>(base, rowoff[it] + de[1]);
            }
          }
      }
    };
    // ---- staging: first-pass values of k step kt into LDS buffer buf (zeros for k steps
    // past a block's end, so that its waves may multiply them in with no effect)
    // (both block slots always: with one block the second repeats the first into a plane
    // nothing reads, so that the staging is branch-free and can interleave with products).
    // The coefficients of a block's entries at k step kt (the same for every row) are read
    // from LDS at the start of the k step before, so that no unit waits for them.
    struct Coef {
      float c[4];      // c0, c1 of the lane's two entries
      uint32_t keep;   // all ones, or zeros past the block's end (no branch)
    };
    auto stage_coef = [&](int kt, int b) {
      const int bb = b < nb ? b : nb - 1;
      const bool live = kt < P.nkc[bb];
      const int kk = live ? kt : P.nkc[bb] - 1;
      const int32_t *d = sdesc + 4 * (P.desc_off[bb] + 32 * kk + 2 * kp);
      const u32x2 w0 = *reinterpret_cast<const u32x2 *>(d + 2), w1 = *reinterpret_cast<const u32x2 *>(d + 6);
      Coef cf;
      cf.c[0] = __uint_as_float(w0[0]);
      cf.c[1] = __uint_as_float(w0[1]);
      cf.c[2] = __uint_as_float(w1[0]);
      cf.c[3] = __uint_as_float(w1[1]);
      cf.keep = live ? 0xffffffffu : 0u;
      return cf;
    };
    auto stage_unit = [&](const Coef &cf, int buf, const float (&x)[NX][ITEMS][2][2], int b, int it) {
      const uint32_t keep = cf.keep;
      const int s = NX == 2 ? b : 0;
      char *plane = abuf + buf * buf_bytes + b * PL * kPlane;
      const int idx = tid + kThreads * it;
      if ((BM * 16) % kThreads != 0 && idx >= BM * 16) return;   // MT = 3: rows 48 .. 63 do not exist
      const int row = idx >> 4;
      float v[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        if constexpr (NS == 3)   // a copy: block b's value is element b (^ pair_swap) of the pair
          v[e] = first_pass(cf.c[2 * e], 0.0f, (b != 0) != (P.pair_swap != 0) ? x[0][it][e][1] : x[0][it][e][0], 0.0f);
        else if constexpr (NS == 4)
          v[e] = first_pass(cf.c[2 * e], 0.0f, x[s][it][e][0], 0.0f);
        else
          v[e] = first_pass(cf.c[2 * e], cf.c[2 * e + 1], x[s][it][e][0], x[s][it][e][1]);
      }
      if constexpr (PREC == 0) {
        *reinterpret_cast<u32x2 *>(plane + row * AROW + 8 * kp) =
            u32x2{__float_as_uint(v[0]) & keep, __float_as_uint(v[1]) & keep};
      } else {
        const uint32_t hw = bf16_pair(v[0], v[1]);
        *reinterpret_cast<uint32_t *>(plane + row * AROW + 4 * kp) = hw & keep;
        if constexpr (PL == 2) {
          const uint32_t lw = bf16_pair(v[0] - __uint_as_float(hw << 16), v[1] - __uint_as_float(hw & 0xffff0000u));
          *reinterpret_cast<uint32_t *>(plane + kPlane + row * AROW + 4 * kp) = lw & keep;
        }
      }
    };
    auto stage_store = [&](int kt, int buf, const float (&x)[NX][ITEMS][2][2]) {
      const Coef cf[2] = {stage_coef(kt, 0), stage_coef(kt, 1)};
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) stage_unit(cf[b], buf, x, b, it);
    };

    floatx4 acc[MT][8];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // the first steps' inputs: loaded here for the first panel (and every panel with split
    // blocks), before the last pass of the panel before for the others
    if (!kPrefetchPanel || panel == (int64_t)blockIdx.x) {
      set_panel(panel);
#pragma unroll
      for (int q = 0; q < D; ++q) stage_load(q, sx[q]);
    }
    stage_store(0, 0, sx[0]);
    __syncthreads();
    // one k step (kt = Q mod D): the loads of step kt + D into the set that step kt used,
    // the products of step kt, the staging of step kt + 1
    auto step = [&](int kt, auto Qc) {
      constexpr int Q = decltype(Qc)::value;
      stage_load(kt + D, sx[Q]);
      const Coef cf[2] = {stage_coef(kt + 1, 0), stage_coef(kt + 1, 1)};
      // No branch around the products and the B reloads: a load under a branch makes the
      // compiler wait for every outstanding load where the paths join (which would expose
      // the next step's B fragments here), and accumulators under a branch get copied.
      // Past its block's end a wave multiplies the zero tiles staged for it; tiles past a
      // wave's count (and every tile of an idle wave) repeat a valid fragment into
      // accumulators that are never stored.
      const char *ab = abuf + (kt & 1) * buf_bytes + wbs * PL * kPlane;
      // next k chunk; past the wave's last one, the first (the steps left multiply zero
      // tiles, and the next panel starts with it)
      const int kn = kt + 1 < wnk ? kt + 1 : 0;
      if constexpr (PREC == 0) {
        // FP32 blocks: two halves of 16 k, each four 16x16x4 products per tile (lane group g
        // gives k = 16 h + 4 g + kk of MFMA kk: the three-pass FP32 GEMM's k order).  One
        // fragment register per tile: the second half's fragment of this step is loaded
        // right after the first half's last use, the next step's first half after the second.
        // (the staging units go in the second half, so that this step's input loads, issued
        // at its start, have had half a step to arrive)
        const int kc = kt < wnk ? kt : wnk - 1;
        constexpr int kUnits = 2 * ITEMS, kEvery = 8 / kUnits;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          floatx4 af[MT];
#pragma unroll
          for (int i = 0; i < MT; ++i)
            af[i] = *reinterpret_cast<const floatx4 *>(ab + (16 * i + r) * AROW + 64 * h + 16 * g);
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const floatx4 bf = __builtin_bit_cast(floatx4, bh[j]);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
#pragma unroll
              for (int i = 0; i < MT; ++i)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][kk], bf[kk], acc[i][j], 0, 0, 0);
            bh[j] = h == 0 ? frag_at(kc, j, 1) : frag_at(kn, j, 0);
            if (h == 1 && j % kEvery == kEvery - 1) {
              const int u = j / kEvery;
              __builtin_amdgcn_sched_barrier(0);
              stage_unit(cf[u / ITEMS], (kt + 1) & 1, sx[(Q + 1) % D], u / ITEMS, u % ITEMS);
              __builtin_amdgcn_sched_barrier(0);
            }
          }
        }
      } else {
        u32x4 ah[MT], al[MT];
#pragma unroll
        for (int i = 0; i < MT; ++i) {
          ah[i] = *reinterpret_cast<const u32x4 *>(ab + (16 * i + r) * AROW + 16 * g);
          if constexpr (PL == 2) al[i] = *reinterpret_cast<const u32x4 *>(ab + kPlane + (16 * i + r) * AROW + 16 * g);
        }
        // The staging of step kt + 1 into the other buffer (last read before the previous
        // barrier; past the last step it writes zeros that nothing reads) is independent of
        // this step's products: its 2 x ITEMS units go between the MFMA groups, fenced from
        // the scheduler, so the matrix core runs each group while the wave issues the VALU
        // work of a unit.
        constexpr int kUnits = 2 * ITEMS, kEvery = 8 / kUnits;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
#pragma unroll
          for (int i = 0; i < MT; ++i) {
            const bf16x8 a = __builtin_bit_cast(bf16x8, ah[i]), b = __builtin_bit_cast(bf16x8, bh[j]);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
            if constexpr (PL == 2) {
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, __builtin_bit_cast(bf16x8, bl[j]), acc[i][j], 0, 0, 0);
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, al[i]), b, acc[i][j], 0, 0, 0);
            }
          }
          bh[j] = frag_at(kn, j, 0);
          if constexpr (PL == 2) bl[j] = frag_at(kn, j, 1);
          if (j % kEvery == kEvery - 1) {
            const int u = j / kEvery;
            __builtin_amdgcn_sched_barrier(0);
            stage_unit(cf[u / ITEMS], (kt + 1) & 1, sx[(Q + 1) % D], u / ITEMS, u % ITEMS);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
      __syncthreads();
    };
    // whole groups of D steps with no branch inside (the compiler's waits stay exact), then
    // the remaining steps
    int kt = 0;
    for (; kt + D <= P.nk; kt += D) {
      step(kt, std::integral_constant<int, 0>{});
      if constexpr (D == 2) step(kt + 1, std::integral_constant<int, 1 % D>{});
    }
    if (D == 2 && kt < P.nk) step(kt, std::integral_constant<int, 0>{});
    if constexpr (kPrefetchPanel) {
      // the next panel's first steps, loaded ahead of this panel's last pass so that their
      // latency passes during it (past the last panel: this panel's last step again, still
      // in L2, never used)
      const int64_t nx = panel + gridDim.x;
      const bool more = nx < npanels;
      set_panel(more ? nx : panel);
#pragma unroll
      for (int q = 0; q < D; ++q) stage_load(more ? q : P.nk - 1, sx[q]);
    }

    // ---- last pass, one slab of SR rows at a time (row tile s, half h when SR = 8); each
    // result column goes to its workspace column, or (DIRECT) its output column (-1: none)
    [[maybe_unused]] int dcol[8];
    if constexpr (DIRECT) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int c = 16 * (nt0 + j) + r;
        dcol[j] = wb >= 0 && j < wcnt && c < wK ? somap[wcol + c] : -1;
      }
    }
#pragma unroll
    for (int s = 0; s < MT; ++s)
#pragma unroll
    for (int h = 0; h < 16 / SR; ++h) {
      if constexpr (DIRECT) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          if (dcol[j] >= 0) {
            float *dst = slab + dcol[j];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int lr = 4 * g + v - SR * h;   // the lanes of this half write
              if (lr >= 0 && lr < SR) dst[lr * sstr] = acc[s][j][v];
            }
          }
        }
      } else if (wb >= 0) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int c = 16 * (nt0 + j) + r;
          if (j < wcnt && c < wK) {
            float *dst = slab + wcol + c;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int lr = 4 * g + v - SR * h;
              if (lr >= 0 && lr < SR) dst[lr * sstr] = acc[s][j][v];
            }
          }
        }
      }
      __syncthreads();
      for (int st = 0; st < P.num_stages3; ++st) {
        const int off = P.stages3[2 * st], cnt = P.stages3[2 * st + 1];
        for (int u = tid; u < cnt; u += kThreads) {
          const uint32_t op = sops[off + u];
          const int i = (int)(op & 0xffffu), j = (int)(op >> 16);
          // every row's operands read before any is written (the rows do not alias, which
          // the compiler cannot see: in one loop it would wait for each row in turn)
          if (j != 0xffff) {
            float a[SR], b[SR];
#pragma unroll
            for (int rr = 0; rr < SR; ++rr) {
              a[rr] = slab[rr * sstr + i];
              b[rr] = slab[rr * sstr + j];
            }
#pragma unroll
            for (int rr = 0; rr < SR; ++rr) {
              slab[rr * sstr + i] = a[rr] + b[rr];
              slab[rr * sstr + j] = a[rr] - b[rr];
            }
          } else {
            float a[SR];
#pragma unroll
            for (int rr = 0; rr < SR; ++rr) a[rr] = slab[rr * sstr + i];
#pragma unroll
            for (int rr = 0; rr < SR; ++rr) slab[rr * sstr + i] = a[rr] * kSqrt2f;
          }
        }
        __syncthreads();
      }
      const int64_t rb = row0 + 16 * s + SR * h;
      const int nr = S - rb < SR ? (int)(S - rb) : SR;
      if ((n & 3) == 0) {
        const int nq = n >> 2;
#pragma unroll 4
        for (int idx = tid; idx < SR * nq; idx += kThreads) {
          const int rr = idx / nq, q = idx - rr * nq;
          if (rr >= nr) continue;
          const float *srow = slab + rr * sstr;
          floatx4 v;
          if constexpr (DIRECT) {
            v = *reinterpret_cast<const floatx4 *>(srow + 4 * q);
          } else {
            const int4 gi = *reinterpret_cast<const int4 *>(sgather + 4 * q);
            v[0] = gi.x >= 0 ? srow[gi.x] : 0.0f;
            v[1] = gi.y >= 0 ? srow[gi.y] : 0.0f;
            v[2] = gi.z >= 0 ? srow[gi.z] : 0.0f;
            v[3] = gi.w >= 0 ? srow[gi.w] : 0.0f;
          }
          const int64_t o = (rb + rr) * n + 4 * q;
          if (out16)
            __builtin_nontemporal_store(
                u32x2{bf16_pair(v[0], v[1]), bf16_pair(v[2], v[3])},
                reinterpret_cast<u32x2 *>(static_cast<uint16_t *>(out) + o));
          else
            __builtin_nontemporal_store(v, reinterpret_cast<floatx4 *>(static_cast<float *>(out) + o));
        }
      } else {
        for (int idx = tid; idx < SR * n; idx += kThreads) {
          const int rr = idx / n, c = idx - rr * n;
          if (rr >= nr) continue;
          const int gi = DIRECT ? c : sgather[c];
          const float v = gi >= 0 ? slab[rr * sstr + gi] : 0.0f;
          const int64_t o = (rb + rr) * n + c;
          if (out16) static_cast<uint16_t *>(out)[o] = (uint16_t)bf16_bits(v);
          else static_cast<float *>(out)[o] = v;
        }
      }
      __syncthreads();
    }
  }
}

template <int PREC, int NS, bool IN16>
hipError_t launch_op(const OnePass &P, const void *in, void *out, int64_t S, bool out16, int grid, hipStream_t st) {
  hipLaunchKernelGGL((gft_onepass<PREC, NS, IN16>), dim3((unsigned)grid), dim3(kThreads), 0, st, P, in, out, S,
                     out16 ? 1 : 0);
  return hipGetLastError();
}

template <int PREC, int NS, bool IN16>
int occupancy_op() {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, (const void *)gft_onepass<PREC, NS, IN16>, kThreads, 0) !=
      hipSuccess)
    return 1;
  return blocks > 0 ? blocks : 1;
}

// The instance for a plan direction's source mode (OnePass::src_mode) and input storage.
template <int PREC, bool IN16>
hipError_t launch_mode(const OnePass &P, const void *in, void *out, int64_t S, bool out16, int grid, hipStream_t st) {
  switch (P.src_mode) {
    case 1: return launch_op<PREC, 1, IN16>(P, in, out, S, out16, grid, st);
    case 3: return launch_op<PREC, 3, IN16>(P, in, out, S, out16, grid, st);
    case 4: return launch_op<PREC, 4, IN16>(P, in, out, S, out16, grid, st);
    case 5: return launch_op<PREC, 5, IN16>(P, in, out, S, out16, grid, st);
    default: return launch_op<PREC, 2, IN16>(P, in, out, S, out16, grid, st);
  }
}

template <int PREC>
hipError_t launch_prec(const OnePass &P, const void *in, void *out, int64_t S, bool in16, bool out16, int grid,
                       hipStream_t st) {
  return in16 ? launch_mode<PREC, true>(P, in, out, S, out16, grid, st)
              : launch_mode<PREC, false>(P, in, out, S, out16, grid, st);
}

template <int PREC, bool IN16>
int occupancy_mode(int src_mode) {
  return src_mode == 1   ? occupancy_op<PREC, 1, IN16>()
         : src_mode == 3 ? occupancy_op<PREC, 3, IN16>()
         : src_mode == 4 ? occupancy_op<PREC, 4, IN16>()
         : src_mode == 5 ? occupancy_op<PREC, 5, IN16>()
                         : occupancy_op<PREC, 2, IN16>();
}

template <int PREC>
int occupancy_prec(int src_mode, bool in16) {
  return in16 ? occupancy_mode<PREC, true>(src_mode) : occupancy_mode<PREC, false>(src_mode);
}

}  // namespace onepass
}  // namespace gft
