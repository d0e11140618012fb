// Separable-engine kernel and launch templates (see gft_product.hip), shared by the FP32-
// and BF16-storage translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_program.hpp"

namespace gft {

// Factor size padded to 16, 32 or 64 (0 above 64).
inline int product_pad_size(int n) { return n <= 16 ? 16 : (n <= 32 ? 32 : (n <= 64 ? 64 : 0)); }

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kPWaves = 4;
constexpr int kFP32 = 0, kBF16 = 1, kSPLIT = 3;   // gft_precision values (include/gft.h)

// FP32 -> BF16 bits, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint32_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float floatx2_t __attribute__((ext_vector_type(2)));
// Two values rounded to BF16 in one gfx950 conversion (v_cvt_pk_bf16_f32; nearest even,
// FP32 denormals preserved: as bf16_rne for every value but NaN
// payloads): a in the low half, b in the high half.
__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(floatx2_t{a, b}, bf16x2_t));
}

// Four values as a 16x16x16 BF16 MFMA operand: hi = BF16(x), lo = BF16(x - hi) (the split
// form; lo unused with plain BF16 blocks).
struct Frag16 {
  u32x2 hi, lo;
};
__device__ __forceinline__ Frag16 pack16(float a, float b, float c, float d) {
  const uint32_t w0 = bf16_pair(a, b), w1 = bf16_pair(c, d);
  Frag16 f;
  f.hi = u32x2{w0, w1};
  f.lo = u32x2{bf16_pair(a - __uint_as_float(w0 << 16), b - __uint_as_float(w0 & 0xffff0000u)),
               bf16_pair(c - __uint_as_float(w1 << 16), d - __uint_as_float(w1 & 0xffff0000u))};
  return f;
}

// acc += A * B on 16x16x16 BF16 MFMA; SPLIT: hi*hi + hi*lo + lo*hi (FP32-level products).
template <bool SPLIT>
__device__ __forceinline__ floatx4 mfma16(const Frag16 &a, const Frag16 &b, floatx4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(bf16x4, a.hi), __builtin_bit_cast(bf16x4, b.hi), acc, 0, 0, 0);
  if constexpr (SPLIT) {
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(bf16x4, a.hi), __builtin_bit_cast(bf16x4, b.lo), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(bf16x4, a.lo), __builtin_bit_cast(bf16x4, b.hi), acc, 0, 0, 0);
  }
  return acc;
}

// acc += A * B over two k chunks at once on gfx950's 16x16x32 BF16 MFMA: each lane gives
// its four values of chunk 0 then its four of chunk 1, in A and in B alike.  Whatever k the
// MFMA assigns to each of a lane's eight slots, A and B slots pair up as in two 16x16x16
// steps, so the sum is the same contraction at half the MFMA issue count.
template <bool SPLIT>
__device__ __forceinline__ floatx4 mfma32(const Frag16 &a0, const Frag16 &a1, const Frag16 &b0,
                                          const Frag16 &b1, floatx4 acc) {
  auto cat = [](const u32x2 &x, const u32x2 &y) { return __builtin_bit_cast(bf16x8, u32x4{x[0], x[1], y[0], y[1]}); };
  const bf16x8 ah = cat(a0.hi, a1.hi), bh = cat(b0.hi, b1.hi);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
  if constexpr (SPLIT) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, cat(b0.lo, b1.lo), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cat(a0.lo, a1.lo), bh, acc, 0, 0, 0);
  }
  return acc;
}

// Orders this wave's LDS accesses: every lane's earlier LDS operations complete before any
// later one.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Halving reversal stages of a 64-node axis, compiled: stage R (R = 64, 32, ..., 2) pairs
// node i < R / 2 with R - 1 - i (V_X = i) and computes x + y at i, x - y at R - 1 - i,
// unscaled (the 2^(-depth/2) of the leaves is in their matrices).  The inverse runs the
// same pairs from R = 2 up to R = 64.
//
// Columns (axis b), on a signal row held in the load layout: lane l holds columns 4c .. 4c+3
// (c = l % 16) of its rows, so the partner of column 4c + e at R >= 8 is element 3 - e of
// lane 15 - c, 7 - c, 3 - c or 1 - c of the same 16-lane row (DPP row mirror, row half
// mirror and the quad permutations 3210 and 1032); at R = 4 and 2 it is in the lane.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}

template <int CTRL, int Q>   // Q = R / 4 lanes of 4 columns take part
__device__ __forceinline__ void col_stage(floatx4 &v, int c) {
  // every lane reads its partner's values (DPP needs its source lanes active)
  const floatx4 p = {dpp_f<CTRL>(v[3]), dpp_f<CTRL>(v[2]), dpp_f<CTRL>(v[1]), dpp_f<CTRL>(v[0])};
  if (c < Q) {
    const bool xs = c < Q / 2;   // the lane holds the V_X side
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = xs ? v[e] + p[e] : p[e] - v[e];
  }
}

__device__ __forceinline__ void col_stage4(floatx4 &v, int c) {   // R = 4: (0, 3), (1, 2)
  if (c == 0) v = floatx4{v[0] + v[3], v[1] + v[2], v[1] - v[2], v[0] - v[3]};
}

__device__ __forceinline__ void col_stage2(floatx4 &v, int c) {   // R = 2: (0, 1)
  if (c == 0) v = floatx4{v[0] + v[1], v[0] - v[1], v[2], v[3]};
}

template <bool INV>
__device__ __forceinline__ void halving_cols(floatx4 &v, int c) {
  if constexpr (!INV) {
    col_stage<0x140, 16>(v, c);   // R = 64: row mirror, lane 15 - c
    col_stage<0x141, 8>(v, c);    // R = 32: row half mirror, lane 7 - c
    col_stage<0x1B, 4>(v, c);     // R = 16: quad permutation 3210, lane 3 - c
    col_stage<0xB1, 2>(v, c);     // R = 8: quad permutation 1032, lane 1 - c
    col_stage4(v, c);
    col_stage2(v, c);
  } else {
    col_stage2(v, c);
    col_stage4(v, c);
    col_stage<0xB1, 2>(v, c);
    col_stage<0x1B, 4>(v, c);
    col_stage<0x141, 8>(v, c);
    col_stage<0x140, 16>(v, c);
  }
}

// Rows (axis a): lane c works on column c of the wave's tile (64 rows, stride STR).  The
// R = 64 stage pairs rows i and 63 - i in place in LDS; the other stages act on rows 0..31
// only, which the lane reads into registers, combines there and writes back (holding the
// whole column in registers instead made the forward kernel spill).  Each 64-lane access
// touches 64 consecutive words of one row.
template <bool INV, int STR>
__device__ __forceinline__ void halving_rows(float *T, int c) {
  auto stage64 = [&]() {
#pragma unroll 8
    for (int i = 0; i < 32; ++i) {
      const float x = T[i * STR + c], y = T[(63 - i) * STR + c];
      T[i * STR + c] = x + y;
      T[(63 - i) * STR + c] = x - y;
    }
  };
  if constexpr (!INV) stage64();
  float col[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) col[i] = T[i * STR + c];
#pragma unroll
  for (int t = 0; t < 5; ++t) {
    const int R = INV ? (2 << t) : (32 >> t);
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      const float x = col[i], y = col[R - 1 - i];
      col[i] = x + y;
      col[R - 1 - i] = x - y;
    }
  }
#pragma unroll
  for (int i = 0; i < 32; ++i) T[i * STR + c] = col[i];
  if constexpr (INV) stage64();
}

// Tile pattern TP of the products' T x T grid of 16 x 16 tiles (T = NA / 16 or NB / 16):
// 0 every tile (dense factors); 1 staged 64-node factors with the halving stages above,
// whose block-diagonal leaf matrices (blocks of 32, 16, 8, 4, 2, 1, 1 nodes in ascending
// node order) fill tiles (0,0), (1,1) and the 2 x 2 group {2, 3}.  The tile loops are fully
// unrolled, so the test folds away and zero tiles cost no MFMA and no fragment registers.
template <int TP, int T>
__device__ __forceinline__ constexpr bool tile_nz(int r, int c) {
  return TP == 0 || r == c || (T == 4 && r >= 2 && c >= 2);
}

template <int NA, int NB>
constexpr size_t product_lds_bytes(int n) {
  return (size_t)kPWaves * NA * (NB + 1) * sizeof(float) + (((size_t)n * 2 + 15) & ~(size_t)15);
}

}  // namespace

// SAME: the two factors are one matrix (U_a = U_b, square products of one graph), whose
// fragments then serve both products.  PREC: FP32 (16x16x4 FP32 MFMA), BF16 or split BF16
// (16x16x16 BF16 MFMA with FP32 accumulation; the data operand of each product is rounded
// to BF16, or split into hi + lo, as it enters the MFMA).
// TP: 0 dense factors, FP32 storage; 1 staged 64-node factors (tile pattern 1 above), FP32
// storage; 2 dense factors, BF16 storage of signals and coefficients (16-byte groups of 8
// values, widened exactly as they enter the tile, rounded to nearest even as they leave).
template <int NA, int NB, int DIR, bool SAME, int PREC, int TP>
__global__ __launch_bounds__(64 * kPWaves) __attribute__((amdgpu_waves_per_eu(2))) void gft_product(
    PProgram P, const void *in_raw, void *out_raw, int64_t nsig) {
  static_assert(!SAME || NA == NB, "one matrix needs equal factor sizes");
  static_assert(TP != 1 || (NA == 64 && NB == 64), "tile pattern 1: 64 x 64 factors only");
  constexpr bool IO16 = TP == 2;
  constexpr int TPM = TP == 1 ? 1 : 0;   // tile pattern of the products
  const float *in = static_cast<const float *>(in_raw);
  float *out = static_cast<float *>(out_raw);
  const uint16_t *in16 = static_cast<const uint16_t *>(in_raw);
  uint16_t *out16 = static_cast<uint16_t *>(out_raw);
  constexpr bool B16 = PREC != kFP32;
  constexpr int STR = NB + 1;
  constexpr int TW = NA * STR;
  constexpr int MAXV = NA * NB / 256;   // 16-byte groups per lane of a full NA x NB signal
  constexpr int MA = NA / 16, MB = NB / 16;
  extern __shared__ __attribute__((aligned(16))) float psmem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g4 = lane >> 4;
  float *T = psmem + wave * TW;
  uint16_t *perm = reinterpret_cast<uint16_t *>(psmem + kPWaves * TW);
  const int na = P.na, nb = P.nb, n = na * nb;
  for (int i = threadIdx.x; i < n; i += 64 * kPWaves) perm[i] = P.perm[i];
  for (int i = lane; i < TW; i += 64) T[i] = 0.0f;
  __syncthreads();

  // Y1 stays in the MFMA result registers: lane (g4, r16) holds Y1[16 mt + 4 g4 + v]
  // [16 nt + r16] in y1[mt][nt][v], so Y2 = A * Y1 sums over k in the order (mt, v, g4): MFMA
  // step (mt, v) takes row 16 mt + 4 g4 + v of Y1 from lane group g4, and the A fragment of
  // that step holds A[16 mo + r16][16 mt + 4 g4 + v].  Y1 = Z * B sums over k in the same
  // order, so its B fragment for step (mk, v) holds B[16 mk + 4 g4 + v][16 nt + r16]; with
  // one matrix for both factors that is af[nt][mk][v] (both are U[16 mk + 4 g4 + v]
  // [16 nt + r16], forward and inverse alike).
  // FP32 fragments (B16: unused, size 1)
  float bf[SAME || B16 ? 1 : MB][4][SAME || B16 ? 1 : MB];
  float af[B16 ? 1 : MA][B16 ? 1 : MA][4];
  // BF16 fragments: the 16x16x16 MFMA takes k = 16 kk + 4 g4 + j, j < 4, from lane group g4,
  // so step 1's B fragment (kk, nt) holds B[16 kk + 4 g4 + j][16 nt + r16] and step 2's A
  // fragment (mo, mt) holds A[16 mo + r16][16 mt + 4 g4 + j] (= B fragment (mt, mo) with one
  // matrix for both factors)
  Frag16 bq[B16 && !SAME ? MB : 1][B16 && !SAME ? MB : 1];
  Frag16 aq[B16 ? MA : 1][B16 ? MA : 1];
  if constexpr (B16) {
#pragma unroll
    for (int mo = 0; mo < MA; ++mo)
#pragma unroll
      for (int mt = 0; mt < MA; ++mt) {
        const float *a = P.amat + (16 * mo + r16) * NA + 16 * mt + 4 * g4;
        aq[mo][mt] = pack16(a[0], a[1], a[2], a[3]);
      }
    if constexpr (!SAME) {
#pragma unroll
      for (int kk = 0; kk < MB; ++kk)
#pragma unroll
        for (int nt = 0; nt < MB; ++nt) {
          const float *b = P.bmat + (16 * kk + 4 * g4) * NB + 16 * nt + r16;
          bq[kk][nt] = pack16(b[0], b[NB], b[2 * NB], b[3 * NB]);
        }
    }
  }
  if constexpr (!SAME && !B16) {
#pragma unroll
    for (int mk = 0; mk < MB; ++mk)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int nt = 0; nt < MB; ++nt) bf[mk][v][nt] = P.bmat[(16 * mk + 4 * g4 + v) * NB + 16 * nt + r16];
  }
  if constexpr (!B16) {
#pragma unroll
    for (int mo = 0; mo < MA; ++mo)
#pragma unroll
      for (int mt = 0; mt < MA; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) af[mo][mt][v] = P.amat[(16 * mo + r16) * NA + 16 * mt + 4 * g4 + v];
  }

  // LDS word of signal element e in node order (row e / nb, column e mod nb)
  const bool full = nb == NB;
  auto natural = [&](int e) -> int {
    const int i = full ? e / NB : e / nb;
    return i * STR + (e - i * nb);
  };
  auto lds_in = [&](int e) -> int { return DIR == 0 ? natural(e) : (int)perm[e]; };
  auto lds_out = [&](int e) -> int { return DIR == 0 ? (int)perm[e] : natural(e); };

  const int64_t W = (int64_t)gridDim.x * kPWaves;
  // Whole signals move as 16-byte groups when n % 4 == 0 (n % 8 == 0 with BF16 storage:
  // every signal then starts 16-byte aligned).  Load latency is covered by the other wave of
  // the SIMD, not by a prefetch (whose registers would cost that second wave).
  const bool vec = IO16 ? (n & 7) == 0 : (n & 3) == 0;
  const int nv = n >> 2;
  constexpr int MAXV8 = (NA * NB / 512) > 0 ? NA * NB / 512 : 1;   // 8-value groups per lane
  for (int64_t s = (int64_t)blockIdx.x * kPWaves + wave; s < nsig; s += W) {
    if (IO16 && vec) {
      const int nv8 = n >> 3;
      const u32x4 *src = reinterpret_cast<const u32x4 *>(in16 + s * n);
      u32x4 ld[MAXV8];
#pragma unroll
      for (int k = 0; k < MAXV8; ++k) {
        const int v = lane + 64 * k;
        ld[k] = __builtin_nontemporal_load(src + (v < nv8 ? v : nv8 - 1));
      }
#pragma unroll
      for (int k = 0; k < MAXV8; ++k) {
        const int v = lane + 64 * k;
        if (v < nv8) {
          float f[8];
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            f[2 * h] = __uint_as_float(ld[k][h] << 16);
            f[2 * h + 1] = __uint_as_float(ld[k][h] & 0xffff0000u);
          }
          if (DIR == 0 && (nb & 7) == 0) {   // a group of 8 stays inside one row
            float *row = T + natural(8 * v);
#pragma unroll
            for (int j = 0; j < 8; ++j) row[j] = f[j];
          } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) T[lds_in(8 * v + j)] = f[j];
          }
        }
      }
    } else if (IO16) {
      for (int e = lane; e < n; e += 64) T[lds_in(e)] = __uint_as_float((uint32_t)in16[s * n + e] << 16);
    } else if (vec) {
      const floatx4 *src = reinterpret_cast<const floatx4 *>(in + s * n);
      floatx4 ld[MAXV];
#pragma unroll
      for (int k = 0; k < MAXV; ++k) {
        const int v = lane + 64 * k;
        ld[k] = __builtin_nontemporal_load(src + (v < nv ? v : nv - 1));
      }
      if constexpr (TP == 1 && DIR == 0) {   // staged: the column stages in the load registers
#pragma unroll
        for (int k = 0; k < MAXV; ++k) halving_cols<false>(ld[k], r16);
      }
#pragma unroll
      for (int k = 0; k < MAXV; ++k) {
        const int v = lane + 64 * k;
        if (v < nv) {
          if (DIR == 0 && (nb & 3) == 0) {   // a group of 4 stays inside one row
            float *row = T + natural(4 * v);
#pragma unroll
            for (int j = 0; j < 4; ++j) row[j] = ld[k][j];
          } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) T[lds_in(4 * v + j)] = ld[k][j];
          }
        }
      }
    } else {
      for (int e = lane; e < n; e += 64) T[lds_in(e)] = in[s * n + e];
    }
    wave_sync();
    if constexpr (TP == 1 && DIR == 0) {   // staged: the row stages through the tile
      halving_rows<false, STR>(T, lane);
      wave_sync();
    }

    // Y1 = Z * B
    floatx4 y1[MA][MB];
#pragma unroll
    for (int mt = 0; mt < MA; ++mt) {
#pragma unroll
      for (int nt = 0; nt < MB; ++nt) y1[mt][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
      if constexpr (B16 && MB % 2 == 0) {   // k chunks kk = 2 kp, 2 kp + 1 per MFMA
#pragma unroll
        for (int kp = 0; kp < MB / 2; ++kp) {
          const float *z = T + (16 * mt + r16) * STR + 32 * kp + 4 * g4;
          const Frag16 a0 = pack16(z[0], z[1], z[2], z[3]), a1 = pack16(z[16], z[17], z[18], z[19]);
#pragma unroll
          for (int nt = 0; nt < MB; ++nt) {
            const bool on0 = tile_nz<TPM, MB>(2 * kp, nt), on1 = tile_nz<TPM, MB>(2 * kp + 1, nt);
            Frag16 b0, b1;
            if constexpr (SAME) {
              b0 = aq[nt][2 * kp];
              b1 = aq[nt][2 * kp + 1];
            } else {
              b0 = bq[2 * kp][nt];
              b1 = bq[2 * kp + 1][nt];
            }
            if (on0 && on1) y1[mt][nt] = mfma32<PREC == kSPLIT>(a0, a1, b0, b1, y1[mt][nt]);
            else if (on0) y1[mt][nt] = mfma16<PREC == kSPLIT>(a0, b0, y1[mt][nt]);
            else if (on1) y1[mt][nt] = mfma16<PREC == kSPLIT>(a1, b1, y1[mt][nt]);
          }
        }
      } else if constexpr (B16) {
#pragma unroll
        for (int kk = 0; kk < MB; ++kk) {
          const float *z = T + (16 * mt + r16) * STR + 16 * kk + 4 * g4;
          const Frag16 a = pack16(z[0], z[1], z[2], z[3]);
#pragma unroll
          for (int nt = 0; nt < MB; ++nt) {
            if (!tile_nz<TPM, MB>(kk, nt)) continue;
            if constexpr (SAME) y1[mt][nt] = mfma16<PREC == kSPLIT>(a, aq[nt][kk], y1[mt][nt]);
            else y1[mt][nt] = mfma16<PREC == kSPLIT>(a, bq[kk][nt], y1[mt][nt]);
          }
        }
      } else {
#pragma unroll
        for (int mk = 0; mk < MB; ++mk)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float a = T[(16 * mt + r16) * STR + 16 * mk + 4 * g4 + v];
#pragma unroll
            for (int nt = 0; nt < MB; ++nt) {
              if (!tile_nz<TPM, MB>(mk, nt)) continue;
              float b;
              if constexpr (SAME) b = af[nt][mk][v];
              else b = bf[mk][v][nt];
              y1[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, y1[mt][nt], 0, 0, 0);
            }
          }
      }
    }
    wave_sync();   // every read of Z is done before Y2 overwrites the tile

    // Y2 = A * Y1, one 16-column block at a time, into the tile
#pragma unroll
    for (int nt = 0; nt < MB; ++nt) {
      floatx4 acc[MA];
#pragma unroll
      for (int mo = 0; mo < MA; ++mo) acc[mo] = floatx4{0.f, 0.f, 0.f, 0.f};
      if constexpr (B16 && MA % 2 == 0) {
        // the result registers y1[mt][nt] are already the B operand of k chunk mt; chunks
        // 2 mp and 2 mp + 1 go to one MFMA
#pragma unroll
        for (int mp = 0; mp < MA / 2; ++mp) {
          const floatx4 y0 = y1[2 * mp][nt], y1v = y1[2 * mp + 1][nt];
          const Frag16 b0 = pack16(y0[0], y0[1], y0[2], y0[3]), b1 = pack16(y1v[0], y1v[1], y1v[2], y1v[3]);
#pragma unroll
          for (int mo = 0; mo < MA; ++mo) {
            const bool on0 = tile_nz<TPM, MA>(mo, 2 * mp), on1 = tile_nz<TPM, MA>(mo, 2 * mp + 1);
            if (on0 && on1) acc[mo] = mfma32<PREC == kSPLIT>(aq[mo][2 * mp], aq[mo][2 * mp + 1], b0, b1, acc[mo]);
            else if (on0) acc[mo] = mfma16<PREC == kSPLIT>(aq[mo][2 * mp], b0, acc[mo]);
            else if (on1) acc[mo] = mfma16<PREC == kSPLIT>(aq[mo][2 * mp + 1], b1, acc[mo]);
          }
        }
      } else if constexpr (B16) {
        // the result registers y1[mt][nt] are already the B operand of k chunk mt
#pragma unroll
        for (int mt = 0; mt < MA; ++mt) {
          const floatx4 y = y1[mt][nt];
          const Frag16 b = pack16(y[0], y[1], y[2], y[3]);
#pragma unroll
          for (int mo = 0; mo < MA; ++mo)
            if (tile_nz<TPM, MA>(mo, mt)) acc[mo] = mfma16<PREC == kSPLIT>(aq[mo][mt], b, acc[mo]);
        }
      } else {
#pragma unroll
        for (int mt = 0; mt < MA; ++mt)
#pragma unroll
          for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int mo = 0; mo < MA; ++mo)
              if (tile_nz<TPM, MA>(mo, mt))
                acc[mo] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mo][mt][v], y1[mt][nt][v], acc[mo], 0, 0, 0);
      }
#pragma unroll
      for (int mo = 0; mo < MA; ++mo)
#pragma unroll
        for (int v = 0; v < 4; ++v) T[(16 * mo + 4 * g4 + v) * STR + 16 * nt + r16] = acc[mo][v];
    }
    wave_sync();
    if constexpr (TP == 1 && DIR == 1) {   // staged: the row stages through the tile
      halving_rows<true, STR>(T, lane);
      wave_sync();
    }

    if (IO16 && vec) {
      const int nv8 = n >> 3;
      u32x4 *dst = reinterpret_cast<u32x4 *>(out16 + s * n);
      for (int v = lane; v < nv8; v += 64) {
        const int e = 8 * v;
        u32x4 o;
#pragma unroll
        for (int h = 0; h < 4; ++h)
          o[h] = bf16_pair(T[lds_out(e + 2 * h)], T[lds_out(e + 2 * h + 1)]);
        __builtin_nontemporal_store(o, dst + v);
      }
    } else if (IO16) {
      for (int e = lane; e < n; e += 64) out16[s * n + e] = (uint16_t)bf16_rne(T[lds_out(e)]);
    } else if (TP == 1 && DIR == 1) {   // staged inverse (full 64 x 64 signals): the column stages
      floatx4 *dst = reinterpret_cast<floatx4 *>(out + s * n);
#pragma unroll
      for (int k = 0; k < MAXV; ++k) {
        const int v = lane + 64 * k;
        const float *row = T + natural(4 * v);
        floatx4 o = {row[0], row[1], row[2], row[3]};
        halving_cols<true>(o, r16);
        __builtin_nontemporal_store(o, dst + v);
      }
    } else if (vec) {
      floatx4 *dst = reinterpret_cast<floatx4 *>(out + s * n);
#pragma unroll 2
      for (int v = lane; v < nv; v += 64) {
        const int e = 4 * v;
        const floatx4 o = {T[lds_out(e)], T[lds_out(e + 1)], T[lds_out(e + 2)], T[lds_out(e + 3)]};
        __builtin_nontemporal_store(o, dst + v);
      }
    } else {
      for (int e = lane; e < n; e += 64) out[s * n + e] = T[lds_out(e)];
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------------------- launch

// grid_cap > 0: launch at most that many workgroups; num_cus < 0: only report the
// occupancy through *occ_out.
template <int NA, int NB, int DIR, bool SAME, int PREC, int TP>
static hipError_t launch_pdp(const PProgram &P, const void *in, void *out, int64_t nsig,
                             hipStream_t stream, int num_cus, int grid_cap, int *occ_out) {
  const size_t lds = product_lds_bytes<NA, NB>(P.na * P.nb);
  const void *k = (const void *)gft_product<NA, NB, DIR, SAME, PREC, TP>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, gft_product<NA, NB, DIR, SAME, PREC, TP>, 64 * kPWaves, lds) !=
          hipSuccess || occ < 1)
    occ = 1;
  if (occ_out) *occ_out = occ;
  if (num_cus < 0) return hipSuccess;
  const int64_t want = (nsig + kPWaves - 1) / kPWaves;
  const int64_t cap = grid_cap > 0 ? grid_cap : (int64_t)occ * (num_cus > 0 ? num_cus : 1);
  const int grid = (int)(want < cap ? want : cap);
  hipLaunchKernelGGL((gft_product<NA, NB, DIR, SAME, PREC, TP>), dim3(grid > 0 ? grid : 1), dim3(64 * kPWaves), lds,
                     stream, P, in, out, nsig);
  return hipGetLastError();
}

template <int NA, int NB, int DIR, bool SAME, int TP>
static hipError_t launch_pdt(const PProgram &P, const void *in, void *out, int64_t nsig,
                             hipStream_t stream, int num_cus, int grid_cap, int *occ_out) {
  switch (P.prec) {
    case kFP32: return launch_pdp<NA, NB, DIR, SAME, kFP32, TP>(P, in, out, nsig, stream, num_cus, grid_cap, occ_out);
    case kBF16: return launch_pdp<NA, NB, DIR, SAME, kBF16, TP>(P, in, out, nsig, stream, num_cus, grid_cap, occ_out);
    case kSPLIT: return launch_pdp<NA, NB, DIR, SAME, kSPLIT, TP>(P, in, out, nsig, stream, num_cus, grid_cap, occ_out);
    default: return hipErrorInvalidValue;
  }
}

// IO16: the BF16-storage instantiations (tile pattern 2, dense factors), compiled in their
// own translation unit; else FP32 storage, dense (pattern 0) or staged (pattern 1).
template <int NA, int NB, int DIR, bool SAME, bool IO16>
static hipError_t launch_pd(const PProgram &P, const void *in, void *out, int64_t nsig,
                            hipStream_t stream, int num_cus, int grid_cap, int *occ_out) {
  if constexpr (IO16) {
    if (P.tile_pattern != 2) return hipErrorInvalidValue;
    return launch_pdt<NA, NB, DIR, SAME, 2>(P, in, out, nsig, stream, num_cus, grid_cap, occ_out);
  } else {
    if constexpr (NA == 64 && NB == 64) {
      if (P.tile_pattern == 1) {
        if (P.na != 64 || P.nb != 64) return hipErrorInvalidValue;
        return launch_pdt<NA, NB, DIR, SAME, 1>(P, in, out, nsig, stream, num_cus, grid_cap, occ_out);
      }
    }
    if (P.tile_pattern != 0) return hipErrorInvalidValue;
    return launch_pdt<NA, NB, DIR, SAME, 0>(P, in, out, nsig, stream, num_cus, grid_cap, occ_out);
  }
}

template <int NA, int NB, bool IO16>
static hipError_t launch_pab(const PProgram &P, const void *in, void *out, int64_t nsig,
                             hipStream_t stream, int num_cus, int grid_cap, int *occ_out) {
  if constexpr (NA == NB) {
    if (P.same)
      return P.dir == 0 ? launch_pd<NA, NB, 0, true, IO16>(P, in, out, nsig, stream, num_cus, grid_cap, occ_out)
                        : launch_pd<NA, NB, 1, true, IO16>(P, in, out, nsig, stream, num_cus, grid_cap, occ_out);
  }
  return P.dir == 0 ? launch_pd<NA, NB, 0, false, IO16>(P, in, out, nsig, stream, num_cus, grid_cap, occ_out)
                    : launch_pd<NA, NB, 1, false, IO16>(P, in, out, nsig, stream, num_cus, grid_cap, occ_out);
}

template <bool IO16>
static hipError_t dispatch_product(const PProgram &P, const void *in, void *out, int64_t nsig,
                                   hipStream_t stream, int num_cus, int grid_cap, int *occ_out) {
  const int NA = product_pad_size(P.na), NB = product_pad_size(P.nb);
  if (P.stride != NB + 1) return hipErrorInvalidValue;
#define GFT_PROD_CASE(a, b) \
  if (NA == a && NB == b) return launch_pab<a, b, IO16>(P, in, out, nsig, stream, num_cus, grid_cap, occ_out);
  GFT_PROD_CASE(16, 16)
  GFT_PROD_CASE(16, 32)
  GFT_PROD_CASE(16, 64)
  GFT_PROD_CASE(32, 16)
  GFT_PROD_CASE(32, 32)
  GFT_PROD_CASE(32, 64)
  GFT_PROD_CASE(64, 16)
  GFT_PROD_CASE(64, 32)
  GFT_PROD_CASE(64, 64)
#undef GFT_PROD_CASE
  return hipErrorInvalidValue;
}

}  // namespace gft
