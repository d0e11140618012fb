// Register-butterfly tile loop of the GFT kernels (gfx950), shared by the single-graph
// butterfly kernel and the mixed-batch kernel.
//
// A plan whose S butterfly stages each pair every node (eq. B_phi with V_Z empty), with
// 2^S equal leaf blocks of M nodes, factors U^T as 2^S dense M x M sub-GFTs after S
// stages of Haar units; every Haar orbit holds one node of every block (the grid of
// Fig. grid_coords under LR then UD symmetry is the case n = 64, S = 2, M = 16).  One-stage
// plans of other shapes are laid out on padded slots (GEN below).
// Each wave works alone on tiles of 16 signals, with no workgroup barriers:
//   HBM --16B loads, prefetched PF tiles ahead--> registers (native vector type: arrays
//   of the HIP float4 struct are not promoted out of scratch) --> wave-private LDS tile
//   --gather--> registers in MFMA operand order: lane (g, r) holds, for signal r, the
//   2^S slots of the orbits assigned to lane group g
//   --> Haar stages as register add/sub (forward) --> v_mfma_f32_16x16x4_f32 with the
//   block matrices resident in registers --> Haar stages (inverse) --> scatter to the
//   LDS tile in output order --> 16B stores.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_program.hpp"

namespace gft {
namespace bfly {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// x with its sign flipped when bit f is set.
__device__ __forceinline__ float flip_sign(float x, uint32_t f) {
  return __int_as_float(__float_as_int(x) ^ (int)(f << 31));
}

// Orders this wave's LDS accesses: every lane's earlier LDS operations complete (and the
// compiler keeps them in place) before any later one.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// FP32 <- BF16 pairs packed in a 32-bit word (element 2i in the low half).
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// FP32 -> BF16 bits, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// LDS words one wave's tile region needs: the tile (16 rows of stride N + 4), then the zero
// and scratch words of padded slots.
template <int S, int M>
constexpr int tile_words() { return 16 * ((M << S) + 4) + 4; }

// IN16 / OUT16: the tile is read / written as BF16 (16-byte accesses of 8 values) instead
// of FP32 (16-byte accesses of 4 values); everything between runs in FP32.
// GEN: a one-stage program with n = P.n <= N signal values (n >= 8), padded slots: a
// gather column of -1 reads a zero word and a scatter column of -1 writes a scratch word.
// The LDS tile keeps the 16 signals' own contiguous layout (row stride n) when n is odd or
// n = 2 mod 4, where 16 rows at stride n fall in distinct banks; for 4 | n rows are padded
// to a stride = 4 mod 8 (n + 4 or n + 8), which keeps 16-byte groups inside a row.
// BF: BF16 leaf blocks (one-stage programs): the block inputs are rounded to BF16 after the
// FP32 Haar stage and multiplied on 16x16x16 BF16 MFMA with FP32 accumulation.
// Tiles wt, wt + step, ... (< wend) of the nsig signals at in / out, by this wave, with T
// its private LDS region of tile_words<S, M>() words.
// LEAN: fewer live registers, for kernels that hold several forms at once: the LDS offsets
// are kept as 16-bit pairs and a tile's loads are issued when the tile starts (no prefetch
// of the next tile; other waves cover the latency).
// PF (not LEAN): tiles whose loads are in flight while a tile is computed.  One suffices
// where many waves share a SIMD; a kernel held to few waves by its register budget keeps
// more loads in flight per wave with PF register sets (the tile loop is unrolled PF times,
// so that each set keeps fixed registers).
template <int S, int M, int DIR, bool IN16, bool OUT16, bool GEN, bool BF, bool LEAN = false,
          int PF = 1>
__device__ __forceinline__ void butterfly_tiles(const UProgram &P, const void *in, void *out,
                                                int64_t nsig, int64_t wt, int64_t wend,
                                                int64_t step, float *T) {
  constexpr int NB = 1 << S;      // leaf blocks = slots per orbit
  constexpr int KC = M / 4;       // K chunks of a block
  constexpr int NT = M / 16;      // 16-row tiles of a block
  constexpr int N = M * NB;       // slots per signal (= n unless GEN)
  constexpr int Q = N / 4;        // values per lane
  constexpr int STR = N + 4;      // LDS row stride: 16-byte rows, offset banks
  constexpr int NF = NB * NT * KC;

  const int lane = threadIdx.x & 63;
  const int g = lane >> 4;
  const int r = lane & 15;
  const int n = GEN ? P.n : N;           // values per signal in memory
  // LDS row stride (GEN: n + 8 <= N + 4 when n = 4 mod 8, since then n <= N - 4)
  const int rstride = !GEN ? STR : ((n & 3) ? n : ((n & 7) ? n + 8 : n + 4));
  const bool packed = GEN && rstride == n;   // tile word e of the signals is LDS word e
  constexpr int kZero = 16 * STR, kScratch = 16 * STR + 1;   // past any tile word (GEN)
  // LDS word of tile element e < 16 n (a row-padded tile: row e / n, column e % n)
  auto tw = [&](int e) -> int { return packed ? e : (GEN ? (e / n) * rstride + e % n : (e / N) * STR + (e % N)); };

  // LDS offsets of this lane's gathers and scatters
  constexpr int QO = LEAN ? (Q + 1) / 2 : Q;   // offset registers (LEAN: two per register)
  int gc[QO], sc[QO];
  constexpr int NAF = BF ? NF / 2 : NF;   // BF16: 2 words per 4-k fragment
  float af[NAF];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int gq = P.gcol[g * Q + q], sq = P.scol[g * Q + q];
    const int go = gq >= 0 ? r * rstride + gq : kZero;
    const int so = sq >= 0 ? r * rstride + sq : kScratch;
    if constexpr (LEAN) {   // words < 2^16: the tile region has at most 16 * 100 + 4 words
      if (q & 1) {
        gc[q / 2] |= go << 16;
        sc[q / 2] |= so << 16;
      } else {
        gc[q / 2] = go;
        sc[q / 2] = so;
      }
    } else {
      gc[q] = go;
      sc[q] = so;
    }
  }
  auto gat = [&](int q) -> int { return LEAN ? (gc[q / 2] >> (16 * (q & 1))) & 0xffff : gc[q]; };
  auto sat = [&](int q) -> int { return LEAN ? (sc[q / 2] >> (16 * (q & 1))) & 0xffff : sc[q]; };
  if constexpr (GEN) {
    if (lane == 0) T[kZero] = 0.0f;
  }
#pragma unroll
  for (int f = 0; f < NAF; ++f) af[f] = BF ? P.afrag[((f >> 1) * 64 + lane) * 2 + (f & 1)] : P.afrag[f * 64 + lane];
  constexpr int PPS = NB / 2;
  constexpr int FB = S * PPS;
  const uint64_t flips = ((uint64_t)P.flips[2 * g + 1] << 32) | P.flips[2 * g];


  // Prefetch of a tile into registers.  The loads are unconditional, so that they stay in
  // flight while the previous tile is computed: past the last valid signal a lane
  // re-reads the tile's last 16 bytes (lim >= n >= 8), whose rows are never stored.
  constexpr int EI = IN16 ? 8 : 4;          // values per 16-byte load
  constexpr int VI = N / (4 * EI);          // loads per lane per 16-signal tile (16n <= 16N)
  constexpr int H = EI / 4;                 // LDS groups of 4 values per load
  static_assert(PF >= 1 && (PF == 1 || !LEAN), "prefetch depth");
  u32x4 pre[PF][VI];
  // LDS words of this lane's load groups (-1: past the tile's 16 rows, never written)
  int ld_at[VI * H];
#pragma unroll
  for (int k = 0; k < VI; ++k)
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int e = EI * (lane + 64 * k) + 4 * h;
      ld_at[k * H + h] = packed || e < 16 * n ? tw(e) : -1;
    }
  // Whole 16-byte groups only: a tile's last lim mod EI values (GEN partial tiles) are read
  // by scalar loads in the loop below.
  auto issue = [&](int64_t t, u32x4(&dst)[VI]) {
    const int64_t rem = nsig - 16 * t;
    const int limv = ((int)(rem < 16 ? rem : 16) * n) & ~(EI - 1);
#pragma unroll
    for (int k = 0; k < VI; ++k) {
      const int e = EI * (lane + 64 * k);
      const int ec = e < limv ? e : limv - EI;
      if constexpr (IN16)
        dst[k] = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(static_cast<const uint16_t *>(in) + t * 16 * n + ec));
      else
        dst[k] = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(static_cast<const float *>(in) + t * 16 * n + ec));
    }
  };
  // loads of the first PF tiles (tiles past the wave's last one re-read that tile rather
  // than branch around the loads)
  if (!LEAN && wt < wend) {
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int64_t t = wt + j * step;
      issue(t < wend ? t : wend - 1, pre[j]);
    }
  }

  constexpr int EO = OUT16 ? 8 : 4;         // values per 16-byte store
  constexpr int VO = N / (4 * EO);
  constexpr int HO = EO / 4;
  // LDS words of this lane's store groups (past the tile's 16 rows: word 0, never stored)
  int st_at[VO * HO];
#pragma unroll
  for (int k = 0; k < VO; ++k)
#pragma unroll
    for (int h = 0; h < HO; ++h) {
      const int e = EO * (lane + 64 * k) + 4 * h;
      st_at[k * HO + h] = packed || e < 16 * n ? tw(e) : 0;
    }

  while (wt < wend) {
#pragma unroll
    for (int j = 0; j < PF; ++j, wt += step) {
      if (wt >= wend) break;
      u32x4(&cur)[VI] = pre[j];
      const int64_t rem = nsig - 16 * wt;
      const int lim = (int)(rem < 16 ? rem : 16) * n;
      if constexpr (LEAN) issue(wt, cur);
#pragma unroll
      for (int k = 0; k < VI; ++k) {
        // a group of 4 values never crosses a row (4 | N, and 4 | n where GEN rows are
        // padded); a packed GEN tile is contiguous and the words past 16n it receives are
        // never gathered
        if constexpr (IN16) {
          const u32x4 w = cur[k];
          if (ld_at[2 * k] >= 0)
            *reinterpret_cast<floatx4 *>(T + ld_at[2 * k]) = floatx4{bf16_lo(w[0]), bf16_hi(w[0]), bf16_lo(w[1]), bf16_hi(w[1])};
          if (ld_at[2 * k + 1] >= 0)
            *reinterpret_cast<floatx4 *>(T + ld_at[2 * k + 1]) = floatx4{bf16_lo(w[2]), bf16_hi(w[2]), bf16_lo(w[3]), bf16_hi(w[3])};
        } else {
          if (ld_at[k] >= 0) *reinterpret_cast<u32x4 *>(T + ld_at[k]) = cur[k];
        }
      }
      if constexpr (GEN) {
        for (int e = (lim & ~(EI - 1)) + lane; e < lim; e += 64) {   // partial tile's tail
          if constexpr (IN16)
            T[tw(e)] = __uint_as_float((uint32_t)static_cast<const uint16_t *>(in)[wt * 16 * n + e] << 16);
          else
            T[tw(e)] = static_cast<const float *>(in)[wt * 16 * n + e];
        }
      }
      wave_lds_sync();
      // loads of the tile PF steps ahead into the register set just emptied
      if constexpr (!LEAN) {
        const int64_t nxt = wt + PF * step;
        issue(nxt < wend ? nxt : wend - 1, cur);
      }

      float d[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) d[q] = T[gat(q)];

      if (DIR == 0) {
        // forward Haar stages, in stage order: slots lo and lo | bit, bit = 2^(S-1-t)
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
          for (int t = 0; t < S; ++t) {
            const int bit = 1 << (S - 1 - t);
            int k = 0;
#pragma unroll
            for (int b = 0; b < NB; ++b)
              if (!(b & bit)) {
                const uint32_t f = (uint32_t)(flips >> (kc * FB + t * PPS + k)) & 1u;
                const float a = d[kc * NB + b], c = d[kc * NB + (b | bit)];
                d[kc * NB + b] = a + c;
                d[kc * NB + (b | bit)] = flip_sign(a - c, f);
                ++k;
              }
          }
      }

      float res[Q];
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          floatx4 acc = {0.f, 0.f, 0.f, 0.f};
          if constexpr (BF) {
#pragma unroll
            for (int k4 = 0; k4 < KC / 4; ++k4) {
              const int f = (b * NT + nt) * (KC / 4) + k4;
              const u32x2 aw = {__float_as_uint(af[2 * f]), __float_as_uint(af[2 * f + 1])};
              const u32x2 bw = {bf16_bits(d[(4 * k4) * NB + b]) | (bf16_bits(d[(4 * k4 + 1) * NB + b]) << 16),
                                bf16_bits(d[(4 * k4 + 2) * NB + b]) | (bf16_bits(d[(4 * k4 + 3) * NB + b]) << 16)};
              acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(bf16x4, aw),
                                                              __builtin_bit_cast(bf16x4, bw), acc, 0, 0, 0);
            }
          } else {
#pragma unroll
            for (int kc = 0; kc < KC; ++kc)
              acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[(b * NT + nt) * KC + kc], d[kc * NB + b],
                                                         acc, 0, 0, 0);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if (DIR == 0) res[(b * NT + nt) * 4 + v] = acc[v];
            else res[(nt * 4 + v) * NB + b] = acc[v];
          }
        }

      if (DIR == 1) {
        // inverse Haar stages, in reverse stage order, on each orbit's 2^S slots
#pragma unroll
        for (int o = 0; o < NT * 4; ++o)
#pragma unroll
          for (int t = S - 1; t >= 0; --t) {
            const int bit = 1 << (S - 1 - t);
            int k = 0;
#pragma unroll
            for (int b = 0; b < NB; ++b)
              if (!(b & bit)) {
                const uint32_t f = (uint32_t)(flips >> (o * FB + t * PPS + k)) & 1u;
                const float a = res[o * NB + b], c = flip_sign(res[o * NB + (b | bit)], f);
                res[o * NB + b] = a + c;
                res[o * NB + (b | bit)] = a - c;
                ++k;
              }
          }
      }

      wave_lds_sync();
#pragma unroll
      for (int q = 0; q < Q; ++q) T[sat(q)] = res[q];
      wave_lds_sync();
      u32x4 o[VO];
#pragma unroll
      for (int k = 0; k < VO; ++k) {
        const float *src = T + st_at[k * HO];
        if constexpr (OUT16) {
          const floatx4 a = *reinterpret_cast<const floatx4 *>(src);
          const floatx4 b = *reinterpret_cast<const floatx4 *>(T + st_at[k * HO + 1]);
          o[k] = u32x4{bf16_bits(a[0]) | (bf16_bits(a[1]) << 16), bf16_bits(a[2]) | (bf16_bits(a[3]) << 16),
                       bf16_bits(b[0]) | (bf16_bits(b[1]) << 16), bf16_bits(b[2]) | (bf16_bits(b[3]) << 16)};
        } else {
          o[k] = *reinterpret_cast<const u32x4 *>(src);
        }
      }
      auto dst_at = [&](int e) -> u32x4 * {
        if constexpr (OUT16)
          return reinterpret_cast<u32x4 *>(static_cast<uint16_t *>(out) + wt * 16 * n + e);
        else
          return reinterpret_cast<u32x4 *>(static_cast<float *>(out) + wt * 16 * n + e);
      };
      if (!GEN && lim == 16 * N) {   // full tile (wave-uniform branch)
#pragma unroll
        for (int k = 0; k < VO; ++k) __builtin_nontemporal_store(o[k], dst_at(EO * (lane + 64 * k)));
      } else {
        const int limv = lim & ~(EO - 1);   // whole groups; GEN tail values stored one by one
#pragma unroll
        for (int k = 0; k < VO; ++k)
          if (EO * (lane + 64 * k) < limv) __builtin_nontemporal_store(o[k], dst_at(EO * (lane + 64 * k)));
        if constexpr (GEN) {
          for (int e = limv + lane; e < lim; e += 64) {
            if constexpr (OUT16)
              static_cast<uint16_t *>(out)[wt * 16 * n + e] = (uint16_t)bf16_bits(T[tw(e)]);
            else
              static_cast<float *>(out)[wt * 16 * n + e] = T[tw(e)];
          }
        }
      }
      wave_lds_sync();
    }
  }
}

}  // namespace bfly
}  // namespace gft
