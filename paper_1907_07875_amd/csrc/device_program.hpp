// Device image of a plan: the data-driven program the GFT kernels interpret.
//
// One program per (graph, direction).  The forward program runs the Haar stages before
// the blocks; the inverse runs the blocks first and the stages after, in reverse order
// (each B_phi is symmetric and orthogonal, eq. Bnp, so the same add/sub undoes it).
#pragma once

#include <cstdint>

namespace gft {

// A butterfly stage: `cnt` ops starting at `off` in the op table.  op = (i, j): Haar unit
// x_i <- x_i + x_j, x_j <- x_i - x_j; op = (c, -1): x_c <- sqrt(2) x_c (a V_Z node).
// magic = ceil(2^32 / cnt) for division of (signal, op) item indices by cnt.
struct DevStage {
  int32_t off;
  int32_t cnt;
  uint32_t magic;
  int32_t pad;
};

// A dense leaf block, applied as a [T x K] * [K x N] product on MFMA 16x16x4 f32 tiles.
// gidx[gidx_off + k], k < 4*kchunks: source column of input k (padding points at a valid
// column; its matrix row is zero).  sidx[sidx_off + c], c < size: destination column of
// output c.  The matrix is stored as per-lane fragments: frag[frag_off +
// ((kc * ntiles) + nt) * 64 + lane] = M[4*kc + lane/16][16*nt + lane%16] (zero padded).
struct DevBlock {
  int32_t size;
  int32_t kchunks;
  int32_t ntiles;
  int32_t gidx_off;
  int32_t sidx_off;
  int32_t frag_off;
  int32_t pad[2];
};

struct DevProgram {
  int32_t n;          // signal length
  int32_t stride;     // LDS row stride in floats (odd, >= n)
  int32_t mt;         // 16-signal M-tiles per tile; tile = 16*mt signals
  int32_t num_pre;    // stages [0, num_pre) run before the blocks
  int32_t num_post;   // stages [num_pre, num_pre+num_post) run after the blocks
  int32_t num_items;  // (block, n-tile) work items of the block phase
  int32_t num_blocks;
  int32_t total_ops;  // op-table length
  int32_t gidx_len;
  int32_t sidx_len;
  uint32_t magic_n;   // ceil(2^32 / n)
  int32_t table_words;  // int32 words of the LDS-resident tables
  // stages (4 words each) | ops (2 each) | blocks (8 each) | items | gidx | sidx,
  // contiguous; each workgroup copies it to LDS once
  const int32_t *table;
  const float *frag;
};

}  // namespace gft
