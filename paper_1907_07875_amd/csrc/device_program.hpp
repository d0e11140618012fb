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

// A dense leaf block, applied as a [T x K] * [K x N] product on 16x16 MFMA tiles whose K
// step is KS = 4 (FP32, v_mfma_f32_16x16x4_f32) or 16 (BF16/FP16/split, the 16x16x16
// MFMAs).  gidx[gidx_off + k], k < KS*kchunks: source column of input k (padding points at
// a valid column; its matrix row is zero).  sidx[sidx_off + c], c < size: destination
// column of output c.  The matrix is stored as per-lane fragments, at 32-bit word offset
// frag_off, one fragment per (kc, nt) in the order (kc * ntiles + nt):
//   FP32:   1 word per lane:  M[4*kc + lane/16][16*nt + lane%16];
//   16-bit: 2 words per lane: M[16*kc + 4*(lane/16) + j][16*nt + lane%16], j = 0..3;
//   split:  4 words per lane: the hi fragment's 2 words, then the lo fragment's 2 words.
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
  int32_t stride;     // LDS row stride in floats: n (n odd), n + 4 (4 | n), else n + 1
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
  int32_t frag_lds;     // 1: the fragments are copied to LDS after the tables (else read
                        // from global memory)
  int32_t frag_words;   // 32-bit words of `frag`
  int32_t prec;         // gft_precision of the leaf blocks
  // stages (4 words each) | ops (2 each) | blocks (8 each) | items | gidx | sidx,
  // contiguous; each workgroup copies it to LDS once
  const int32_t *table;
  const uint32_t *frag;
};

// Register-butterfly program (uniform hypercube plans, and one-stage plans with n >= 8
// padded to 2M slots, gen = 1, where gcol / scol entries of -1 read a zero / write nowhere): S stages,
// 2^S leaf blocks of M nodes, n = M * 2^S; orbit o (o < M) holds node node(o, b) of every block b at block
// position o, and stage t pairs slots b and b ^ 2^(S-1-t).  Lane l of a wave works on
// signal l % 16 of a 16-signal tile and on lane group g = l / 16.
//   gcol[g * Q + q] (Q = n/4): LDS column the lane gathers into data register q;
//   scol[g * Q + q]: LDS column the lane scatters result register q to;
//   afrag[f * 64 + l]: MFMA A-operand fragment f for lane l;
//   flips[2g], flips[2g+1]: low and high words of the 64 sign-flip bits of group g.
// A node enters at its initial slot and leaves stage S-1 at its final slot, which is its
// leaf block.  At stage t every orbit combines slots (lo, hi = lo | 2^(S-1-t)) into
// (lo + hi, +-(lo - hi)); the sign is flipped where the V_X node started in slot hi.
// Flip bit of orbit register set j, stage t, lo-slot rank k: j * S * 2^(S-1) + t * 2^(S-1) + k,
// where j = kc (forward) or nt * 4 + v (inverse).
// BF16 programs (16x16x16 MFMA, 4 k values per lane) put orbit 16(kc/4) + 4g + kc%4 in data
// register set kc instead, and their afrag holds 2 words (4 BF16) per lane per fragment
// f = (b * M/16 + nt) * M/16 + kc/4.
// Register order (forward): data q = kc * 2^S + b (orbit 4kc+g, slot b); results
// q = (b * M/16 + nt) * 4 + v (coefficient 16nt+4g+v of block b).  Inverse: data
// q = kc * 2^S + b (coefficient 4kc+g of block b); results q = (nt * 4 + v) * 2^S + b
// (orbit 16nt+4g+v, slot b).  Fragment f = (b * M/16 + nt) * M/4 + kc.
struct UProgram {
  int32_t S;
  int32_t M;
  int32_t n;
  int32_t dir;
  int32_t prec;             // gft_precision of the blocks: FP32, or BF16 (one-stage programs)
  int32_t gen;              // 1: the padded one-stage layout (n <= 2M), 0: uniform (n = M 2^S)
  const int32_t *gcol;
  const int32_t *scol;
  const uint32_t *flips;
  const float *afrag;
};

// Register-butterfly shapes with a compiled single-graph kernel: uniform (gen = 0) S = 1
// with M = 16 or 32, S = 2 or 3 with M = 16; padded (gen = 1) S = 1 with M = 16, 32 or 48,
// S = 2 with M = 16 or 32.
inline bool butterfly_shape_compiled(int S, int M, bool gen) {
  if (gen) return (S == 1 && (M == 16 || M == 32 || M == 48)) || (S == 2 && (M == 16 || M == 32));
  return (S == 1 && (M == 16 || M == 32)) || ((S == 2 || S == 3) && M == 16);
}

// Large-signal engine (signals that do not fit a workgroup's LDS tile, or large leaf
// blocks): three passes through a block-contiguous workspace W with row stride ldw.
//   pass 1 / pass 3 (stage + gather): a tile of a few signal rows is copied as is into LDS
//     (row stride in_cols), the Haar stages run on it (pass with num_stages > 0 only; the
//     op indices are tile columns), and output column c of each row takes tile column
//     gather[c] (-1: zero; gather null: identity);
//   pass 2 (grouped GEMM): W2[:, off_b : off_b + b] = W[:, off_b : off_b + b] * M_b for
//     every leaf block b, MFMA tiles.  With BF16 blocks, W and the matrices are stored in
//     BF16 (pass 1 rounds its output), W2 stays FP32.  M_b is stored transposed (row c of the stored
//     matrix is column c of M_b, row stride ld_b), so both operands are contiguous in k.
// Forward: x -[stages, gather]-> W (block layout) -[GEMM]-> W2 -[gather]-> y (output order).
// Inverse: y -[gather]-> W (block layout) -[GEMM]-> W2 -[stages, gather]-> x.
struct PermPass {
  int32_t in_cols;          // input row length = input row stride = tile row stride
  int32_t out_cols;         // output row length = output row stride
  int32_t num_stages;       // Haar stages applied to the tile
  const int32_t *gather;    // out_cols entries: tile column of each output column (or null)
  const int32_t *stages;    // 2 words per stage: op offset, op count
  const uint32_t *ops;      // per op: i | j << 16 (tile columns); j = 0xffff: scale i by sqrt 2
};

struct LBlock {
  int32_t size;     // b
  int32_t col;      // column offset in the workspace (multiple of 8)
  int32_t mat;      // offset of M_b^T in the matrix array (elements, multiple of 8)
  int32_t ld;       // row stride of M_b^T (multiple of 8, >= b)
  int32_t omap;     // offset of the block's output positions in the output map (forward)
};

// Product-graph program (one direction): the GFT of a Cartesian product G_a x G_b (node
// (i, j) = i * nb + j) is U_a (x) U_b, so a signal X (na x nb, row-major) maps to
// U_a^T X U_b.  The kernel computes Y1 = Z * B then Y2 = A * Y1 on zero-padded NA x NA and
// NB x NB matrices, Z the signal (forward) or the coefficients placed by perm (inverse).
//   forward: B = U_b, A = U_a^T, the coefficients leave in output order through perm;
//   inverse: B = U_b^T, A = U_a, the signal leaves in node order.
struct PProgram {
  int32_t na, nb;           // factor sizes (<= the kernel's NA, NB)
  int32_t dir;
  int32_t stride;           // LDS row stride of the wave's tile (NB + 1)
  int32_t same;             // 1: U_a = U_b (one graph squared), one set of fragments
  int32_t prec;             // gft_precision of the products: FP32, BF16 or split BF16
  const float *amat;        // NA x NA row-major, zero beyond na
  const float *bmat;        // NB x NB row-major, zero beyond nb
  const uint16_t *perm;     // na * nb entries: LDS word p * stride + q of output-order
                            // coefficient k (its factor indices p, q)
  // 0: dense factors.  1: staged 64-node factors whose stages are the halving reversals
  // (R = 64, 32, ..., 2: node i < R/2 paired with R - 1 - i), compiled into the kernel;
  // amat and bmat then hold the block-diagonal leaf matrices (rows and columns: node
  // positions and block-order coefficients) and the stages run as add/sub on the signal.
  int32_t tile_pattern;
};

}  // namespace gft

namespace gft {

// One-pass form of the large-signal engine (plans whose first pass has at most one Haar
// stage and whose leaf blocks, one or two, fit one workgroup's columns): one kernel stages
// the first pass's values straight from the input rows, multiplies them by the blocks on
// MFMA tiles and runs the last pass (its stages and gather) on the results in LDS, so no
// workspace array exists.  A workgroup owns 16*MT signal rows and every workspace column:
// wave w multiplies block wblk[w] (-1: none) over n-tiles wnt0[w] .. wnt0[w] + wcnt[w] - 1.
//   desc[4 e .. 4 e + 3] (entry e = desc_off[b] + k, k < 32 nkc[b]): the first-pass value of
//     workspace column col[b] + k is  c1 * x1 + c0 * x0  (one multiply, one fused
//     multiply-add), x0 and x1 the input row's values at byte offsets word 0 and word 1,
//     c0 = word 2, c1 = word 3 (float bits): a sum x_i + x_j (1, 1), a difference x_i - x_j
//     (1, -1), sqrt(2) x_c of a V_Z node (sqrt 2, 0), a copy (1, 0) or padding (0, 0); with
//     c1 = 0 the second offset repeats the first (c1 = 0 skips the add, c0 = 0 gives 0);
//   src_mode: how the inputs of a k step are loaded: 1, one set for both blocks (every valid
//     entry of the second block has the offsets of the first block's entry at the same k:
//     one left stage, sums and differences of the same Haar units; or one block); 3, one
//     load of two adjacent values per entry, at the first block's offset (both blocks copy
//     and their sources are neighbours: the inverse of one-stage plans whose two blocks'
//     coefficients alternate), the first value to block pair_swap, the second to the other;
//     4, one set per block of one value per entry (every entry a copy or a sqrt 2 scaling:
//     the first pass has no stage, as in the inverse); 5, as 1, with each lane's two
//     entries 2m, 2m + 1 read as two pairs: the first sources at word 0 of entry 2m and the
//     next position (entry 2m + 1's), the second sources at word 1 of entry 2m + 1 and the
//     next position (entry 2m's) — the units of a mirror involution in rank order — and a
//     last pass without stages that gathers no workspace column twice, whose results are
//     written to the slab at their output columns (omap3[w]: output column of workspace
//     column w, -1: none; the other columns hold zeros) and leave as they are; 2, one set
//     per block;
//   frag: the block matrices in MFMA B-operand order, 16 bytes per lane per fragment, per
//     (kc, nt) at index frag_off[b] + kc * ntl[b] + nt: BF16 blocks, one 16x16x32 fragment
//     (column 16 nt + lane % 16, k = 32 kc + 8 (lane / 16) + e); split blocks, a hi and a lo
//     fragment of that shape; FP32 blocks, two halves h = 0, 1 of four 16x16x4 k groups
//     (k = 32 kc + 16 h + 4 (lane / 16) + e, e < 4: the k order of the three-pass FP32 GEMM);
//     the rounding is the same as the three-pass GEMM's;
//   the last pass: num_stages3 stages (stages3: offset, count pairs; ops3: i | j << 16,
//     j = 0xffff: scale by sqrt 2) on workspace columns, 16 rows at a time, then output
//     column c takes slab column gather3[c] (-1: zero); ops3 and gather3 are read from LDS
//     copies, so that the last pass issues no global loads (their waits would also wait for
//     the output stores before them).
struct OnePass {
  int32_t n;              // input and output row length
  int32_t ldw;            // workspace columns
  int32_t slab_stride;    // LDS row stride of the result slab (floats)
  int32_t nblocks;        // 1 or 2
  int32_t nk;             // k steps of 32 (the longest block)
  int32_t src_mode;
  int32_t pair_swap;      // src_mode 3: 1 when the second block's source comes first
  int32_t num_stages3;
  int32_t desc_words;     // int32 words of desc (copied to LDS)
  int32_t ops3_words;     // entries of ops3 (copied to LDS, with gather3)
  int32_t K[2], col[2], nkc[2], ntl[2], desc_off[2], frag_off[2];
  int32_t wblk[8], wnt0[8], wcnt[8];
  const int32_t *desc;
  const uint32_t *frag;
  const int32_t *gather3;
  const int32_t *stages3;
  const uint32_t *ops3;
  const int32_t *omap3;   // ldw entries (source mode 5)
};

}  // namespace gft
