// Host construction of the device programs of a plan (see device_program.hpp).
#pragma once

#include <cstdint>
#include <vector>

#include "device_program.hpp"
#include "plan.hpp"

namespace gft {

// Host-side image of one program before upload: the LDS table and the matrix fragments.
struct ProgramImage {
  DevProgram prog{};          // pointers left null until upload
  std::vector<int32_t> table;
  std::vector<uint32_t> frag; // 32-bit words (FP32 values or packed 16-bit pairs)
};

// Largest LDS bytes a workgroup of the apply kernel may use.
constexpr size_t kMaxLdsBytes = 160 * 1024;

// Build the program of graph plan `p` for direction 0 (forward) or 1 (inverse).  The tile
// size (16*mt signals) is `tile_override`/16 if nonzero, else the largest of 8,4,2,1
// M-tiles whose LDS footprint fits `lds_budget` bytes.  Returns false if even one M-tile
// does not fit.
bool build_program(const GraphPlan &p, int direction, int tile_override, size_t lds_budget,
                   ProgramImage &out, int precision = GFT_FP32);

// Round-to-nearest-even conversions used for the 16-bit block fragments.
uint16_t to_bf16_bits(float x);
uint16_t to_f16_bits(float x);

size_t program_lds_bytes(const DevProgram &P);

// Host image of a register-butterfly program (see UProgram).
struct UProgramImage {
  UProgram prog{};
  std::vector<int32_t> gcol, scol;
  std::vector<uint32_t> flips;
  std::vector<float> afrag;
};

// Build the register-butterfly program of `p` if the plan is a uniform hypercube (or, failing
// that, a one-stage plan with 8 <= n <= 64 whose sides have at most 32 nodes, laid out on
// padded slots: UProgram::gen): every
// stage pairs every node (no V_Z), 2^S leaf blocks of equal size M (a multiple of 16),
// and each Haar orbit can be laid out on 2^S register slots so that every stage-t pair
// differs only in slot bit S-1-t (a 2-colouring per stage; orientation is fixed by a
// per-orbit sign flip).  The leaf block of a node is its slot after the last stage.
// Returns false (out untouched) otherwise.
// `precision`: GFT_FP32 (every shape above) or GFT_BF16 (one-stage programs only).
bool build_butterfly(const GraphPlan &p, int direction, UProgramImage &out, int precision = 0);

// Host image of the large-signal engine for one direction (see PermPass, LBlock).
struct LargeImage {
  int32_t n = 0, ldw = 0;
  PermPass pass[2]{};          // pointers left null until upload
  std::vector<int32_t> gather[2], stages[2];
  std::vector<uint32_t> ops[2];
  std::vector<LBlock> blocks;
  std::vector<int32_t> block_sizes;
  std::vector<float> mats;
  std::vector<uint16_t> mats16;         // the same matrices rounded to BF16 (RNE)
  std::vector<int32_t> omap;            // final position of every block output
  const LBlock *dev_blocks = nullptr;   // device copies, set at upload
  const float *dev_mats = nullptr;
  const uint16_t *dev_mats16 = nullptr;
  const int32_t *dev_omap = nullptr;
};

// Widest tile row (input columns or workspace columns) of the large-signal engine: each
// stage pass stages at least one whole FP32 row in LDS (160 KB), and op indices are 16-bit.
constexpr int kLargeMaxCols = (int)(kMaxLdsBytes / 4);

// Workspace columns of the large-signal engine for plan `p`: every leaf block's span
// padded to a multiple of 8.
int64_t large_workspace_cols(const GraphPlan &p);

// Build the large-signal engine image of `p` for direction 0 (forward) or 1 (inverse).
// Returns false when the input row or the workspace row would exceed kLargeMaxCols.
bool build_large(const GraphPlan &p, int direction, LargeImage &out);

// Host image of the one-pass form (see OnePass) for one direction.
struct OnePassImage {
  OnePass P{};                   // pointers left null until upload
  int mt = 4;                    // 16-signal row tiles per workgroup
  std::vector<int32_t> desc;
  std::vector<uint32_t> frag;
  std::vector<int32_t> omap;     // OnePass::omap3 (source mode 5)
};

// Table limits of the one-pass kernel (its LDS arrays are sized for them): entries of the
// two blocks' k steps, and k steps.
constexpr int kOnePassMaxEntries = 1088;
constexpr int kOnePassMaxSteps = 32;
constexpr int kOnePassMaxOps3 = 2048;   // last-pass Haar operations (all its stages)
constexpr int kOnePassMaxN = 1024;      // row length (the output gather table)

// The one-pass form of large image `L` (built for `precision`: GFT_FP32, GFT_BF16 or GFT_SPLIT_BF16,
// with L's host matrices still present; in16: the direction's input rows hold BF16).
// Returns false when the plan does not fit it: a first pass with more than one stage, more
// than two leaf blocks, or more columns than eight waves hold.  general: the general source
// modes only (1 with one block, 2 with two: each entry's two sources loaded as they are),
// for testing the specialised modes against them.
bool build_onepass(const LargeImage &L, int precision, bool in16, OnePassImage &out, bool general = false);

}  // namespace gft
