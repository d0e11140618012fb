// Separable GFT of Cartesian product graphs (gfx950).
//
// The Laplacian of G_a x G_b is L_a (x) I + I (x) L_b, so U_a (x) U_b is a GFT of the product
// graph (eigenvalue lambda_p + mu_q for basis vector (p, q)): the fast GFT of a grid whose
// stages act along one axis at a time (Sec. V-D) has leaf blocks that are Kronecker
// products of the axes' leaf blocks, and applying it axis by axis replaces the 2-D leaf
// products by two 1-D transforms.  Per signal X (na x nb, row-major) the kernel computes
// U_a^T X U_b as two MFMA products on a wave-private LDS tile:
//   HBM --16B loads--> registers --> LDS tile (row stride NB + 1: odd, so the 16 rows an
//   MFMA operand spans fall in distinct banks)
//   --> Y1 = Z * B into MFMA result registers
//   --> Y2 = A * Y1 straight from those registers (the contraction order over k follows
//   the result layout), one 16-column block at a time, written into the tile
//   --> LDS words in output order (perm) --> 16B stores.
// Both matrices stay in registers as MFMA fragments (v_mfma_f32_16x16x4_f32: lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; the result D[4 (l / 16) + v][l % 16]).  Padding
// rows and columns of the tile and of the matrices are zero, so they stay zero.
// Staged factors: a factor with Haar stages is applied in its fast form, the stages as
// add/sub on the tile (rows for axis a, columns for axis b; before the products forward,
// after them inverse) and its leaf blocks as one block-diagonal matrix whose all-zero
// 16x16 tiles the products skip (a compiled tile pattern): the 64 x 64 grid's halving
// stages leave blocks of 32, 16, 8, 4, 2, 1, 1 per axis, 6 of 16 tiles.
#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "product_core.hpp"

namespace gft {

int product_pad(int n) { return product_pad_size(n); }

hipError_t launch_product(const PProgram &P, const float *in, float *out, int64_t nsig,
                          hipStream_t stream, int num_cus, int grid_cap) {
  if (P.tile_pattern == 2) return launch_product_io16(P, in, out, nsig, stream, num_cus, grid_cap);
  return dispatch_product<false>(P, in, out, nsig, stream, num_cus, grid_cap, nullptr);
}

int product_occupancy(const PProgram &P) {
  if (P.tile_pattern == 2) return product_occupancy_io16(P);
  int occ = 1;
  if (dispatch_product<false>(P, nullptr, nullptr, 0, nullptr, -1, 0, &occ) != hipSuccess) return 1;
  return occ;
}

}  // namespace gft
