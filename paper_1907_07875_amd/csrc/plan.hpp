// Host-side plan of the fast GFT: stages of Haar units and dense leaf blocks.
//
// A GraphPlan is the factorisation U = B_{phi_1} ... B_{phi_k} * P * diag(V_b) * Pi of the
// paper (eq. left_gft applied recursively, Sec. IV-C), stored as
//   - stages: for each pairing, the Haar units (i in V_X, j = phi(i) in V_Y) and the
//     fixed nodes V_Z of every sub-graph the stage splits;
//   - blocks: the connected components of the leaf sub-graphs, each with its node list,
//     eigenvalues and FP64 eigenvectors V_b, and its depth (number of splits above it);
//   - out_pos: the output position (coefficient index) of each block eigenvector.
// Kernels run the stages unscaled (x_i + x_j, x_i - x_j, and sqrt(2) x_c on V_Z), which is
// sqrt(2) B_phi on every split sub-graph; the 2^(-depth/2) factor is folded into the
// block matrices.  This is the normalisation-absorption of Sec. III (Fig. haar).
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/gft.h"

namespace gft {

struct PlanError {
  gft_status status;
  std::string message;
};

struct HostStage {
  std::vector<int32_t> pair_x;  // V_X member of each Haar unit
  std::vector<int32_t> pair_y;  // its partner phi(x) in V_Y
  std::vector<int32_t> znodes;  // fixed nodes of the sub-graphs split at this stage
};

struct HostBlock {
  int32_t size = 0;
  int32_t depth = 0;
  double scale = 1.0;               // 2^(-depth/2)
  std::vector<int32_t> nodes;       // node labels, ascending
  std::vector<double> lambda;       // eigenvalue of column k (ascending for dense blocks)
  std::vector<double> V;            // size*size, V[j*size + k]
  std::vector<int32_t> out_pos;     // output position of eigenvector k
};

struct GraphPlan;

// Leaf blocks that are Kronecker products.  The Laplacian of a Cartesian product G_a x G_b
// (node (i, j) labelled i * nb + j) is L_a (x) I + I (x) L_b, and a stage that acts along
// one axis, phi((i, j)) = (phi_a(i), j) or (i, phi_b(j)), splits it into sub-graphs that
// are again products (Sec. V-D: grids decompose axis by axis).  So every leaf block is a
// product B_a x B_b of leaf blocks of the two factor plans (their stages being the stages
// along each axis, in order), and V_a (x) V_b is an eigenbasis of it (eigenvalue
// lambda + mu) and U_a (x) U_b the plan's whole basis: the leaves are separable and the
// transform is U_a^T X U_b per signal X (na x nb).
struct KronPlan {
  int32_t na = 0, nb = 0;
  std::shared_ptr<const GraphPlan> fa, fb;   // factor plans (eigenvalue output order)
  std::vector<int32_t> order;                // coefficient k is factor pair (order[k] / nb, order[k] % nb)
  int64_t separable_mults = 0;               // sum over leaves of b_a b_b (b_a + b_b)
};

struct GraphPlan {
  int32_t n = 0;
  int32_t num_stages_given = 0;
  std::vector<HostStage> stages;    // stages that split something (others dropped)
  // Right Haar units (Sec. III, eq. right_gft) after the blocks, on output positions:
  // forward y[pair_x] = a + b, y[pair_y] = a - b with a, b the two blocks' outputs there
  // (the 1/sqrt 2 is folded into those block columns).  znodes unused.
  HostStage right;
  std::vector<HostBlock> blocks;
  std::vector<double> lambda_out;   // eigenvalues in output order
  gft_plan_stats stats{};
  std::shared_ptr<const KronPlan> kron;   // set when every leaf block is a Kronecker product
};

// Search up to max_stages pairings stage by stage (each stage searched inside every current
// sub-graph, as the plan splits them); returns the number found, phi_out = stages * n.
// `budget` caps the search steps per sub-graph.  Throws PlanError on a bad graph.
int find_pairing(const gft_graph &g, const gft_options &opts, int max_stages, int64_t budget,
                 std::vector<int32_t> &phi_out);

// Build the plan of one graph.  Throws PlanError.  recognize_products: look for the
// row-major Cartesian product structure above (factors of 2 to 64 nodes) and, when found,
// give the leaf blocks their Kronecker bases.
GraphPlan build_graph_plan(const gft_graph &g, const gft_pairing *pairing,
                           const gft_options &opts, bool recognize_products = true);

// FP64 host application of the factorisation (direction 0 forward, 1 inverse).
void apply_host(const GraphPlan &p, int direction, const double *x, double *y, int64_t S);

}  // namespace gft
