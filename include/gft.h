/*
 * gft.h -- C ABI of the MI355X fast graph Fourier transform library (libgft.so).
 *
 * What it computes (Lu & Ortega, "Fast Graph Fourier Transforms Based on Graph Symmetry
 * and Bipartition"):
 *   - The GFT of a graph signal x in R^n is c = U^T x, where L = U diag(lambda) U^T is the
 *     eigendecomposition of the Laplacian L = D - W + S (Sec. II-B, eqs. def_laplacian and
 *     l_from_sw), with the basis ordered by increasing eigenvalue (graph frequency).
 *   - A plan factors U as a product of butterfly stages of Haar units (eq. B_phi, one
 *     stage per node pairing phi, Sec. IV-B) and a block-diagonal set of small dense
 *     sub-GFTs, the eigenbases of the leaf sub-graphs reached by the recursive
 *     decomposition G -> (G+, G-) of Thm. decompose (Sec. IV-C).  Leaf sub-graphs are
 *     further split into connected components (the G- of Fig. Gsk).
 *   - gft_forward applies U^T to a batch of signals; gft_inverse applies U (the inverse
 *     and the adjoint, since U is orthogonal and every B_phi is its own inverse, Sec. III).
 *
 * Conventions.
 *   - Signals are signal-major: a batch of S signals is an S x n row-major array, the n
 *     node values of one signal contiguous in node-label order.  Coefficients use the
 *     same layout, in the plan's output order (ascending eigenvalue by default).
 *   - Node labels are 0-based.
 *   - Every function returns a gft_status.  No C++ exception crosses this boundary.  On
 *     error, gft_last_error() returns a thread-local message naming the argument, stage
 *     or node at fault.
 *   - Host arrays passed in (graph, pairing, options) are borrowed for the call only; the
 *     plan copies what it needs.  Device buffers (x, y) are owned by the caller.
 *   - Streams are passed as void* and are hipStream_t values (NULL = the null stream).
 *     Launches are asynchronous and stream-ordered; a device fault surfaces at the
 *     caller's next synchronisation, not as a return code of the launching call.
 */
#ifndef GFT_H_
#define GFT_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GFT_OK = 0,
  GFT_ERR_INVALID_ARG = 1,              /* NULL pointer, negative size, bad option value   */
  GFT_ERR_GRAPH = 2,                    /* bad edge list: label out of range, i == j,      */
                                        /* duplicate edge, non-finite weight or self-loop  */
  GFT_ERR_NOT_INVOLUTION = 3,           /* phi(phi(i)) != i or phi(i) out of range         */
  GFT_ERR_PAIRING_CROSSES_SUBGRAPH = 4, /* phi maps a node of one current sub-graph into   */
                                        /* another (stages act inside G+ and G-)           */
  GFT_ERR_NOT_SYMMETRIC = 5,            /* a current sub-graph is not phi-symmetric        */
  GFT_ERR_EIGENSOLVE = 6,               /* leaf eigensolver did not converge               */
  GFT_ERR_ORTHOGONALITY = 7,            /* plan-time check ||V^T V - I|| or residual failed*/
  GFT_ERR_ALIGNMENT = 8,                /* device pointer not 16-byte aligned, or x and y  */
                                        /* overlap without being equal                     */
  GFT_ERR_UNSUPPORTED = 9,              /* shape or precision the library does not run     */
  GFT_ERR_OOM = 10,                     /* host or device allocation failed                */
  GFT_ERR_HIP = 11                      /* a HIP runtime call failed                       */
} gft_status;

/* Opaque plan.  Immutable after creation except for a per-device cache of its device
 * image, filled on first use on each device (thread safe). */
typedef struct gft_plan_s *gft_plan_t;

/* Undirected weighted graph G(V, E, W) with self-loops s_i = w_ii (Sec. II-B).
 * Each edge {src[e], dst[e]} (src != dst) is listed once with a finite real weight.
 * self_loop is an array of n finite reals, or NULL for no self-loops.  Weights need not
 * be positive: sub-graphs of the decomposition carry negative weights (Sec. IV-C). */
typedef struct {
  int32_t n;
  int32_t num_edges;
  const int32_t *src;
  const int32_t *dst;
  const double *weight;
  const double *self_loop;
} gft_graph;

/* Node pairings, one involution per butterfly stage (Definition 1 and eq. p_phi;
 * recursion of Sec. IV-C).  phi[s*n + i] is the partner of node i at stage s, i for a
 * fixed node.  Stage s acts on each current sub-graph separately: it must map each
 * sub-graph's node set onto itself, and each sub-graph it moves must be phi-symmetric
 * (Definition 2).  A sub-graph left fixed by phi is not split at that stage.
 * Of each pair, the smaller label joins V_X and its partner V_Y (eq. B_phi). */
typedef struct {
  int32_t num_stages;
  const int32_t *phi;
} gft_pairing;

/* Arithmetic of the dense leaf blocks.  Haar stages always run in FP32. */
typedef enum {
  GFT_FP32 = 0,        /* FP32 products, FP32 accumulation (MFMA 16x16x4 f32)         */
  GFT_BF16 = 1,        /* BF16 operands, FP32 accumulation                            */
  GFT_FP16 = 2,        /* FP16 operands, FP32 accumulation                            */
  GFT_SPLIT_BF16 = 3   /* hi+lo BF16 split, three products, FP32 accumulation         */
} gft_precision;

/* Storage type of signals or coefficients in device memory.  The arithmetic does not
 * change: BF16 values are widened to FP32 when loaded and rounded to the nearest BF16
 * (ties to even) when stored. */
typedef enum {
  GFT_DTYPE_FP32 = 0,
  GFT_DTYPE_BF16 = 1
} gft_dtype;

/* Which Laplacian the GFT diagonalises (Sec. II-B). */
typedef enum {
  GFT_LAPLACIAN_COMBINATORIAL = 0,  /* L = D - W + S (eq. l_from_sw)                        */
  GFT_LAPLACIAN_NORMALIZED = 1      /* D^{-1/2} L D^{-1/2}, d_i = sum_{j != i} w_ij; every  */
                                    /* node needs d_i > 0 (else GFT_ERR_GRAPH).  The left   */
                                    /* Haar decomposition holds for it as well (Sec. IV-B) */
} gft_laplacian;

/* Right (bipartite) Haar stages (Sec. III, eq. right_gft, Thm. right_haar): a leaf
 * sub-graph (connected component) whose Laplacian has a constant diagonal c and whose
 * edges join two parts S1, S2 (a k-regular bipartite graph, or any bipartite graph under
 * the normalized Laplacian) is applied as two blocks E (on S1) and F (on S2) followed by
 * right Haar units: eigenvectors (u1; u2) at c - s and (u1; -u2) at c + s (Lemma k-rbg)
 * share E's column sqrt2 u1 and F's column sqrt2 u2.  Cost |S1|^2 + |S2|^2 instead of
 * (|S1| + |S2|)^2 multiplications. */
typedef enum {
  GFT_RIGHT_HAAR_AUTO = 0,   /* use them on every leaf that qualifies                  */
  GFT_RIGHT_HAAR_OFF = 1     /* dense leaf blocks only                                 */
} gft_right_haar;

typedef enum {
  GFT_ORDER_EIGENVALUE = 0,  /* ascending eigenvalue; ties by leaf-block order, then  */
                             /* local index (any basis of an eigenspace is a GFT)     */
  GFT_ORDER_BLOCK = 1        /* leaf-block order (depth first, G+ before G-), then    */
                             /* ascending eigenvalue inside each block                */
} gft_order;

/* Kernel family.  AUTO picks, for single-graph plans without right Haar units: the
 * register-butterfly engine when the plan is a uniform hypercube (every stage pairs every
 * node, 2^S equal connected leaf blocks, each Haar orbit holding one node of every block)
 * of a compiled shape with FP32 blocks, or a one-stage plan with 8 <= n <= 96 and sides of
 * at most 48 nodes (FP32 or BF16 blocks), or a two-stage plan whose orbits and leaf blocks
 * fit 16 or 32 slots per side (FP32 blocks); else the large-signal engine when a tile of 16
 * signals does not fit a workgroup's LDS or a leaf block has 192 nodes or more (the
 * product engine instead when every leaf block has a Kronecker basis, see num_kron_leaves,
 * with factors of at most 64 nodes, FP32 storage and FP32, BF16 or split BF16 blocks); else
 * the generic engine.  Batch plans run each graph that a register-butterfly form of the batch
 * kernel covers (one stage with sides of at most 48 nodes, two stages on 16- or 32-slot
 * sides, FP32 blocks; BF16 blocks: one stage) in its register phase and the others on their
 * generic-engine programs; GFT_ENGINE_GENERIC puts every graph on the latter. */
typedef enum {
  GFT_ENGINE_AUTO = 0,
  GFT_ENGINE_GENERIC = 1,     /* LDS-program engine (one fused kernel)                  */
  GFT_ENGINE_BUTTERFLY = 2,   /* register-butterfly engine (else GFT_ERR_UNSUPPORTED at  */
                              /* the first apply)                                       */
  GFT_ENGINE_LARGE = 3,       /* large-signal engine: Haar stages and permutations in    */
                              /* streaming passes, leaf blocks as MFMA GEMM tiles over a */
                              /* stream-ordered workspace (hipMallocAsync, freed in      */
                              /* stream order) of S*w floats (2*S*w when the last pass   */
                              /* has Haar stages or there are more than 8 leaf blocks),  */
                              /* w = n plus each leaf block padded to                    */
                              /* a multiple of 8 (the workspace stays FP32 or BF16 with  */
                              /* BF16 blocks whatever the storage); FP16 is unsupported  */
  GFT_ENGINE_PRODUCT = 4      /* separable engine: U_a^T X U_b per signal on MFMA.  The  */
                              /* engine of product-graph plans (gft_plan_product); as   */
                              /* options.engine it runs a gft_plan whose leaves have    */
                              /* Kronecker bases (else GFT_ERR_UNSUPPORTED at the first */
                              /* apply)                                                 */
} gft_engine;

typedef struct {
  int32_t precision;       /* gft_precision                                           */
  int32_t order;           /* gft_order                                               */
  int32_t tile_override;   /* 0 = autotuned at plan preparation (generic engine);     */
                           /* else signals per tile: 16, 32, 64 or 128                */
  int32_t engine;          /* gft_engine                                              */
  double sym_tol;          /* relative tolerance of the phi-symmetry test on sub-graph*/
                           /* Laplacians; <= 0 selects 1e-12                          */
  int32_t in_dtype;        /* gft_dtype of signals x: read by the forward, written by */
                           /* the inverse                                             */
  int32_t out_dtype;       /* gft_dtype of coefficients y: written by the forward,    */
                           /* read by the inverse.  BF16 storage runs on every engine:*/
                           /* any combination on the butterfly, generic and large     */
                           /* engines; product and batch plans store signals and      */
                           /* coefficients in one type (else GFT_ERR_UNSUPPORTED at   */
                           /* planning); in place needs equal types                   */
  int32_t laplacian;       /* gft_laplacian                                           */
  int32_t right_haar;      /* gft_right_haar                                          */
  int32_t autotune;        /* gft_autotune: launch choices timed at preparation (0,  */
                           /* the default) or the built-in ones (1); see             */
                           /* gft_plan_tuning                                         */
} gft_options;

typedef enum {
  GFT_AUTOTUNE_ON = 0,     /* time the candidates at preparation, or reuse the cache  */
  GFT_AUTOTUNE_OFF = 1     /* built-in launch choices                                 */
} gft_autotune;

/* Where a plan's launch choices on a device came from. */
typedef enum {
  GFT_TUNE_BUILTIN = 0,    /* built-in choices (autotune off, or nothing to choose)   */
  GFT_TUNE_TIMED = 1,      /* candidates timed at preparation on this device          */
  GFT_TUNE_CACHED = 2      /* taken from the tuning cache (same device kind, same     */
                           /* plan image): no timing                                  */
} gft_tune_source;

/* Launch choices of a plan on the current device (gft_plan_tuning).  None of them changes
 * the arithmetic of a signal: every choice gives bit-identical results. */
typedef struct {
  int32_t engine;          /* gft_engine the plan runs on                             */
  int32_t fwd_tile;        /* signals per tile: generic engine 16 * m (tuned), butterfly */
  int32_t inv_tile;        /* 16 (per wave), product 1 (per wave), large 0, batch 0    */
  int32_t grid_fwd;        /* butterfly and product engines, and the large engine's   */
  int32_t grid_inv;        /* one-pass form: most workgroups launched (tuned; the tile */
                           /* or panel loop strides over the rest; 0: one per tile or */
                           /* panel); else 0                                          */
  int32_t variant;         /* product: 1 staged factors, 0 dense; large: 2 one-pass   */
                           /* form, 1 forward output order written by the GEMM        */
                           /* epilogue, 0 three passes (tuned where several exist);   */
                           /* else 0                                                  */
  int32_t batch_rounds;    /* batch: rounds of resident workgroups (tuned)            */
  int32_t batch_cost16;    /* batch: register-phase fixed cost per signal in          */
                           /* sixteenths of the padded slot count (tuned)             */
  int32_t large_tile_kb;   /* large: stage-pass tile size in KB (tuned)               */
  int32_t source;          /* gft_tune_source                                         */
  double tune_ms;          /* host milliseconds spent timing candidates (0 if none)   */
  int32_t onepass_fwd;     /* large engine, one-pass form (where the plan fits it):   */
  int32_t onepass_inv;     /* how a k step's inputs are loaded, per direction: 1 one  */
                           /* set for both blocks, 2 one set per block, 3 pairs split */
                           /* between the blocks, 4 one value per entry and block, 5  */
                           /* pairs of neighbours, results at their output columns;  */
                           /* 0 without the form                                      */
} gft_tuning;

typedef struct {
  int32_t n;
  int32_t num_stages;      /* stages given                                            */
  int32_t num_units;       /* Haar units over all stages, left and right              */
  int32_t num_blocks;      /* dense leaf blocks                                       */
  int32_t max_block;       /* largest leaf block                                      */
  int32_t num_z_scalings;  /* sum over stages of |V_Z| in the sub-graphs split        */
  int64_t adds;            /* 2 * units + sum_b b(b-1)           (Table tab:runtime)  */
  int64_t mults;           /* sum_b b^2 + num_z_scalings          (Table tab:runtime)  */
  double max_residual;     /* max over blocks of ||L_b V_b - V_b Lambda_b||_F/||L_b||_F*/
  double max_orth_error;   /* max over blocks of ||V_b^T V_b - I||_max                */
  int32_t num_right_units; /* right Haar units (included in num_units and adds)       */
  int32_t num_right_leaves;/* leaf components applied with right Haar units           */
  int32_t num_kron_leaves; /* leaf blocks with Kronecker bases V_a (x) V_b: the graph is */
                           /* a row-major Cartesian product whose stages act along one  */
                           /* axis each (Sec. V-D); 0 or num_blocks                     */
  int64_t separable_mults; /* mults with those leaves applied separably, V_a^T Z V_b:   */
                           /* sum b_a b_b (b_a + b_b) + num_z_scalings (else = mults)   */
  int32_t num_closed_form_leaves; /* leaves whose basis is the closed form DCT-II (a    */
                           /* uniform path plus c I) or DST-IV (the same with a self-   */
                           /* loop 2w at one end), not an eigensolve (Sec. V-C)         */
} gft_plan_stats;

/* Build a plan for one graph.  Validates the graph and every stage, forms the sub-graph
 * Laplacians of Thm. decompose (eqs. blkdiag_G and Lpm), splits leaves into connected
 * components, solves each leaf block's eigenproblem in FP64, checks orthogonality and
 * residual, and orders the output.  opts may be NULL (FP32, eigenvalue order).
 * Host-only: touches no GPU.  On success *out owns the plan (free with
 * gft_plan_destroy). */
gft_status gft_plan(const gft_graph *graph, const gft_pairing *pairing,
                    const gft_options *opts, gft_plan_t *out);

/* Search node pairings for the left Haar stages (Sec. V-F, pruning based on the degree
 * list), stage by stage: stage s is an involution that acts inside each sub-graph produced
 * by the stages before it (as gft_plan splits them) and keeps each such sub-graph
 * phi-symmetric (Definition 2), chosen to have the most node pairs (fewest multiplications,
 * p^2 + (n - p)^2).  A node is only paired with nodes of equal diagonal and equal sorted
 * list of edge weights; a depth-first search, most constrained nodes first, checks
 * l_ij = l_phi(i)phi(j) as it assigns and stops at a perfect pairing or after max_steps
 * steps per sub-graph (<= 0: 200000), keeping the best found.  The search stops when no
 * sub-graph has a non-trivial symmetry or max_stages is reached.
 * graph: host, as for gft_plan; opts: its laplacian and sym_tol are used (NULL = defaults).
 * phi: host array of max_stages * n int32 written with the stages found (phi[s*n + i]),
 * the gft_pairing input of gft_plan.  *num_stages receives their number (0: none). */
gft_status gft_find_pairing(const gft_graph *graph, const gft_options *opts, int32_t max_stages,
                            int64_t max_steps, int32_t *phi, int32_t *num_stages);

/* Build one plan covering num_graphs graphs (arrays of num_graphs graphs and pairings)
 * for gft_forward_batch / gft_inverse_batch.  Each graph is planned as by gft_plan. */
gft_status gft_plan_batch(int32_t num_graphs, const gft_graph *graphs,
                          const gft_pairing *pairings, const gft_options *opts,
                          gft_plan_t *out);

/* Build a plan for the Cartesian product G_a x G_b of two graphs (node (i, j) has label
 * i * n_b + j; edges (i, j)-(i', j) of weight w_a(i, i') and (i, j)-(i, j') of weight
 * w_b(j, j'); self-loop s_a(i) + s_b(j)).  Its Laplacian is L_a (x) I + I (x) L_b, so the
 * Kronecker product U_a (x) U_b of the factor GFTs is a GFT of the product (eigenvalue
 * lambda_p + mu_q for basis vector (p, q)): the separable form of the grid GFTs of
 * Sec. V-D, whose axis-wise stages leave leaf blocks that are Kronecker products of the
 * axes' leaves.  Each factor is planned as by gft_plan (its stages, if any, shape its
 * basis); the transform runs as y = U_a^T X U_b per signal X (n_a x n_b, row-major) on MFMA
 * (options.precision: FP32, BF16 or split BF16 products with FP32 accumulation), then the
 * coefficients in output order (ascending lambda_p + mu_q, ties by p then q;
 * GFT_ORDER_BLOCK: p * n_b + q).  The factors run as dense matrices, or in their fast
 * form where it is compiled: two 64-node factors whose stages are the halving reversals
 * (stage t pairs i < R/2 with R - 1 - i, R = 64 >> t) with FP32 products run the stages as
 * add/sub on the signal and the leaf blocks (32, 16, 8, 4, 2, 1, 1 nodes) as block-diagonal
 * matrices, skipping their zero 16x16 tiles (3/8 of the dense MFMA work).  The environment
 * variable GFT_PRODUCT_FORM=dense or staged forces either form where both exist.
 * Requires n_a, n_b <= 64, one storage type for signals and coefficients, and
 * options.engine 0 (else GFT_ERR_UNSUPPORTED; FP16 precision is unsupported too).  The
 * normalized Laplacian (Sec. II-B) is accepted when both factors are regular (constant
 * weighted degree d_a, d_b): the product's is then L / (d_a + d_b), the same basis with the
 * eigenvalues scaled; otherwise it is no Kronecker sum (GFT_ERR_UNSUPPORTED).  gft_plan_info reports the two factor GFTs
 * as num_blocks = 2 with their dense costs; gft_plan_blocks is unsupported.  Host-only. */
gft_status gft_plan_product(const gft_graph *graph_a, const gft_pairing *pairing_a,
                            const gft_graph *graph_b, const gft_pairing *pairing_b,
                            const gft_options *opts, gft_plan_t *out);

/* y = U^T x for num_signals signals (coefficients; Sec. II-B).
 * x: device, num_signals x n values of options.in_dtype (FP32 unless set), 16-byte
 * aligned.  y: device, num_signals x n values of options.out_dtype, 16-byte aligned;
 * y == x (in place) is allowed when the two types are equal, other overlaps are rejected.
 * num_signals == 0 is a no-op.  Single-graph plans only.  The large-signal engine's
 * three-pass and GEMM-epilogue forms (gft_plan_tuning variant 0 or 1) take a workspace from
 * the stream-ordered pool per call and return GFT_ERR_UNSUPPORTED on a stream under capture
 * (gft_apply_noalloc serves such callers); its one-pass form (variant 2) and every other
 * engine allocate nothing per call. */
gft_status gft_forward(gft_plan_t plan, const void *x, void *y, int64_t num_signals,
                       void *stream);

/* x = U y (inverse and adjoint of gft_forward).  Same layout and rules. */
gft_status gft_inverse(gft_plan_t plan, const void *y, void *x, int64_t num_signals,
                       void *stream);

/* Allocation-free apply, for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  direction 0 runs
 * gft_forward, 1 gft_inverse, with the same arguments, layout, kernels and results (bit
 * for bit).  It calls no hipMalloc, hipFree or allocating routine: the plan must already
 * have an image on the current device (gft_plan_prepare there, which allocates; else
 * GFT_ERR_INVALID_ARG), and the large-signal engine takes its workspace from a static
 * array of 64 MiB per GPU held by the library until the process ends (each call needs
 * num_signals * w * 4 bytes, twice that when its output order is not fused, w = n plus
 * each leaf block padded to 8; larger calls are rejected with GFT_ERR_INVALID_ARG and the
 * largest signal count in gft_last_error).  Every call on a GPU shares that GPU's array:
 * calls that overlap in time on one GPU (different streams or threads) race on it and must
 * be serialised by the caller; the other engines use no workspace.  Batch plans are
 * rejected (gft_forward_batch allocates nothing once the plan is prepared). */
gft_status gft_apply_noalloc(gft_plan_t plan, int32_t direction, const void *in, void *out,
                             int64_t num_signals, void *stream);

/* Mixed batch in one persistent launch.  signal_offsets: device int64 array of
 * num_graphs+1 non-decreasing entries, graph g owning signals [off[g], off[g+1]).
 * Graph g's data starts at element sum_{h<g} (off[h+1]-off[h]) * n_h of x (and of y):
 * the graphs' [S_g x n_g] arrays are packed back to back.  total_elements bounds that
 * sum (the caller's buffer length in elements); the kernel never touches more.  The
 * offsets are read on the device, so the call does not synchronise. */
gft_status gft_forward_batch(gft_plan_t plan, const void *x, void *y,
                             const int64_t *signal_offsets, int64_t total_elements,
                             void *stream);
gft_status gft_inverse_batch(gft_plan_t plan, const void *y, void *x,
                             const int64_t *signal_offsets, int64_t total_elements,
                             void *stream);

/* Upload the plan's device image to the current device now (otherwise done on the first
 * apply on each device, with a synchronous copy).  Call it before capturing an apply into
 * a hipGraph.  Needs a GPU. */
gft_status gft_plan_prepare(gft_plan_t plan);

/* Engine (gft_engine: GFT_ENGINE_GENERIC, GFT_ENGINE_BUTTERFLY, GFT_ENGINE_LARGE or
 * GFT_ENGINE_PRODUCT) the
 * plan's image on the current device runs; builds the image like gft_plan_prepare.
 * Needs a GPU. */
gft_status gft_plan_engine(gft_plan_t plan, int32_t *engine_out);

/* Signals per tile of the forward and inverse kernels on the current device (single-graph
 * plans; builds the image like gft_plan_prepare): the generic engine's tile height, which
 * options.tile_override fixes or, when it is 0, the plan-time autotuner picks by timing
 * every height that fits in LDS on a synthetic batch (same results for every height);
 * 16 for the butterfly engine (per wave); 0 for the large-signal engine; 1 for product
 * plans (one signal per wave).  Needs a GPU. */
gft_status gft_plan_tiles(gft_plan_t plan, int32_t *fwd_tile, int32_t *inv_tile);

/* Launch choices of the plan on the current device (builds the image like
 * gft_plan_prepare).  With options.autotune = GFT_AUTOTUNE_ON preparation times the
 * candidates of the plan's engine on a synthetic batch (generic: every tile height that
 * fits in LDS; butterfly and product: grids of 1/2, 3/4, 1 and 2 times the resident
 * workgroups; batch: 1 to 4 rounds of resident workgroups x register-phase cost 8, 11 or
 * 14 sixteenths; large: fused or three-pass output order x stage-pass tiles of 20, 40 or
 * 80 KB, and the one-pass form with the resident workgroups or, where the timed batch holds
 * more panels than that, one workgroup per panel) and keeps the fastest (3% better than
 * the built-in choice at least), unless the
 * tuning cache holds a choice for the same device kind and plan image.  The cache lives in
 * memory and in the text file named by the environment variable GFT_TUNE_CACHE (default
 * $HOME/.cache/libgft/tuning-v2.txt; empty or "off": memory only).  Needs a GPU. */
gft_status gft_plan_tuning(gft_plan_t plan, gft_tuning *out);

/* Statistics of graph `index` of a plan (0 for single-graph plans). */
gft_status gft_plan_info(gft_plan_t plan, int32_t index, gft_plan_stats *out);

/* Number of graphs in the plan, and n of graph `index`. */
gft_status gft_plan_num_graphs(gft_plan_t plan, int32_t *out);
gft_status gft_plan_size(gft_plan_t plan, int32_t index, int32_t *n_out);

/* Eigenvalues (n doubles, host) of graph `index` in output order. */
gft_status gft_plan_eigenvalues(gft_plan_t plan, int32_t index, double *lambda);

/* FP64 fast basis of graph `index` (n*n doubles, host, row-major): U[i*n + k] is node i
 * of basis vector k, k in output order.  Computed on the host by running the plan's
 * factorisation (stages and blocks) in FP64 on unit vectors. */
gft_status gft_plan_basis(gft_plan_t plan, int32_t index, double *U);

/* Apply the plan's factorisation in FP64 on the host (reference path of the plan's own
 * algebra; no GPU).  x, y: host, num_signals x n doubles.  direction 0 = forward,
 * 1 = inverse. */
gft_status gft_plan_apply_host(gft_plan_t plan, int32_t index, int32_t direction,
                               const double *x, double *y, int64_t num_signals);

/* Leaf-block description of graph `index`: sizes[b] for b < num_blocks (num_blocks
 * from gft_plan_info).  nodes, if not NULL, receives the n node labels grouped by block
 * (block b's nodes contiguous, in block order). */
gft_status gft_plan_blocks(gft_plan_t plan, int32_t index, int32_t *sizes, int32_t *nodes);

gft_status gft_plan_destroy(gft_plan_t plan);

/* Thread-local detail string of the last error on this thread ("" if none). */
const char *gft_last_error(void);

/* Library version string. */
const char *gft_version(void);

/* Streaming copy of `bytes` bytes from src to dst on `stream` (a hipStream_t; NULL = the
 * null stream), stream-ordered and asynchronous.  Not an operation of the transform: the
 * reference kernel for what moving data through HBM alone reaches on this device
 * (non-temporal 16-byte loads and stores, as the transform kernels use for signal data),
 * quoted beside the GFT kernels' HBM rooflines.  src, dst: device memory, 16-byte aligned,
 * not overlapping, owned by the caller; bytes a multiple of 16 (0 is a no-op).  Errors:
 * GFT_ERR_INVALID_ARG (size, NULL), GFT_ERR_ALIGNMENT (alignment, overlap), GFT_ERR_HIP
 * (launch). */
gft_status gft_stream_copy(const void *src, void *dst, int64_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GFT_H_ */
