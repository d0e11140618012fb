// C ABI of libgft (include/gft.h): argument checking, plan ownership, per-device images.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <functional>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/gft.h"
#include "launch.hpp"
#include "plan.hpp"
#include "program.hpp"
#include "tune.hpp"

using namespace gft;

namespace {

thread_local std::string g_last_error;

gft_status set_error(gft_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

gft_status ok() {
  g_last_error.clear();
  return GFT_OK;
}

// Device image of a plan on one GPU: one allocation holding every program's table and
// fragments, and the programs with their device pointers filled in.
struct DeviceImage {
  int device = -1;
  int num_cus = 1;
  void *mem = nullptr;
  void *mem2 = nullptr;
  std::vector<DevProgram> fwd, inv;
  std::vector<int> grid_cap_fwd, grid_cap_inv;
  // register-butterfly programs (single-graph plans whose shape qualifies)
  bool butterfly = false;
  UProgram bfwd{}, binv{};
  // large-signal engine (single-graph plans)
  bool large = false;
  LargeImage lg[2];
  // product-graph plans: the two factor matrices and the output permutation per direction
  // (staged: the factors' stages and block-diagonal leaf matrices)
  bool product = false, product_staged = false;
  PProgram pfwd{}, pinv{};
  // batch plans: device arrays of the G forward and G inverse programs, and of their
  // register-butterfly programs (S = 0 where a graph runs its LDS program; null if none)
  const DevProgram *dev_fwd = nullptr, *dev_inv = nullptr;
  const UProgram *dev_ufwd = nullptr, *dev_uinv = nullptr;
  size_t batch_lds = 0;
  int batch_occ = 1;       // resident batch workgroups per CU
  int reg_groups = 0;
  // Launch choices (gft_plan_tuning): built-in values, replaced at preparation by the
  // fastest candidates on this device or by the tuning cache's choice for this image.
  std::string key;                     // tuning-cache key: device kind, engine, image hash
  int grid[2] = {0, 0};                // butterfly / product: most workgroups (0: resident)
  int batch_rounds = 2;                // batch grid = rounds x resident workgroups
  int batch_cost16 = 11;               // register-phase fixed cost, sixteenths of N
  int lmode[2] = {0, 0};               // large: 0 three passes, 1 GEMM epilogue writes the
                                       // output order, 2 one pass (no workspace)
  int ltile_kb[2] = {40, 40};          // large: stage-pass tile size
  int op_grid[2] = {0, 0};             // large, one pass: most workgroups (0: one per panel;
                                       // built in: the resident workgroups, persistent)
  int lforce[2] = {-1, -1};            // large: form forced by GFT_LARGE_FORM (-1: none)
  bool op_ok[2] = {false, false};      // large: the one-pass form exists for this direction
  OnePass op[2]{};                     // large: one-pass programs (device pointers)
  int tune_source = GFT_TUNE_BUILTIN;
  double tune_ms = 0.0;
};

// Byte blob assembled on the host and uploaded in one copy; offsets are 256-aligned.
struct Blob {
  std::vector<char> bytes;
  size_t add(const void *p, size_t n) {
    const size_t off = bytes.size();
    bytes.resize(off + ((n + 255) & ~(size_t)255), 0);
    if (n) std::memcpy(bytes.data() + off, p, n);
    return off;
  }
};

}  // namespace

struct gft_plan_s {
  std::vector<GraphPlan> graphs;
  gft_options opts{};
  bool batch = false;
  // Product-graph plans: graphs[0] describes the product (n, eigenvalues, statistics); the
  // factor plans and factor bases (node i of basis vector k at [i * n + k], FP64) act along
  // the two axes; order[k] = p * nb + q gives the factor indices of output coefficient k.
  bool product = false;
  GraphPlan fa, fb;
  std::vector<double> ua, ub;
  std::vector<int32_t> order;
  // Plans whose leaf blocks have Kronecker bases (graphs[0].kron): the factor plans' FP64
  // bases, for the separable engine.
  std::vector<double> kua, kub;
  std::mutex mu;
  std::map<int, std::unique_ptr<DeviceImage>> images;

  ~gft_plan_s() {
    for (auto &kv : images) {
      if (kv.second && kv.second->mem) {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess) {
          (void)hipSetDevice(kv.first);
          (void)hipFree(kv.second->mem);
          if (kv.second->mem2) (void)hipFree(kv.second->mem2);
          (void)hipSetDevice(cur);
        }
      }
    }
  }
};

namespace {

gft_options default_options(const gft_options *o) {
  gft_options d{};
  d.precision = GFT_FP32;
  d.order = GFT_ORDER_EIGENVALUE;
  d.tile_override = 0;
  d.engine = GFT_ENGINE_AUTO;
  d.sym_tol = 1e-12;
  if (o) d = *o;
  return d;
}

constexpr size_t kFuseMaxBlocks = 8;   // large engine: fused output permutation up to here

gft_status check_options(const gft_options &o) {
  if (o.precision < GFT_FP32 || o.precision > GFT_SPLIT_BF16)
    return set_error(GFT_ERR_INVALID_ARG, "options.precision is not a gft_precision value");
  if (o.order != GFT_ORDER_EIGENVALUE && o.order != GFT_ORDER_BLOCK)
    return set_error(GFT_ERR_INVALID_ARG, "options.order must be 0 or 1");
  if (o.engine < GFT_ENGINE_AUTO || o.engine > GFT_ENGINE_PRODUCT)
    return set_error(GFT_ERR_INVALID_ARG, "options.engine must be 0, 1, 2, 3 or 4");
  if (o.right_haar != GFT_RIGHT_HAAR_AUTO && o.right_haar != GFT_RIGHT_HAAR_OFF)
    return set_error(GFT_ERR_INVALID_ARG, "options.right_haar must be a gft_right_haar value");
  if (o.autotune != GFT_AUTOTUNE_ON && o.autotune != GFT_AUTOTUNE_OFF)
    return set_error(GFT_ERR_INVALID_ARG, "options.autotune must be a gft_autotune value");
  if (o.laplacian != GFT_LAPLACIAN_COMBINATORIAL && o.laplacian != GFT_LAPLACIAN_NORMALIZED)
    return set_error(GFT_ERR_INVALID_ARG, "options.laplacian must be a gft_laplacian value");
  if ((o.in_dtype != GFT_DTYPE_FP32 && o.in_dtype != GFT_DTYPE_BF16) ||
      (o.out_dtype != GFT_DTYPE_FP32 && o.out_dtype != GFT_DTYPE_BF16))
    return set_error(GFT_ERR_INVALID_ARG, "options.in_dtype and options.out_dtype must be gft_dtype values");
  if (o.tile_override != 0 && o.tile_override != 16 && o.tile_override != 32 &&
      o.tile_override != 64 && o.tile_override != 128)
    return set_error(GFT_ERR_INVALID_ARG, "options.tile_override must be 0, 16, 32, 64 or 128");
  return GFT_OK;
}

// ---------------------------------------------------------------------------- tuning

// Zero-filled device memory for timing candidates; freed on scope exit.
struct TuneMem {
  void *p = nullptr;
  explicit TuneMem(size_t bytes) {
    if (hipMalloc(&p, bytes) != hipSuccess || hipMemset(p, 0, bytes) != hipSuccess) {
      if (p) (void)hipFree(p);
      p = nullptr;
    }
  }
  ~TuneMem() {
    if (p) (void)hipFree(p);
  }
  TuneMem(const TuneMem &) = delete;
  TuneMem &operator=(const TuneMem &) = delete;
};

// A timing stream; destroyed on scope exit.
struct TuneStream {
  hipStream_t st = nullptr;
  TuneStream() {
    if (hipStreamCreate(&st) != hipSuccess) st = nullptr;
  }
  ~TuneStream() {
    if (st) (void)hipStreamDestroy(st);
  }
};

// Signals of a timing batch of about 16 M values (at least `floor` signals).
int64_t tune_signals(int64_t n, int64_t floor) { return std::max<int64_t>((int64_t)(16 << 20) / n, floor); }

// Key of an image in the tuning cache: device kind, engine, storage and precision, and a
// hash of the uploaded image (programs, matrices and tables) with the plan's sizes.
std::string tune_key(int dev, char engine, const gft_options &o, const std::vector<char> &blob,
                     const std::vector<int32_t> &sizes) {
  uint64_t h = fnv1a(blob.data(), blob.size());
  h = fnv1a(sizes.data(), sizes.size() * sizeof(int32_t), h);
  char hex[17];
  std::snprintf(hex, sizeof hex, "%016llx", (unsigned long long)h);
  return device_tag(dev) + "|" + engine + "|p" + std::to_string(o.precision) + "i" + std::to_string(o.in_dtype) +
         "o" + std::to_string(o.out_dtype) + "t" + std::to_string(o.tile_override) + "|" + hex;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Generic engine: tile height 16 m, every m whose LDS footprint fits `budget` (the products
// run in the same order for any m).
bool tune_generic(DeviceImage *img, size_t budget, bool io16[2][2], std::vector<int32_t> &choice) {
  TuneStream ts;
  if (!ts.st) return false;
  for (int dir = 0; dir < 2; ++dir) {
    DevProgram &P = dir == 0 ? img->fwd[0] : img->inv[0];
    int &cap = dir == 0 ? img->grid_cap_fwd[0] : img->grid_cap_inv[0];
    const int64_t S = tune_signals(P.n, 16 * 8 * (int64_t)img->num_cus);
    TuneMem mem(2 * (size_t)S * P.n * 4);
    if (!mem.p) return false;
    const float *in = static_cast<const float *>(mem.p);
    float *outp = static_cast<float *>(mem.p) + (size_t)S * P.n;
    std::vector<DevProgram> cand;
    std::vector<int> caps;
    int base = -1;
    for (int mt : {8, 4, 2, 1}) {
      DevProgram C = P;
      C.mt = mt;
      if (program_lds_bytes(C) > budget) continue;
      if (mt == P.mt) base = (int)cand.size();
      cand.push_back(C);
      caps.push_back(img->num_cus * apply_occupancy(C));
    }
    if (base < 0) return false;
    const int pick = time_candidates((int)cand.size(), base, [&](int c, hipStream_t st) {
      return launch_apply(cand[c], in, outp, S, st, caps[c], io16[dir][0], io16[dir][1]);
    }, ts.st);
    if (pick < 0) return false;
    P.mt = cand[pick].mt;
    cap = caps[pick];
    choice.push_back(P.mt);
  }
  return true;
}

void apply_generic(DeviceImage *img, const std::vector<int32_t> &choice) {
  for (int dir = 0; dir < 2; ++dir) {
    DevProgram &P = dir == 0 ? img->fwd[0] : img->inv[0];
    P.mt = choice[dir];
    (dir == 0 ? img->grid_cap_fwd[0] : img->grid_cap_inv[0]) = img->num_cus * apply_occupancy(P);
  }
}

// Butterfly and product engines: the persistent grid, 1/2, 3/4, 1 or 2 times the resident
// workgroups (each tile is computed the same way by whichever wave takes it).
bool tune_grid(DeviceImage *img, int n, const std::function<int(int)> &occupancy,
               const std::function<hipError_t(int, const void *, void *, int64_t, hipStream_t, int)> &launch,
               std::vector<int32_t> &choice) {
  TuneStream ts;
  if (!ts.st) return false;
  const int64_t S = tune_signals(n, 4096);
  TuneMem mem(2 * (size_t)S * n * 4);
  if (!mem.p) return false;
  const float *in = static_cast<const float *>(mem.p);
  float *outp = static_cast<float *>(mem.p) + (size_t)S * n;
  for (int dir = 0; dir < 2; ++dir) {
    const int res = occupancy(dir) * img->num_cus;
    const int cand[4] = {std::max(1, res / 2), std::max(1, (3 * res) / 4), res, 2 * res};
    const int pick = time_candidates(4, 2, [&](int c, hipStream_t st) {
      return launch(dir, in, outp, S, st, cand[c]);
    }, ts.st);
    if (pick < 0) return false;
    img->grid[dir] = pick == 2 ? 0 : cand[pick];
    choice.push_back(img->grid[dir]);
  }
  return true;
}

// Large engine: output order by the GEMM epilogue or by a third pass (where the last pass
// has no Haar stage), x stage-pass tiles of 20, 40 or 80 KB.
bool tune_large(gft_plan_s *plan, DeviceImage *img, std::vector<int32_t> &choice);

void run_tuning(gft_plan_s *plan, DeviceImage *img, size_t budget);

// Batch kernel: 1 to 4 rounds of resident workgroups x register-phase cost 8, 11 or 14
// sixteenths of the slot count, on a synthetic batch of the plan's graphs (log-uniform
// 256 .. 65536 signals each, scaled to at most 32 M values).
bool tune_batch(gft_plan_s *plan, DeviceImage *img, std::vector<int32_t> &choice);

// The two factors of a separable plan: their plans, FP64 bases (node i of basis vector k
// at [i * n + k], factor output order) and the factor coefficient pair order[k] = p * nb + q
// of every output coefficient k.
struct Factors {
  int na = 0, nb = 0;
  const GraphPlan *fa = nullptr, *fb = nullptr;
  const std::vector<double> *ua = nullptr, *ub = nullptr;
  const std::vector<int32_t> *order = nullptr;
};

// A factor in its fast form, after its Haar stages: its leaf blocks as one block-diagonal
// matrix Q[pos][c] (pos: node position after the stages, c: coefficient in block order,
// each block scaled by 2^(-depth/2)); bo[p]: block-order index of factor output position p.
struct StagedFactor {
  std::vector<double> Q;
  std::vector<int32_t> bo;
};

StagedFactor staged_factor(const GraphPlan &F) {
  StagedFactor sf;
  const int m = F.n;
  sf.Q.assign((size_t)m * m, 0.0);
  sf.bo.assign(m, -1);
  int c0 = 0;
  for (const HostBlock &B : F.blocks) {
    for (int j = 0; j < B.size; ++j)
      for (int k = 0; k < B.size; ++k)
        sf.Q[(size_t)B.nodes[j] * m + c0 + k] = B.scale * B.V[(size_t)j * B.size + k];
    for (int k = 0; k < B.size; ++k) sf.bo[B.out_pos[k]] = c0 + k;
    c0 += B.size;
  }
  return sf;
}

// Are a 64-node factor's stages the halving reversals the product kernel compiles (stage t
// pairs node i < R/2 with R - 1 - i, R = 64 >> t, six stages, no fixed node), and do its
// leaf matrix's non-zero entries lie in that kernel's tiles ((0,0), (1,1), and the 2 x 2
// group {2, 3} of 16 x 16 tiles)?
bool halving_factor(const GraphPlan &F, const std::vector<double> &Q) {
  if (F.n != 64 || F.stages.size() != 6) return false;
  for (int t = 0; t < 6; ++t) {
    const HostStage &st = F.stages[t];
    const int R = 64 >> t;
    if (!st.znodes.empty() || (int)st.pair_x.size() != R / 2) return false;
    for (int u = 0; u < R / 2; ++u)
      if (st.pair_x[u] != u || st.pair_y[u] != R - 1 - u) return false;
  }
  for (int r = 0; r < 64; ++r)
    for (int c = 0; c < 64; ++c) {
      const int tr = r / 16, tc = c / 16;
      if (Q[(size_t)r * 64 + c] != 0.0 && tr != tc && !(tr >= 2 && tc >= 2)) return false;
    }
  return true;
}

// Device image of a separable plan on device `dev` (caller holds plan->mu): per direction
// the zero-padded factor matrices (dense form: forward B = U_b, A = U_a^T; inverse B = U_b^T,
// A = U_a; staged form: the same with the block-diagonal leaf matrices Q in place of U, and
// the stages compiled into the kernel) and the LDS word of every output-order coefficient.
// The staged form runs where the kernel has it compiled (two 64-node factors with the
// halving stages: 3/8 of the dense MFMA work) with FP32 products; GFT_PRODUCT_FORM=dense or
// staged in the environment forces either form where both exist (tests, measurements).
gft_status product_image(gft_plan_s *plan, const Factors &F, int dev, DeviceImage **out) {
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return set_error(GFT_ERR_HIP, "hipDeviceGetAttribute(CU count)");
  const int na = F.na, nb = F.nb, n = na * nb;
  const std::vector<double> &ua = *F.ua, &ub = *F.ub;
  const std::vector<int32_t> &order = *F.order;
  const int NA = product_pad(na), NB = product_pad(nb), stride = NB + 1;
  const StagedFactor sa = staged_factor(*F.fa), sb = staged_factor(*F.fb);

  // the two forms' matrices (direction d, dense/staged)
  auto build = [&](int d, bool staged, std::vector<float> &A, std::vector<float> &B) {
    A.assign((size_t)NA * NA, 0.0f);
    B.assign((size_t)NB * NB, 0.0f);
    const std::vector<double> &xa = staged ? sa.Q : ua, &xb = staged ? sb.Q : ub;
    for (int i = 0; i < na; ++i)
      for (int k = 0; k < na; ++k) {
        const float u = (float)xa[(size_t)i * na + k];   // row: node (position), column: vector
        if (d == 0) A[(size_t)k * NA + i] = u;
        else A[(size_t)i * NA + k] = u;
      }
    for (int j = 0; j < nb; ++j)
      for (int q = 0; q < nb; ++q) {
        const float u = (float)xb[(size_t)j * nb + q];
        if (d == 0) B[(size_t)j * NB + q] = u;
        else B[(size_t)q * NB + j] = u;
      }
  };
  // FP32 products are MFMA-bound in the dense form (0.70 ms on the 64 x 64 grid against
  // 0.49 ms staged); BF16 and split BF16 are bound by memory and conversions and gain
  // nothing from the staged form (measured 0.43 vs 0.45 ms, 0.54 vs 0.56 ms)
  const bool io16 = plan->opts.in_dtype == GFT_DTYPE_BF16;   // both BF16 (checked at planning)
  const bool compiled = !io16 && halving_factor(*F.fa, sa.Q) && halving_factor(*F.fb, sb.Q);
  bool staged = compiled && plan->opts.precision == GFT_FP32;
  if (const char *f = std::getenv("GFT_PRODUCT_FORM")) {
    if (!std::strcmp(f, "dense")) staged = false;
    else if (!std::strcmp(f, "staged")) staged = compiled;
  }

  Blob blob;
  size_t off[2][3];
  bool same[2];
  for (int d = 0; d < 2; ++d) {
    std::vector<float> A, B;
    build(d, staged, A, B);
    same[d] = na == nb && (staged ? sa.Q == sb.Q : ua == ub);
    std::vector<uint16_t> perm(n);
    for (int k = 0; k < n; ++k) {
      int p = order[k] / nb, q = order[k] % nb;
      if (staged) {
        p = sa.bo[p];
        q = sb.bo[q];
      }
      perm[k] = (uint16_t)(p * stride + q);
    }
    off[d][0] = blob.add(A.data(), A.size() * 4);
    off[d][1] = blob.add(B.data(), B.size() * 4);
    off[d][2] = blob.add(perm.data(), perm.size() * 2);
  }
  auto img = std::make_unique<DeviceImage>();
  img->device = dev;
  img->num_cus = std::max(1, cus);
  img->product_staged = staged;
  e = hipMalloc(&img->mem, blob.bytes.size());
  if (e != hipSuccess) return set_error(GFT_ERR_OOM, "hipMalloc of the plan image failed");
  e = hipMemcpy(img->mem, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(img->mem);
    return set_error(GFT_ERR_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  const char *base = static_cast<const char *>(img->mem);
  PProgram *dst[2] = {&img->pfwd, &img->pinv};
  for (int d = 0; d < 2; ++d) {
    PProgram &P = *dst[d];
    P.na = na;
    P.nb = nb;
    P.dir = d;
    P.stride = stride;
    P.same = same[d];
    P.prec = plan->opts.precision;
    P.amat = reinterpret_cast<const float *>(base + off[d][0]);
    P.bmat = reinterpret_cast<const float *>(base + off[d][1]);
    P.perm = reinterpret_cast<const uint16_t *>(base + off[d][2]);
    P.tile_pattern = io16 ? 2 : (staged ? 1 : 0);
  }
  img->product = true;
  img->key = tune_key(dev, 'P', plan->opts, blob.bytes, {na, nb, staged ? 1 : 0});
  run_tuning(plan, img.get(), 0);
  *out = img.get();
  plan->images[dev] = std::move(img);
  return GFT_OK;
}

// Built-in output order of a large-engine apply: with no Haar stage in pass 3 and few leaf
// blocks the GEMM writes the final positions itself (no W2, no pass 3).  With many blocks
// whose outputs interleave in the output order, each output line collects partial writes
// from many workgroups and the m-panel tile order spoils the reuse of the block matrices in
// L2: measured slower on the 64x64 grid (49 blocks), faster on the 1024-node path (2
// blocks).  The tuner may choose either where the last pass has no stage.
bool large_fusable(const LargeImage &L) { return L.pass[1].num_stages == 0; }
bool large_fused(const LargeImage &L) { return large_fusable(L) && L.blocks.size() <= kFuseMaxBlocks; }

// Whether form `mode` (DeviceImage::lmode) can run direction dir of the image.
bool large_mode_ok(const DeviceImage *img, int dir, int mode) {
  return mode == 0 || (mode == 1 && large_fusable(img->lg[dir])) || (mode == 2 && img->op_ok[dir]);
}

// Workspace of a large-engine apply over S signals: W1 (and W2 unless the GEMM epilogue
// writes the output order) of S rows of ldw FP32 words; none in one pass.
size_t large_ws_bytes(const LargeImage &L, int mode, int64_t S) {
  return mode == 2 ? 0 : (mode == 1 ? 1 : 2) * (size_t)S * (size_t)L.ldw * 4;
}

// The large engine's launches for one apply in form `mode`: one kernel (mode 2), or the
// stage/gather pass, grouped GEMM, and the gather pass unless the GEMM writes the output
// order (mode 1); ws holds large_ws_bytes.  tile_kb: stage-pass tile (modes 0, 1); grid:
// one-pass workgroups (mode 2).
hipError_t launch_large(const gft_plan_s *plan, const DeviceImage *img, int dir, const void *in, void *out,
                        int64_t S, hipStream_t st, void *ws, int mode, int tile_kb, int grid) {
  const LargeImage &L = img->lg[dir];
  // storage: the forward reads signals (in_dtype) and writes coefficients (out_dtype)
  const bool in16 = (dir == 0 ? plan->opts.in_dtype : plan->opts.out_dtype) == GFT_DTYPE_BF16;
  const bool out16 = (dir == 0 ? plan->opts.out_dtype : plan->opts.in_dtype) == GFT_DTYPE_BF16;
  if (mode == 2)
    return launch_onepass(img->op[dir], plan->opts.precision, in, out, S, in16, out16, grid, st);
  const bool fused = mode == 1;
  float *W1 = static_cast<float *>(ws), *W2 = fused ? nullptr : W1 + (size_t)S * L.ldw;
  const bool ws16 = plan->opts.precision == GFT_BF16;   // BF16 workspace and matrices
  hipError_t e = launch_permute_stages(L.pass[0], in, in16, W1, ws16, S, img->num_cus, st, tile_kb);
  if (e == hipSuccess)
    e = launch_block_gemm(plan->opts.precision == GFT_FP32 ? 0 : plan->opts.precision, L.dev_blocks,
                          (int)L.blocks.size(), ws16 ? (const void *)L.dev_mats16 : (const void *)L.dev_mats,
                          W1, fused ? out : (void *)W2, fused && out16, S, L.ldw,
                          block_gemm_grid(L.block_sizes.data(), (int)L.blocks.size(), S),
                          fused ? L.dev_omap : nullptr, L.n, st);
  if (e == hipSuccess && !fused)
    e = launch_permute_stages(L.pass[1], W2, false, out, out16, S, img->num_cus, st, tile_kb);
  return e;
}

bool tune_large(gft_plan_s *plan, DeviceImage *img, std::vector<int32_t> &choice) {
  TuneStream ts;
  if (!ts.st) return false;
  const int n = plan->graphs[0].n;
  const int64_t S = tune_signals(n, 1024);
  const size_t ws = std::max(large_ws_bytes(img->lg[0], 0, S), large_ws_bytes(img->lg[1], 0, S));
  TuneMem mem(2 * (size_t)S * n * 4 + ws);
  if (!mem.p) return false;
  const float *in = static_cast<const float *>(mem.p);
  float *outp = static_cast<float *>(mem.p) + (size_t)S * n;
  void *wsp = static_cast<char *>(mem.p) + 2 * (size_t)S * n * 4;
  for (int dir = 0; dir < 2; ++dir) {
    struct Cand {
      int mode, arg;   // arg: stage-pass tile KB (modes 0, 1) or one-pass grid (mode 2)
    };
    std::vector<Cand> cand;
    int base = 0;
    const bool in16 = (dir == 0 ? plan->opts.in_dtype : plan->opts.out_dtype) == GFT_DTYPE_BF16;
    const int resident =
        img->num_cus * (img->op_ok[dir] ? onepass_occupancy(img->op[dir], plan->opts.precision, in16) : 1);
    for (int m = 0; m < 3; ++m) {
      if (!large_mode_ok(img, dir, m) || (img->lforce[dir] >= 0 && m != img->lforce[dir])) continue;
      // one-pass grids: the resident workgroups, and one workgroup per panel where the
      // timed signals hold more panels than that (else the two are the same launch, and
      // a pick between them would follow timing noise, not the full-size behaviour)
      const int64_t panels = (S + onepass_rows(plan->opts.precision) - 1) / onepass_rows(plan->opts.precision);
      const std::vector<int> args = m != 2 ? std::vector<int>{20, 40, 80}
                                    : panels > resident ? std::vector<int>{0, resident}
                                                        : std::vector<int>{resident};
      for (int a : args) {
        if (m == img->lmode[dir] && a == (m == 2 ? img->op_grid[dir] : img->ltile_kb[dir])) base = (int)cand.size();
        cand.push_back({m, a});
      }
    }
    const int pick = time_candidates((int)cand.size(), base, [&](int c, hipStream_t st) {
      return launch_large(plan, img, dir, in, outp, S, st, wsp, cand[c].mode, cand[c].mode == 2 ? 40 : cand[c].arg,
                          cand[c].mode == 2 ? cand[c].arg : 0);
    }, ts.st);
    if (pick < 0) return false;
    img->lmode[dir] = cand[pick].mode;
    if (cand[pick].mode == 2) img->op_grid[dir] = cand[pick].arg;
    else img->ltile_kb[dir] = cand[pick].arg;
    choice.push_back(cand[pick].mode);
    choice.push_back(cand[pick].arg);
  }
  return true;
}

bool tune_batch(gft_plan_s *plan, DeviceImage *img, std::vector<int32_t> &choice) {
  TuneStream ts;
  if (!ts.st) return false;
  const int G = (int)plan->graphs.size();
  // log-uniform counts from a fixed linear congruential sequence
  std::vector<int64_t> cnt(G);
  uint64_t x = 0x9e3779b97f4a7c15ull;
  int64_t total = 0;
  for (int g = 0; g < G; ++g) {
    x = x * 6364136223846793005ull + 1442695040888963407ull;
    const double u = (double)(x >> 11) / 9007199254740992.0;
    cnt[g] = (int64_t)std::exp(std::log(256.0) + u * (std::log(65536.0) - std::log(256.0)));
    total += cnt[g] * plan->graphs[g].n;
  }
  const int64_t cap = (int64_t)32 << 20;
  if (total > cap)
    for (int g = 0; g < G; ++g) cnt[g] = std::max<int64_t>(16, (int64_t)((double)cnt[g] * cap / total));
  std::vector<int64_t> off(G + 1, 0);
  int64_t E = 0;
  for (int g = 0; g < G; ++g) {
    off[g + 1] = off[g] + cnt[g];
    E += cnt[g] * plan->graphs[g].n;
  }
  TuneMem mem(2 * (size_t)E * 4 + off.size() * 8);
  if (!mem.p) return false;
  const float *in = static_cast<const float *>(mem.p);
  float *outp = static_cast<float *>(mem.p) + E;
  int64_t *doff = reinterpret_cast<int64_t *>(static_cast<char *>(mem.p) + 2 * (size_t)E * 4);
  if (hipMemcpy(doff, off.data(), off.size() * 8, hipMemcpyHostToDevice) != hipSuccess) return false;
  struct Cand {
    int rounds, cost16;
  };
  std::vector<Cand> cand;
  int base = 0;
  for (int r = 1; r <= 4; ++r)
    for (int c : {8, 11, 14}) {
      if (r == img->batch_rounds && c == img->batch_cost16) base = (int)cand.size();
      cand.push_back({r, c});
    }
  const int pick = time_candidates((int)cand.size(), base, [&](int c, hipStream_t st) {
    return launch_apply_batch(plan->opts.precision, 0, plan->opts.in_dtype == GFT_DTYPE_BF16, img->dev_fwd,
                              img->dev_ufwd, G, doff, E, in, outp,
                              img->batch_lds, cand[c].rounds * img->num_cus * img->batch_occ, img->reg_groups,
                              cand[c].cost16, st);
  }, ts.st);
  if (pick < 0) return false;
  img->batch_rounds = cand[pick].rounds;
  img->batch_cost16 = cand[pick].cost16;
  choice = {img->batch_rounds, img->batch_cost16};
  return true;
}

// Tune the image's launch choices (options.autotune on), or take them from the cache.  On
// any failure the built-in choices stay.
void run_tuning(gft_plan_s *plan, DeviceImage *img, size_t budget) {
  const gft_options &o = plan->opts;
  if (o.autotune == GFT_AUTOTUNE_OFF) return;
  enum { GENERIC, BUTTERFLY, PRODUCT, LARGE, BATCH } kind =
      plan->batch ? BATCH : img->product ? PRODUCT : img->butterfly ? BUTTERFLY : img->large ? LARGE : GENERIC;
  if (kind == GENERIC && o.tile_override != 0) return;   // the caller fixed the tile
  if (kind == BATCH && !img->dev_ufwd) {
    // no register phase: only the rounds matter, still tuned below
  }
  bool io16[2][2];
  for (int d = 0; d < 2; ++d) {
    io16[d][0] = (d == 0 ? o.in_dtype : o.out_dtype) == GFT_DTYPE_BF16;
    io16[d][1] = (d == 0 ? o.out_dtype : o.in_dtype) == GFT_DTYPE_BF16;
  }
  // a cached choice, validated before use
  std::vector<int32_t> v;
  if (tune_cache_get(img->key, v)) {
    bool valid = false;
    switch (kind) {
      case GENERIC:
        valid = v.size() == 2;
        for (int d = 0; d < 2 && valid; ++d) {
          DevProgram C = d == 0 ? img->fwd[0] : img->inv[0];
          C.mt = v[d];
          valid = (v[d] == 1 || v[d] == 2 || v[d] == 4 || v[d] == 8) && program_lds_bytes(C) <= budget;
        }
        if (valid) apply_generic(img, v);
        break;
      case BUTTERFLY:
      case PRODUCT:
        valid = v.size() == 2 && v[0] >= 0 && v[1] >= 0;
        if (valid) img->grid[0] = v[0], img->grid[1] = v[1];
        break;
      case LARGE:
        valid = v.size() == 4;
        for (int d = 0; d < 2 && valid; ++d)
          valid = v[2 * d] >= 0 && v[2 * d] <= 2 && large_mode_ok(img, d, v[2 * d]) &&
                  (img->lforce[d] < 0 || v[2 * d] == img->lforce[d]) &&
                  (v[2 * d] == 2 ? v[2 * d + 1] >= 0
                                 : (v[2 * d + 1] == 20 || v[2 * d + 1] == 40 || v[2 * d + 1] == 80));
        if (valid)
          for (int d = 0; d < 2; ++d) {
            img->lmode[d] = v[2 * d];
            if (v[2 * d] == 2) img->op_grid[d] = v[2 * d + 1];
            else img->ltile_kb[d] = v[2 * d + 1];
          }
        break;
      case BATCH:
        valid = v.size() == 2 && v[0] >= 1 && v[0] <= 4 && v[1] >= 1 && v[1] <= 64;
        if (valid) img->batch_rounds = v[0], img->batch_cost16 = v[1];
        break;
    }
    if (valid) {
      img->tune_source = GFT_TUNE_CACHED;
      return;
    }
  }
  // time the candidates
  const double t0 = now_ms();
  std::vector<int32_t> choice;
  bool done = false;
  const std::vector<int> mts = kind == GENERIC ? std::vector<int>{img->fwd[0].mt, img->inv[0].mt} : std::vector<int>{};
  switch (kind) {
    case GENERIC:
      done = tune_generic(img, budget, io16, choice);
      if (!done) apply_generic(img, {mts[0], mts[1]});
      break;
    case BUTTERFLY:
      done = tune_grid(img, plan->graphs[0].n,
                       [&](int d) { return butterfly_occupancy(d == 0 ? img->bfwd : img->binv, io16[d][0], io16[d][1]); },
                       [&](int d, const void *in, void *out, int64_t S, hipStream_t st, int cap) {
                         return launch_butterfly(d == 0 ? img->bfwd : img->binv, in, out, S, st, img->num_cus,
                                                 io16[d][0], io16[d][1], cap);
                       },
                       choice);
      if (!done) img->grid[0] = img->grid[1] = 0;
      break;
    case PRODUCT:
      done = tune_grid(img, plan->graphs[0].n,
                       [&](int d) { return product_occupancy(d == 0 ? img->pfwd : img->pinv); },
                       [&](int d, const void *in, void *out, int64_t S, hipStream_t st, int cap) {
                         return launch_product(d == 0 ? img->pfwd : img->pinv, static_cast<const float *>(in),
                                               static_cast<float *>(out), S, st, img->num_cus, cap);
                       },
                       choice);
      if (!done) img->grid[0] = img->grid[1] = 0;
      break;
    case LARGE: {
      const int m0 = img->lmode[0], m1 = img->lmode[1];
      done = tune_large(plan, img, choice);
      if (!done) {
        img->lmode[0] = m0, img->lmode[1] = m1, img->ltile_kb[0] = img->ltile_kb[1] = 40;
        for (int d = 0; d < 2; ++d)
          if (img->op_ok[d]) {
            const bool in16 = (d == 0 ? plan->opts.in_dtype : plan->opts.out_dtype) == GFT_DTYPE_BF16;
            img->op_grid[d] = img->num_cus * onepass_occupancy(img->op[d], plan->opts.precision, in16);
          }
      }
      break;
    }
    case BATCH:
      done = tune_batch(plan, img, choice);
      if (!done) img->batch_rounds = 2, img->batch_cost16 = 11;
      break;
  }
  (void)hipGetLastError();
  if (!done) return;
  tune_cache_put(img->key, choice);
  img->tune_source = GFT_TUNE_TIMED;
  img->tune_ms = now_ms() - t0;
}

// Get (building on first use) the image of `plan` on the current device.
gft_status device_image(gft_plan_s *plan, DeviceImage **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(GFT_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  std::lock_guard<std::mutex> lock(plan->mu);
  auto it = plan->images.find(dev);
  if (it != plan->images.end()) {
    *out = it->second.get();
    return GFT_OK;
  }
  if (plan->product) {
    const Factors F{plan->fa.n, plan->fb.n, &plan->fa, &plan->fb, &plan->ua, &plan->ub, &plan->order};
    return product_image(plan, F, dev, out);
  }
  int max_lds = 0, cus = 0;
  e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return set_error(GFT_ERR_HIP, "hipDeviceGetAttribute(shared memory)");
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return set_error(GFT_ERR_HIP, "hipDeviceGetAttribute(CU count)");
  size_t budget = std::min<size_t>(kMaxLdsBytes, (size_t)max_lds);
  const int G = (int)plan->graphs.size();
  if (plan->batch) {
    // the batch kernel keeps G+1 element offsets and the scan's wave totals in LDS as well
    const size_t fixed = batch_lds_bytes(G, 0, false) + 96 + 256;
    if (fixed + 4096 > budget) return set_error(GFT_ERR_UNSUPPORTED, "too many graphs in one batch plan");
    budget -= fixed;
  }

  // Register-butterfly engine for single-graph plans of the shapes it covers (uniform
  // hypercubes, padded one- and two-stage layouts).
  UProgramImage ub[2];
  bool use_bf = false;
  const int prec = plan->opts.precision;
  if (plan->opts.engine == GFT_ENGINE_BUTTERFLY &&
      (plan->batch || (prec != GFT_FP32 && prec != GFT_BF16)))
    return set_error(GFT_ERR_UNSUPPORTED,
                     "the register-butterfly engine runs single-graph FP32 or BF16 plans only");
  if (!plan->batch && (plan->opts.engine == GFT_ENGINE_AUTO || plan->opts.engine == GFT_ENGINE_BUTTERFLY) &&
      (prec == GFT_FP32 || prec == GFT_BF16)) {
    use_bf = build_butterfly(plan->graphs[0], 0, ub[0], prec) && build_butterfly(plan->graphs[0], 1, ub[1], prec) &&
             butterfly_supported(ub[0].prog) && butterfly_supported(ub[1].prog);
    if (!use_bf && plan->opts.engine == GFT_ENGINE_BUTTERFLY)
      return set_error(GFT_ERR_UNSUPPORTED,
                       "the register-butterfly engine does not cover this plan (needs a uniform "
                       "hypercube with a compiled shape, one stage with 8 <= n <= 96 and sides of at "
                       "most 48 nodes, or two stages on sides of at most 32 slots, and no right Haar "
                       "units; BF16 blocks: the one-stage form only)");
  }

  // Batch plans: every graph whose plan the batch kernel's register-butterfly forms cover
  // runs there (unless the generic engine is forced); the others run their LDS programs.
  std::vector<UProgramImage> bub;            // 2 per graph (forward, inverse); empty: LDS program
  std::vector<char> breg(G, 0);
  if (plan->batch && plan->opts.engine == GFT_ENGINE_AUTO) {
    bub.resize((size_t)2 * G);
    for (int g = 0; g < G; ++g) {
      UProgramImage f, i;
      if (build_butterfly(plan->graphs[g], 0, f, prec) && build_butterfly(plan->graphs[g], 1, i, prec) &&
          batch_butterfly_supported(prec, f.prog) && batch_butterfly_supported(prec, i.prog)) {
        bub[2 * g] = std::move(f);
        bub[2 * g + 1] = std::move(i);
        breg[g] = 1;
      }
    }
  }

  // Large-signal engine: signals whose 16-signal tile does not fit LDS, or big leaf blocks.
  bool use_large = false;
  if (!plan->batch && !use_bf && plan->opts.engine != GFT_ENGINE_GENERIC) {
    ProgramImage probe;
    const bool fits = build_program(plan->graphs[0], 0, 0, budget, probe, plan->opts.precision);
    use_large = plan->opts.engine == GFT_ENGINE_LARGE ||
                (plan->opts.engine == GFT_ENGINE_AUTO &&
                 (!fits || plan->graphs[0].stats.max_block >= 192));
    if (use_large && plan->opts.precision == GFT_FP16)
      return set_error(GFT_ERR_UNSUPPORTED, "the large-signal engine runs FP32, BF16 or split BF16 blocks");
  }
  if (plan->opts.engine == GFT_ENGINE_LARGE && plan->batch)
    return set_error(GFT_ERR_UNSUPPORTED, "batch plans run the generic engine");

  // Separable engine for plans whose leaf blocks all have Kronecker bases (Sec. V-D): in
  // place of the large engine, or when asked for.
  const KronPlan *K = plan->batch ? nullptr : plan->graphs[0].kron.get();
  const bool sep_ok = K && prec != GFT_FP16 && plan->opts.in_dtype == plan->opts.out_dtype &&
                      product_pad(K->na) && product_pad(K->nb);
  if (plan->opts.engine == GFT_ENGINE_PRODUCT || (plan->opts.engine == GFT_ENGINE_AUTO && use_large && sep_ok)) {
    if (!sep_ok)
      return set_error(GFT_ERR_UNSUPPORTED,
                       "the separable engine runs single-graph plans whose leaf blocks have Kronecker "
                       "bases (a row-major Cartesian product with stages along the axes, factors of at "
                       "most 64 nodes), one storage type for signals and coefficients and FP32, BF16 or "
                       "split BF16 blocks");
    const Factors F{K->na, K->nb, K->fa.get(), K->fb.get(), &plan->kua, &plan->kub, &K->order};
    return product_image(plan, F, dev, out);
  }

  std::vector<ProgramImage> imgs;
  for (size_t g = 0; g < plan->graphs.size(); ++g)
    for (int dir = 0; dir < 2; ++dir) {
      ProgramImage im;
      if (!build_program(plan->graphs[g], dir, plan->opts.tile_override, budget, im,
                         plan->opts.precision)) {
        if (use_bf || use_large) continue;  // another engine serves this graph
        return set_error(GFT_ERR_UNSUPPORTED,
                         "graph " + std::to_string(g) + " (n = " + std::to_string(plan->graphs[g].n) +
                             ") does not fit the LDS of one workgroup with this tile size");
      }
      imgs.push_back(std::move(im));
    }
  Blob blob;
  std::vector<size_t> toff(imgs.size()), foff(imgs.size());
  for (size_t i = 0; i < imgs.size(); ++i) {
    toff[i] = blob.add(imgs[i].table.data(), imgs[i].table.size() * 4);
    foff[i] = blob.add(imgs[i].frag.data(), imgs[i].frag.size() * 4);
  }
  size_t uoff[2][4] = {};
  if (use_bf)
    for (int d = 0; d < 2; ++d) {
      uoff[d][0] = blob.add(ub[d].gcol.data(), ub[d].gcol.size() * 4);
      uoff[d][1] = blob.add(ub[d].scol.data(), ub[d].scol.size() * 4);
      uoff[d][2] = blob.add(ub[d].afrag.data(), ub[d].afrag.size() * 4);
      uoff[d][3] = blob.add(ub[d].flips.data(), ub[d].flips.size() * 4);
    }
  std::vector<size_t> boff(bub.size() * 4, 0);
  for (size_t k = 0; k < bub.size(); ++k)
    if (breg[k / 2]) {
      boff[4 * k + 0] = blob.add(bub[k].gcol.data(), bub[k].gcol.size() * 4);
      boff[4 * k + 1] = blob.add(bub[k].scol.data(), bub[k].scol.size() * 4);
      boff[4 * k + 2] = blob.add(bub[k].afrag.data(), bub[k].afrag.size() * 4);
      boff[4 * k + 3] = blob.add(bub[k].flips.data(), bub[k].flips.size() * 4);
    }
  LargeImage lgi[2];
  size_t loff[2][8] = {};
  if (use_large)
    for (int d = 0; d < 2; ++d) {
      if (!build_large(plan->graphs[0], d, lgi[d]))
        return set_error(GFT_ERR_UNSUPPORTED, "the large-signal engine takes rows of at most " +
                                                  std::to_string(kLargeMaxCols) +
                                                  " values and workspace columns (one FP32 row in LDS)");
      for (int k = 0; k < 2; ++k) {
        loff[d][2 * k] = blob.add(lgi[d].stages[k].data(), lgi[d].stages[k].size() * 4);
        loff[d][2 * k + 1] = blob.add(lgi[d].gather[k].data(), lgi[d].gather[k].size() * 4);
        loff[d][4 + k] = blob.add(lgi[d].ops[k].data(), lgi[d].ops[k].size() * 4);
      }
      loff[d][6] = blob.add(lgi[d].blocks.data(), lgi[d].blocks.size() * sizeof(LBlock));
      loff[d][7] = blob.add(lgi[d].omap.data(), lgi[d].omap.size() * 4);
      lgi[d].block_sizes.shrink_to_fit();
      // matrices last (largest)
    }
  size_t lmat[2] = {};
  const bool mats16 = plan->opts.precision == GFT_BF16;   // the GEMM reads one of the two
  if (use_large)
    for (int d = 0; d < 2; ++d)
      lmat[d] = mats16 ? blob.add(lgi[d].mats16.data(), lgi[d].mats16.size() * 2)
                       : blob.add(lgi[d].mats.data(), lgi[d].mats.size() * 4);
  // the one-pass form where the plan fits it (its tables and B fragments)
  OnePassImage opi[2];
  bool op_ok[2] = {false, false};
  // GFT_ONEPASS_GENERAL=1: the one-pass form with its general source modes only (testing)
  const char *gen_env = std::getenv("GFT_ONEPASS_GENERAL");
  const bool onepass_general = gen_env && std::strcmp(gen_env, "1") == 0;
  size_t ooff[2][3] = {};
  if (use_large)
    for (int d = 0; d < 2; ++d)
      if ((op_ok[d] = build_onepass(lgi[d], plan->opts.precision,
                                    (d == 0 ? plan->opts.in_dtype : plan->opts.out_dtype) == GFT_DTYPE_BF16,
                                    opi[d], onepass_general))) {
        ooff[d][0] = blob.add(opi[d].desc.data(), opi[d].desc.size() * 4);
        ooff[d][1] = blob.add(opi[d].frag.data(), opi[d].frag.size() * 4);
        if (!opi[d].omap.empty()) ooff[d][2] = blob.add(opi[d].omap.data(), opi[d].omap.size() * 4);
      }
  const size_t bytes = blob.bytes.size();
  auto img = std::make_unique<DeviceImage>();
  img->device = dev;
  img->num_cus = std::max(1, cus);
  e = hipMalloc(&img->mem, bytes ? bytes : 256);
  if (e != hipSuccess) return set_error(GFT_ERR_OOM, "hipMalloc of the plan image failed");
  e = hipMemcpy(img->mem, blob.bytes.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(img->mem);
    return set_error(GFT_ERR_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  char *base = static_cast<char *>(img->mem);
  for (size_t i = 0; i < imgs.size(); ++i) {
    DevProgram P = imgs[i].prog;
    P.table = reinterpret_cast<const int32_t *>(base + toff[i]);
    P.frag = reinterpret_cast<const uint32_t *>(base + foff[i]);
    const int cap = img->num_cus * apply_occupancy(P);
    if (i % 2 == 0) {
      img->fwd.push_back(P);
      img->grid_cap_fwd.push_back(cap);
    } else {
      img->inv.push_back(P);
      img->grid_cap_inv.push_back(cap);
    }
  }
  if (use_bf) {
    img->butterfly = true;
    UProgram *dst[2] = {&img->bfwd, &img->binv};
    for (int d = 0; d < 2; ++d) {
      *dst[d] = ub[d].prog;
      dst[d]->gcol = reinterpret_cast<const int32_t *>(base + uoff[d][0]);
      dst[d]->scol = reinterpret_cast<const int32_t *>(base + uoff[d][1]);
      dst[d]->afrag = reinterpret_cast<const float *>(base + uoff[d][2]);
      dst[d]->flips = reinterpret_cast<const uint32_t *>(base + uoff[d][3]);
    }
  }
  if (use_large) {
    img->large = true;
    // the allocation-free apply's workspace: this device's address of the static scratch
    e = large_scratch_setup(dev);
    if (e != hipSuccess) {
      (void)hipFree(img->mem);
      return set_error(GFT_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    for (int d = 0; d < 2; ++d) {
      LargeImage &L = img->lg[d];
      L = std::move(lgi[d]);
      for (int k = 0; k < 2; ++k) {
        PermPass &P = L.pass[k];
        P.gather = L.gather[k].empty() ? nullptr : reinterpret_cast<const int32_t *>(base + loff[d][2 * k + 1]);
        P.stages = reinterpret_cast<const int32_t *>(base + loff[d][2 * k]);
        P.ops = reinterpret_cast<const uint32_t *>(base + loff[d][4 + k]);
      }
      L.dev_blocks = reinterpret_cast<const LBlock *>(base + loff[d][6]);
      L.dev_omap = reinterpret_cast<const int32_t *>(base + loff[d][7]);
      L.dev_mats = mats16 ? nullptr : reinterpret_cast<const float *>(base + lmat[d]);
      L.dev_mats16 = mats16 ? reinterpret_cast<const uint16_t *>(base + lmat[d]) : nullptr;
      L.mats.clear();
      L.mats.shrink_to_fit();
      L.mats16.clear();
      L.mats16.shrink_to_fit();
      if (op_ok[d]) {
        OnePass &O = img->op[d];
        O = opi[d].P;
        O.desc = reinterpret_cast<const int32_t *>(base + ooff[d][0]);
        O.frag = reinterpret_cast<const uint32_t *>(base + ooff[d][1]);
        O.gather3 = L.pass[1].gather;
        O.stages3 = L.pass[1].stages;
        O.ops3 = L.pass[1].ops;
        O.omap3 = O.src_mode == 5 ? reinterpret_cast<const int32_t *>(base + ooff[d][2]) : nullptr;
        img->op_ok[d] = O.gather3 != nullptr;   // the last pass always gathers
        // built-in grid: the resident workgroups, each taking panels in turn (its LDS tables
        // are copied once; 1.5-6 % faster than one workgroup per panel at 16 panels per CU)
        const bool in16 = (d == 0 ? plan->opts.in_dtype : plan->opts.out_dtype) == GFT_DTYPE_BF16;
        img->op_grid[d] = img->num_cus * onepass_occupancy(O, plan->opts.precision, in16);
      }
      // built-in form: one pass where it exists (no workspace; every value visits HBM
      // once), else the GEMM epilogue writing the output order where the last pass has
      // no stage and few blocks, else three passes; GFT_LARGE_FORM=passes, epilogue or
      // onepass forces a form where the plan allows it
      img->lmode[d] = img->op_ok[d] ? 2 : (large_fused(L) ? 1 : 0);
      if (const char *f = std::getenv("GFT_LARGE_FORM")) {
        const int m = !std::strcmp(f, "passes") ? 0 : !std::strcmp(f, "epilogue") ? 1 : !std::strcmp(f, "onepass") ? 2 : -1;
        if (m >= 0 && large_mode_ok(img.get(), d, m)) img->lmode[d] = img->lforce[d] = m;
      }
    }
  }
  if (plan->batch) {
    std::vector<DevProgram> arr;
    size_t maxlds = 0;
    for (int d = 0; d < 2; ++d)
      for (int g = 0; g < G; ++g) {
        const DevProgram &P = d == 0 ? img->fwd[g] : img->inv[g];
        arr.push_back(P);
        if (!breg[g]) maxlds = std::max(maxlds, program_lds_bytes(P));
      }
    const bool any_reg = std::find(breg.begin(), breg.end(), 1) != breg.end();
    std::vector<UProgram> uarr;
    if (any_reg)
      for (int d = 0; d < 2; ++d)
        for (int g = 0; g < G; ++g) {
          UProgram U{};   // S = 0: the graph runs its LDS program
          if (breg[g]) {
            const size_t k = (size_t)2 * g + d;
            U = bub[k].prog;
            U.gcol = reinterpret_cast<const int32_t *>(base + boff[4 * k + 0]);
            U.scol = reinterpret_cast<const int32_t *>(base + boff[4 * k + 1]);
            U.afrag = reinterpret_cast<const float *>(base + boff[4 * k + 2]);
            U.flips = reinterpret_cast<const uint32_t *>(base + boff[4 * k + 3]);
          }
          uarr.push_back(U);
        }
    const size_t pbytes = arr.size() * sizeof(DevProgram);
    const size_t ubytes = uarr.size() * sizeof(UProgram);
    void *parr = nullptr;
    e = hipMalloc(&parr, pbytes + ubytes);
    if (e != hipSuccess) {
      (void)hipFree(img->mem);
      return set_error(GFT_ERR_OOM, "hipMalloc of the batch program array failed");
    }
    e = hipMemcpy(parr, arr.data(), pbytes, hipMemcpyHostToDevice);
    if (e == hipSuccess && ubytes)
      e = hipMemcpy(static_cast<char *>(parr) + pbytes, uarr.data(), ubytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(parr);
      (void)hipFree(img->mem);
      return set_error(GFT_ERR_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    img->mem2 = parr;
    img->dev_fwd = static_cast<const DevProgram *>(parr);
    img->dev_inv = img->dev_fwd + G;
    if (any_reg) {
      img->dev_ufwd = reinterpret_cast<const UProgram *>(static_cast<char *>(parr) + pbytes);
      img->dev_uinv = img->dev_ufwd + G;
    }
    img->batch_lds = batch_lds_bytes(G, maxlds, any_reg);
    img->batch_occ = batch_occupancy(plan->opts.precision, img->batch_lds, plan->opts.in_dtype == GFT_DTYPE_BF16);
    // built-in: two rounds of resident workgroups (the hardware hands the second round's
    // byte-equal shares of the LDS-program graphs to CUs as they free up, which evens out
    // graphs of different cost per byte, while each share stays long enough to amortise
    // loading its program; measured on the mixed batch: four rounds 193 us, three 195 us,
    // two 187 us); the register phase runs on the first round
    img->batch_rounds = 2;
    img->reg_groups = any_reg ? img->num_cus * img->batch_occ : 0;
  }
  {
    std::vector<int32_t> sizes;
    for (const GraphPlan &g : plan->graphs) sizes.push_back(g.n);
    const char kind = plan->batch ? 'B' : (img->butterfly ? 'F' : (img->large ? 'L' : 'G'));
    img->key = tune_key(dev, kind, plan->opts, blob.bytes, sizes);
  }
  run_tuning(plan, img.get(), budget);
  *out = img.get();
  plan->images[dev] = std::move(img);
  return GFT_OK;
}

gft_status check_buffers(const void *a, int64_t abytes, const void *b, int64_t bbytes,
                         bool same_type) {
  if (!a || !b) return set_error(GFT_ERR_INVALID_ARG, "x and y must be non-NULL device pointers");
  if ((reinterpret_cast<uintptr_t>(a) & 15) || (reinterpret_cast<uintptr_t>(b) & 15))
    return set_error(GFT_ERR_ALIGNMENT, "x and y must be 16-byte aligned");
  const uintptr_t pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  if (pa == pb && !same_type)
    return set_error(GFT_ERR_ALIGNMENT, "in-place transforms need equal storage types for x and y");
  if (pa != pb && pa < pb + (uintptr_t)bbytes && pb < pa + (uintptr_t)abytes)
    return set_error(GFT_ERR_ALIGNMENT, "x and y overlap without being equal");
  return GFT_OK;
}

gft_status check_apply_args(gft_plan_t plan, const void *in, void *out, int64_t S, int dir) {
  if (!plan) return set_error(GFT_ERR_INVALID_ARG, "plan is NULL");
  if (plan->batch) return set_error(GFT_ERR_INVALID_ARG, "batch plans use gft_forward_batch / gft_inverse_batch");
  if (S < 0) return set_error(GFT_ERR_INVALID_ARG, "num_signals must be >= 0");
  if (S == 0) return GFT_OK;
  const int64_t n = plan->graphs[0].n;
  if (S > (int64_t(1) << 40) / n) return set_error(GFT_ERR_INVALID_ARG, "num_signals too large");
  // forward reads signals (in_dtype) and writes coefficients (out_dtype); inverse the reverse
  const bool in16 = (dir == 0 ? plan->opts.in_dtype : plan->opts.out_dtype) == GFT_DTYPE_BF16;
  const bool out16 = (dir == 0 ? plan->opts.out_dtype : plan->opts.in_dtype) == GFT_DTYPE_BF16;
  return check_buffers(in, S * n * (in16 ? 2 : 4), out, S * n * (out16 ? 2 : 4), in16 == out16);
}

// Launch the plan's kernels on S > 0 signals with the image's launch choices.  ws: the
// large engine's workspace (at least large_ws_bytes), or null to take it from the
// stream-ordered pool for this call.
gft_status launch_image(gft_plan_t plan, DeviceImage *img, int dir, const void *in, void *out,
                        int64_t S, void *stream, void *ws) {
  const bool in16 = (dir == 0 ? plan->opts.in_dtype : plan->opts.out_dtype) == GFT_DTYPE_BF16;
  const bool out16 = (dir == 0 ? plan->opts.out_dtype : plan->opts.in_dtype) == GFT_DTYPE_BF16;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (img->product) {
    e = launch_product(dir == 0 ? img->pfwd : img->pinv, static_cast<const float *>(in),
                       static_cast<float *>(out), S, st, img->num_cus, img->grid[dir]);
  } else if (img->large) {
    const int mode = img->lmode[dir];
    const bool pooled = ws == nullptr && mode != 2;
    if (pooled && st != nullptr) {
      // a stream-ordered allocation would become part of a captured graph: refuse it
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return set_error(GFT_ERR_UNSUPPORTED,
                         "this plan's large-signal form takes a workspace per call, which is not "
                         "allocated under stream capture; use gft_apply_noalloc (static scratch) "
                         "or a plan whose large form is the one-pass form");
    }
    if (pooled) {
      e = hipMallocAsync(&ws, large_ws_bytes(img->lg[dir], mode, S), st);
      if (e != hipSuccess) return set_error(GFT_ERR_OOM, "hipMallocAsync of the large-signal workspace failed");
    }
    e = launch_large(plan, img, dir, in, out, S, st, ws, mode, img->ltile_kb[dir], img->op_grid[dir]);
    if (pooled) {
      const hipError_t ef = hipFreeAsync(ws, st);
      if (e == hipSuccess) e = ef;
    }
  } else if (img->butterfly) {
    e = launch_butterfly(dir == 0 ? img->bfwd : img->binv, in, out, S, st, img->num_cus, in16, out16,
                         img->grid[dir]);
  } else {
    const DevProgram &P = dir == 0 ? img->fwd[0] : img->inv[0];
    const int cap = dir == 0 ? img->grid_cap_fwd[0] : img->grid_cap_inv[0];
    e = launch_apply(P, in, out, S, st, cap, in16, out16);
  }
  if (e != hipSuccess) return set_error(GFT_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return ok();
}

gft_status apply(gft_plan_t plan, int dir, const void *in, void *out, int64_t S, void *stream) {
  gft_status st = check_apply_args(plan, in, out, S, dir);
  if (st != GFT_OK || S == 0) return st != GFT_OK ? st : ok();
  DeviceImage *img = nullptr;
  st = device_image(plan, &img);
  if (st != GFT_OK) return st;
  return launch_image(plan, img, dir, in, out, S, stream, nullptr);
}

// FP64 fast basis of a graph plan: U[i * n + k] is node i of basis vector k (column k is the
// inverse transform of the unit coefficient vector e_k, run block-locally).
std::vector<double> plan_basis(const GraphPlan &g) {
  const int n = g.n;
  std::vector<double> U((size_t)n * n, 0.0), e(n, 0.0), col(n);
  for (int k = 0; k < n; ++k) {
    e[k] = 1.0;
    apply_host(g, 1, e.data(), col.data(), 1);
    e[k] = 0.0;
    for (int i = 0; i < n; ++i) U[(size_t)i * n + k] = col[i];
  }
  return U;
}

// FP64 separable application of a product plan: forward y_k = (U_a^T X U_b)[p][q] with
// (p, q) = order[k]; inverse X = U_a Y U_b^T.
void product_apply_host(const gft_plan_s &P, int direction, const double *x, double *y, int64_t S) {
  const int na = P.fa.n, nb = P.fb.n, n = na * nb;
  std::vector<double> Z((size_t)n), T((size_t)n);
  for (int64_t s = 0; s < S; ++s) {
    const double *in = x + s * n;
    double *out = y + s * n;
    if (direction == 0) {
      for (int p = 0; p < na; ++p)                       // T = U_a^T X
        for (int j = 0; j < nb; ++j) {
          double acc = 0.0;
          for (int i = 0; i < na; ++i) acc += P.ua[(size_t)i * na + p] * in[(size_t)i * nb + j];
          T[(size_t)p * nb + j] = acc;
        }
      for (int p = 0; p < na; ++p)                       // Z = T U_b
        for (int q = 0; q < nb; ++q) {
          double acc = 0.0;
          for (int j = 0; j < nb; ++j) acc += T[(size_t)p * nb + j] * P.ub[(size_t)j * nb + q];
          Z[(size_t)p * nb + q] = acc;
        }
      for (int k = 0; k < n; ++k) out[k] = Z[P.order[k]];
    } else {
      for (int k = 0; k < n; ++k) Z[P.order[k]] = in[k];
      for (int i = 0; i < na; ++i)                       // T = U_a Y
        for (int q = 0; q < nb; ++q) {
          double acc = 0.0;
          for (int p = 0; p < na; ++p) acc += P.ua[(size_t)i * na + p] * Z[(size_t)p * nb + q];
          T[(size_t)i * nb + q] = acc;
        }
      for (int i = 0; i < na; ++i)                       // X = T U_b^T
        for (int j = 0; j < nb; ++j) {
          double acc = 0.0;
          for (int q = 0; q < nb; ++q) acc += T[(size_t)i * nb + q] * P.ub[(size_t)j * nb + q];
          out[(size_t)i * nb + j] = acc;
        }
    }
  }
}

// Signals wider than a generic-engine tile run on the large-signal engine only, whose rows
// (input and block-padded workspace) must fit one workgroup's LDS: reject at planning what
// no engine can run.
constexpr int kWideSignal = 2560;   // no 16-signal FP32 tile of wider signals fits 160 KB

gft_status check_runnable(const GraphPlan &g) {
  if (g.n <= kWideSignal) return GFT_OK;
  const int64_t cols = large_workspace_cols(g);
  if (g.n > kLargeMaxCols || cols > kLargeMaxCols)
    return set_error(GFT_ERR_UNSUPPORTED,
                     "n = " + std::to_string(g.n) + " with " + std::to_string(cols) +
                         " block-padded workspace columns: no engine takes signals of more than " +
                         std::to_string(kWideSignal) + " values whose rows exceed " +
                         std::to_string(kLargeMaxCols) + " columns (one FP32 row in LDS)");
  return GFT_OK;
}

gft_status get_graph(gft_plan_t plan, int32_t index, const GraphPlan **g) {
  if (!plan) return set_error(GFT_ERR_INVALID_ARG, "plan is NULL");
  if (index < 0 || index >= (int32_t)plan->graphs.size())
    return set_error(GFT_ERR_INVALID_ARG, "graph index out of range");
  *g = &plan->graphs[index];
  return GFT_OK;
}

}  // namespace

extern "C" {

gft_status gft_plan(const gft_graph *graph, const gft_pairing *pairing, const gft_options *opts,
                    gft_plan_t *out) {
  if (!out) return set_error(GFT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!graph) return set_error(GFT_ERR_INVALID_ARG, "graph is NULL");
  const gft_options o = default_options(opts);
  gft_status st = check_options(o);
  if (st != GFT_OK) return st;
  try {
    auto p = std::make_unique<gft_plan_s>();
    p->opts = o;
    p->graphs.push_back(build_graph_plan(*graph, pairing, o));
    if (const KronPlan *K = p->graphs[0].kron.get()) {
      p->kua = plan_basis(*K->fa);
      p->kub = plan_basis(*K->fb);
    } else {
      st = check_runnable(p->graphs[0]);
      if (st != GFT_OK) return st;
    }
    *out = p.release();
  } catch (const PlanError &err) {
    return set_error(err.status, err.message);
  } catch (const std::bad_alloc &) {
    return set_error(GFT_ERR_OOM, "host allocation failed while planning");
  } catch (const std::exception &ex) {
    return set_error(GFT_ERR_INVALID_ARG, ex.what());
  }
  return ok();
}

gft_status gft_find_pairing(const gft_graph *graph, const gft_options *opts, int32_t max_stages,
                            int64_t max_steps, int32_t *phi, int32_t *num_stages) {
  if (!graph || !phi || !num_stages)
    return set_error(GFT_ERR_INVALID_ARG, "graph, phi and num_stages must be non-NULL");
  if (max_stages < 0) return set_error(GFT_ERR_INVALID_ARG, "max_stages must be >= 0");
  *num_stages = 0;
  const gft_options o = default_options(opts);
  gft_status st = check_options(o);
  if (st != GFT_OK) return st;
  try {
    std::vector<int32_t> found;
    const int k = find_pairing(*graph, o, max_stages, max_steps > 0 ? max_steps : 200000, found);
    std::copy(found.begin(), found.end(), phi);
    *num_stages = k;
  } catch (const PlanError &err) {
    return set_error(err.status, err.message);
  } catch (const std::bad_alloc &) {
    return set_error(GFT_ERR_OOM, "host allocation failed while searching");
  }
  return ok();
}

gft_status gft_plan_batch(int32_t num_graphs, const gft_graph *graphs, const gft_pairing *pairings,
                          const gft_options *opts, gft_plan_t *out) {
  if (!out) return set_error(GFT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (num_graphs <= 0 || !graphs) return set_error(GFT_ERR_INVALID_ARG, "need num_graphs > 0 and graphs");
  const gft_options o = default_options(opts);
  gft_status st = check_options(o);
  if (st != GFT_OK) return st;
  if (o.in_dtype != o.out_dtype)
    return set_error(GFT_ERR_UNSUPPORTED, "batch plans store signals and coefficients in one type (FP32 or BF16)");
  try {
    auto p = std::make_unique<gft_plan_s>();
    p->opts = o;
    p->batch = true;
    for (int32_t g = 0; g < num_graphs; ++g) {
      try {
        p->graphs.push_back(build_graph_plan(graphs[g], pairings ? &pairings[g] : nullptr, o));
      } catch (const PlanError &err) {
        return set_error(err.status, "graph " + std::to_string(g) + ": " + err.message);
      }
    }
    *out = p.release();
  } catch (const std::bad_alloc &) {
    return set_error(GFT_ERR_OOM, "host allocation failed while planning");
  }
  return ok();
}

gft_status gft_plan_product(const gft_graph *graph_a, const gft_pairing *pairing_a,
                            const gft_graph *graph_b, const gft_pairing *pairing_b,
                            const gft_options *opts, gft_plan_t *out) {
  if (!out) return set_error(GFT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!graph_a || !graph_b) return set_error(GFT_ERR_INVALID_ARG, "graph_a and graph_b must be non-NULL");
  const gft_options o = default_options(opts);
  gft_status st = check_options(o);
  if (st != GFT_OK) return st;
  if (o.precision != GFT_FP32 && o.precision != GFT_BF16 && o.precision != GFT_SPLIT_BF16)
    return set_error(GFT_ERR_UNSUPPORTED, "product plans run FP32, BF16 or split BF16 factor products");
  if (o.in_dtype != o.out_dtype)
    return set_error(GFT_ERR_UNSUPPORTED, "product plans store signals and coefficients in one type (FP32 or BF16)");
  // The normalized Laplacian D^{-1/2} L D^{-1/2} of a product is a Kronecker sum only when
  // the degree d_a(i) + d_b(j) is constant, i.e. both factors are regular: then it is
  // L / (d_a + d_b), with the combinatorial product's basis and its eigenvalues scaled.
  double norm_scale = 1.0;
  if (o.laplacian == GFT_LAPLACIAN_NORMALIZED) {
    auto regular_degree = [](const gft_graph &g, double &deg) {
      std::vector<double> d(g.n, 0.0);
      for (int32_t e = 0; e < g.num_edges; ++e) {
        d[g.src[e]] += g.weight[e];
        d[g.dst[e]] += g.weight[e];
      }
      deg = d.empty() ? 0.0 : d[0];
      for (double x : d)
        if (std::fabs(x - deg) > 1e-12 * std::max(1.0, std::fabs(deg))) return false;
      return true;
    };
    double da = 0.0, db = 0.0;
    if (graph_a->n <= 0 || graph_b->n <= 0 || (graph_a->num_edges > 0 && (!graph_a->src || !graph_a->dst || !graph_a->weight)) ||
        (graph_b->num_edges > 0 && (!graph_b->src || !graph_b->dst || !graph_b->weight)))
      return set_error(GFT_ERR_INVALID_ARG, "graph_a and graph_b need n > 0 and their edge arrays");
    for (int32_t e = 0; e < graph_a->num_edges; ++e)
      if (graph_a->src[e] < 0 || graph_a->src[e] >= graph_a->n || graph_a->dst[e] < 0 || graph_a->dst[e] >= graph_a->n)
        return set_error(GFT_ERR_GRAPH, "graph_a: an edge has a label outside [0, n)");
    for (int32_t e = 0; e < graph_b->num_edges; ++e)
      if (graph_b->src[e] < 0 || graph_b->src[e] >= graph_b->n || graph_b->dst[e] < 0 || graph_b->dst[e] >= graph_b->n)
        return set_error(GFT_ERR_GRAPH, "graph_b: an edge has a label outside [0, n)");
    if (!regular_degree(*graph_a, da) || !regular_degree(*graph_b, db) || !(da + db > 0.0))
      return set_error(GFT_ERR_UNSUPPORTED,
                       "the normalized Laplacian of a product graph is a Kronecker sum only when both "
                       "factors are regular (constant weighted degree)");
    norm_scale = 1.0 / (da + db);
  }
  if (o.engine != GFT_ENGINE_AUTO)
    return set_error(GFT_ERR_UNSUPPORTED, "product plans run their own engine (options.engine must be 0)");
  gft_options of = o;   // factors: combinatorial (the normalized product is scaled below)
  of.laplacian = GFT_LAPLACIAN_COMBINATORIAL;
  try {
    auto p = std::make_unique<gft_plan_s>();
    p->opts = o;
    p->product = true;
    try {
      p->fa = build_graph_plan(*graph_a, pairing_a, of);
    } catch (const PlanError &err) {
      return set_error(err.status, "graph_a: " + err.message);
    }
    try {
      p->fb = build_graph_plan(*graph_b, pairing_b, of);
    } catch (const PlanError &err) {
      return set_error(err.status, "graph_b: " + err.message);
    }
    const int na = p->fa.n, nb = p->fb.n, n = na * nb;
    if (na > 64 || nb > 64)
      return set_error(GFT_ERR_UNSUPPORTED, "product plans take factors of at most 64 nodes");
    p->ua = plan_basis(p->fa);
    p->ub = plan_basis(p->fb);
    // eigenvalue of basis vector (p, q): lambda_p + mu_q; output order ascending (ties by p,
    // then q) or, with GFT_ORDER_BLOCK, (p, q) in row-major order
    std::vector<double> lam((size_t)n);
    for (int a = 0; a < na; ++a)
      for (int b = 0; b < nb; ++b) lam[(size_t)a * nb + b] = p->fa.lambda_out[a] + p->fb.lambda_out[b];
    p->order.resize(n);
    for (int k = 0; k < n; ++k) p->order[k] = k;
    if (o.order == GFT_ORDER_EIGENVALUE)
      std::stable_sort(p->order.begin(), p->order.end(),
                       [&](int32_t u, int32_t v) { return lam[u] < lam[v]; });
    GraphPlan g;
    g.n = n;
    g.lambda_out.resize(n);
    for (int k = 0; k < n; ++k) g.lambda_out[k] = norm_scale * lam[p->order[k]];
    g.stats.n = n;
    g.stats.num_blocks = 2;                 // the two factor GFTs, applied as dense matrices
    g.stats.max_block = std::max(na, nb);
    g.stats.mults = (int64_t)n * (na + nb);
    g.stats.adds = (int64_t)n * (na - 1 + nb - 1);
    g.stats.max_residual = std::max(p->fa.stats.max_residual, p->fb.stats.max_residual);
    g.stats.max_orth_error = std::max(p->fa.stats.max_orth_error, p->fb.stats.max_orth_error);
    p->graphs.push_back(std::move(g));
    *out = p.release();
  } catch (const std::bad_alloc &) {
    return set_error(GFT_ERR_OOM, "host allocation failed while planning");
  }
  return ok();
}

gft_status gft_forward(gft_plan_t plan, const void *x, void *y, int64_t num_signals, void *stream) {
  return apply(plan, 0, x, y, num_signals, stream);
}

gft_status gft_inverse(gft_plan_t plan, const void *y, void *x, int64_t num_signals, void *stream) {
  return apply(plan, 1, y, x, num_signals, stream);
}

static gft_status apply_batch(gft_plan_t plan, int dir, const void *in, void *out,
                              const int64_t *signal_offsets, int64_t total_elements, void *stream) {
  if (!plan) return set_error(GFT_ERR_INVALID_ARG, "plan is NULL");
  if (!plan->batch) return set_error(GFT_ERR_INVALID_ARG, "single-graph plans use gft_forward / gft_inverse");
  if (total_elements < 0) return set_error(GFT_ERR_INVALID_ARG, "total_elements must be >= 0");
  if (total_elements == 0) return ok();
  if (!signal_offsets) return set_error(GFT_ERR_INVALID_ARG, "signal_offsets is NULL");
  if (total_elements > (int64_t(1) << 40)) return set_error(GFT_ERR_INVALID_ARG, "total_elements too large");
  const bool io16 = plan->opts.in_dtype == GFT_DTYPE_BF16;   // signals and coefficients alike
  const int64_t esz = io16 ? 2 : 4;
  gft_status st = check_buffers(in, total_elements * esz, out, total_elements * esz, true);
  if (st != GFT_OK) return st;
  DeviceImage *img = nullptr;
  st = device_image(plan, &img);
  if (st != GFT_OK) return st;
  hipError_t e = launch_apply_batch(plan->opts.precision, dir, io16, dir == 0 ? img->dev_fwd : img->dev_inv,
                                    dir == 0 ? img->dev_ufwd : img->dev_uinv,
                                    (int)plan->graphs.size(), signal_offsets, total_elements, in, out,
                                    img->batch_lds, img->batch_rounds * img->num_cus * img->batch_occ,
                                    img->reg_groups, img->batch_cost16,
                                    static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return set_error(GFT_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return ok();
}

gft_status gft_apply_noalloc(gft_plan_t plan, int32_t direction, const void *in, void *out,
                             int64_t num_signals, void *stream) {
  if (direction != 0 && direction != 1) return set_error(GFT_ERR_INVALID_ARG, "direction must be 0 or 1");
  gft_status st = check_apply_args(plan, in, out, num_signals, direction);
  if (st != GFT_OK || num_signals == 0) return st != GFT_OK ? st : ok();
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(GFT_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  DeviceImage *img = nullptr;
  {
    std::lock_guard<std::mutex> lock(plan->mu);
    auto it = plan->images.find(dev);
    if (it != plan->images.end()) img = it->second.get();
  }
  if (!img)
    return set_error(GFT_ERR_INVALID_ARG,
                     "the plan has no image on the current device: call gft_plan_prepare there first "
                     "(building the image allocates device memory)");
  void *ws = nullptr;
  if (img->large) {
    ws = large_scratch(dev);
    if (!ws) return set_error(GFT_ERR_HIP, "the static scratch of this device was not set up");
    const size_t need = large_ws_bytes(img->lg[direction], img->lmode[direction], num_signals);
    if (need > kScratchBytes) {
      const size_t per = large_ws_bytes(img->lg[direction], img->lmode[direction], 1);
      return set_error(GFT_ERR_INVALID_ARG,
                       std::to_string(num_signals) + " signals need " + std::to_string(need) +
                           " bytes of workspace; the static scratch holds " + std::to_string(kScratchBytes) +
                           " bytes: at most " + std::to_string(kScratchBytes / per) +
                           " signals per call on this plan");
    }
  }
  return launch_image(plan, img, direction, in, out, num_signals, stream, ws);
}

gft_status gft_forward_batch(gft_plan_t plan, const void *x, void *y, const int64_t *signal_offsets,
                             int64_t total_elements, void *stream) {
  return apply_batch(plan, 0, x, y, signal_offsets, total_elements, stream);
}

gft_status gft_inverse_batch(gft_plan_t plan, const void *y, void *x, const int64_t *signal_offsets,
                             int64_t total_elements, void *stream) {
  return apply_batch(plan, 1, y, x, signal_offsets, total_elements, stream);
}

gft_status gft_plan_prepare(gft_plan_t plan) {
  if (!plan) return set_error(GFT_ERR_INVALID_ARG, "plan is NULL");
  DeviceImage *img = nullptr;
  gft_status st = device_image(plan, &img);
  return st != GFT_OK ? st : ok();
}

gft_status gft_plan_engine(gft_plan_t plan, int32_t *engine_out) {
  if (!plan || !engine_out) return set_error(GFT_ERR_INVALID_ARG, "plan and engine_out must be non-NULL");
  DeviceImage *img = nullptr;
  gft_status st = device_image(plan, &img);
  if (st != GFT_OK) return st;
  *engine_out = img->product ? GFT_ENGINE_PRODUCT
                : img->butterfly ? GFT_ENGINE_BUTTERFLY : (img->large ? GFT_ENGINE_LARGE : GFT_ENGINE_GENERIC);
  return ok();
}

gft_status gft_plan_tiles(gft_plan_t plan, int32_t *fwd_tile, int32_t *inv_tile) {
  if (!plan || !fwd_tile || !inv_tile) return set_error(GFT_ERR_INVALID_ARG, "plan and outputs must be non-NULL");
  if (plan->batch) return set_error(GFT_ERR_INVALID_ARG, "batch plans keep one tile per graph");
  DeviceImage *img = nullptr;
  gft_status st = device_image(plan, &img);
  if (st != GFT_OK) return st;
  if (img->product) {
    *fwd_tile = *inv_tile = 1;
  } else if (img->butterfly) {
    *fwd_tile = *inv_tile = 16;
  } else if (img->large) {
    *fwd_tile = *inv_tile = 0;
  } else {
    *fwd_tile = 16 * img->fwd[0].mt;
    *inv_tile = 16 * img->inv[0].mt;
  }
  return ok();
}

gft_status gft_plan_tuning(gft_plan_t plan, gft_tuning *out) {
  if (!plan || !out) return set_error(GFT_ERR_INVALID_ARG, "plan and out must be non-NULL");
  DeviceImage *img = nullptr;
  gft_status st = device_image(plan, &img);
  if (st != GFT_OK) return st;
  gft_tuning t{};
  t.engine = img->product ? GFT_ENGINE_PRODUCT
             : img->butterfly ? GFT_ENGINE_BUTTERFLY : (img->large ? GFT_ENGINE_LARGE : GFT_ENGINE_GENERIC);
  if (img->product) {
    t.fwd_tile = t.inv_tile = 1;
    t.variant = img->product_staged ? 1 : 0;
    t.grid_fwd = img->grid[0];
    t.grid_inv = img->grid[1];
  } else if (img->butterfly) {
    t.fwd_tile = t.inv_tile = 16;
    t.grid_fwd = img->grid[0];
    t.grid_inv = img->grid[1];
  } else if (img->large) {
    t.variant = img->lmode[0];
    t.large_tile_kb = img->ltile_kb[0];
    t.grid_fwd = img->op_grid[0];
    t.grid_inv = img->op_grid[1];
    t.onepass_fwd = img->op_ok[0] ? img->op[0].src_mode : 0;
    t.onepass_inv = img->op_ok[1] ? img->op[1].src_mode : 0;
  } else if (!plan->batch) {
    t.fwd_tile = 16 * img->fwd[0].mt;
    t.inv_tile = 16 * img->inv[0].mt;
  }
  if (plan->batch) {
    t.batch_rounds = img->batch_rounds;
    t.batch_cost16 = img->batch_cost16;
  }
  t.source = img->tune_source;
  t.tune_ms = img->tune_ms;
  *out = t;
  return ok();
}

gft_status gft_plan_info(gft_plan_t plan, int32_t index, gft_plan_stats *out) {
  const GraphPlan *g = nullptr;
  gft_status st = get_graph(plan, index, &g);
  if (st != GFT_OK) return st;
  if (!out) return set_error(GFT_ERR_INVALID_ARG, "out is NULL");
  *out = g->stats;
  return ok();
}

gft_status gft_plan_num_graphs(gft_plan_t plan, int32_t *out) {
  if (!plan || !out) return set_error(GFT_ERR_INVALID_ARG, "plan and out must be non-NULL");
  *out = (int32_t)plan->graphs.size();
  return ok();
}

gft_status gft_plan_size(gft_plan_t plan, int32_t index, int32_t *n_out) {
  const GraphPlan *g = nullptr;
  gft_status st = get_graph(plan, index, &g);
  if (st != GFT_OK) return st;
  if (!n_out) return set_error(GFT_ERR_INVALID_ARG, "n_out is NULL");
  *n_out = g->n;
  return ok();
}

gft_status gft_plan_eigenvalues(gft_plan_t plan, int32_t index, double *lambda) {
  const GraphPlan *g = nullptr;
  gft_status st = get_graph(plan, index, &g);
  if (st != GFT_OK) return st;
  if (!lambda) return set_error(GFT_ERR_INVALID_ARG, "lambda is NULL");
  std::memcpy(lambda, g->lambda_out.data(), sizeof(double) * g->n);
  return ok();
}

gft_status gft_plan_basis(gft_plan_t plan, int32_t index, double *U) {
  const GraphPlan *g = nullptr;
  gft_status st = get_graph(plan, index, &g);
  if (st != GFT_OK) return st;
  if (!U) return set_error(GFT_ERR_INVALID_ARG, "U is NULL");
  const int n = g->n;
  if (plan->product) {
    // node (i, j) of basis vector k = (p, q): U_a[i][p] U_b[j][q]
    const int na = plan->fa.n, nb = plan->fb.n;
    for (int i = 0; i < na; ++i)
      for (int j = 0; j < nb; ++j)
        for (int k = 0; k < n; ++k) {
          const int p = plan->order[k] / nb, q = plan->order[k] % nb;
          U[((size_t)i * nb + j) * n + k] = plan->ua[(size_t)i * na + p] * plan->ub[(size_t)j * nb + q];
        }
    return ok();
  }
  const std::vector<double> B = plan_basis(*g);
  std::memcpy(U, B.data(), sizeof(double) * B.size());
  return ok();
}

gft_status gft_plan_apply_host(gft_plan_t plan, int32_t index, int32_t direction, const double *x,
                               double *y, int64_t num_signals) {
  const GraphPlan *g = nullptr;
  gft_status st = get_graph(plan, index, &g);
  if (st != GFT_OK) return st;
  if (direction != 0 && direction != 1) return set_error(GFT_ERR_INVALID_ARG, "direction must be 0 or 1");
  if (num_signals < 0) return set_error(GFT_ERR_INVALID_ARG, "num_signals must be >= 0");
  if (num_signals > 0 && (!x || !y)) return set_error(GFT_ERR_INVALID_ARG, "x and y must be non-NULL");
  if (plan->product) product_apply_host(*plan, direction, x, y, num_signals);
  else apply_host(*g, direction, x, y, num_signals);
  return ok();
}

gft_status gft_plan_blocks(gft_plan_t plan, int32_t index, int32_t *sizes, int32_t *nodes) {
  const GraphPlan *g = nullptr;
  gft_status st = get_graph(plan, index, &g);
  if (st != GFT_OK) return st;
  if (!sizes) return set_error(GFT_ERR_INVALID_ARG, "sizes is NULL");
  if (plan->product)
    return set_error(GFT_ERR_UNSUPPORTED, "product plans have no leaf blocks (two factor GFTs)");
  size_t pos = 0;
  for (size_t b = 0; b < g->blocks.size(); ++b) {
    sizes[b] = g->blocks[b].size;
    if (nodes)
      for (int32_t v : g->blocks[b].nodes) nodes[pos++] = v;
  }
  return ok();
}

gft_status gft_plan_destroy(gft_plan_t plan) {
  delete plan;
  return ok();
}

const char *gft_last_error(void) { return g_last_error.c_str(); }

gft_status gft_stream_copy(const void *src, void *dst, int64_t bytes, void *stream) {
  if (bytes < 0 || (bytes & 15)) return set_error(GFT_ERR_INVALID_ARG, "bytes must be a non-negative multiple of 16");
  if (bytes == 0) return ok();
  if (!src || !dst) return set_error(GFT_ERR_INVALID_ARG, "src and dst must be non-NULL device pointers");
  const uintptr_t ps = reinterpret_cast<uintptr_t>(src), pd = reinterpret_cast<uintptr_t>(dst);
  if ((ps & 15) || (pd & 15)) return set_error(GFT_ERR_ALIGNMENT, "src and dst must be 16-byte aligned");
  if (ps < pd + (uintptr_t)bytes && pd < ps + (uintptr_t)bytes)
    return set_error(GFT_ERR_ALIGNMENT, "src and dst overlap");
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return set_error(GFT_ERR_HIP, std::string("device query: ") + hipGetErrorString(e));
  e = launch_stream_copy(src, dst, bytes, static_cast<hipStream_t>(stream), cus);
  if (e != hipSuccess) return set_error(GFT_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return ok();
}

const char *gft_version(void) { return "libgft 0.1 (gfx950)"; }

}  // extern "C"
