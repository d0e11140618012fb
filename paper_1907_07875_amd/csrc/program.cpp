// Plan -> device program (host side).
#include "program.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>

namespace gft {

uint16_t to_bf16_bits(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

uint16_t to_f16_bits(float x) {
  // IEEE binary16, round to nearest even (finite inputs of block matrices: |x| <= 1)
  uint32_t u;
  std::memcpy(&u, &x, 4);
  const uint32_t sign = (u >> 16) & 0x8000u;
  const int exp = (int)((u >> 23) & 0xff) - 127 + 15;
  uint32_t mant = u & 0x7fffffu;
  if (((u >> 23) & 0xff) == 0xff) return (uint16_t)(sign | 0x7c00u | (mant ? 0x200u : 0u));
  if (exp >= 31) return (uint16_t)(sign | 0x7c00u);
  if (exp <= 0) {  // subnormal half (or zero)
    if (exp < -10) return (uint16_t)sign;
    mant |= 0x800000u;
    const int shift = 14 - exp;
    uint32_t h = mant >> shift;
    const uint32_t rem = mant & ((1u << shift) - 1), half = 1u << (shift - 1);
    if (rem > half || (rem == half && (h & 1u))) ++h;
    return (uint16_t)(sign | h);
  }
  uint32_t h = ((uint32_t)exp << 10) | (mant >> 13);
  const uint32_t rem = mant & 0x1fffu;
  if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) ++h;
  return (uint16_t)(sign | h);
}

namespace {

float bf16_to_float(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

uint32_t magic_for(uint32_t d) {
  // ceil(2^32 / d): floor(e * magic / 2^32) == e / d whenever e * d < 2^32.
  // d == 1 is encoded as 0 (the kernels divide by 1 directly).
  return d <= 1 ? 0u : (uint32_t)((((uint64_t)1 << 32) + d - 1) / d);
}

}  // namespace

size_t program_lds_bytes(const DevProgram &P) {
  const size_t T = 16 * (size_t)P.mt;
  const size_t frag = P.frag_lds ? 4 * (size_t)((P.frag_words + 3) & ~3) : 0;
  return 4 * (size_t)((P.table_words + 3) & ~3) + frag + 2 * T * (size_t)P.stride * 4;
}

bool build_program(const GraphPlan &p, int direction, int tile_override, size_t lds_budget,
                   ProgramImage &out, int precision) {
  const int n = p.n;
  DevProgram &P = out.prog;
  P = DevProgram{};
  P.n = n;
  // Odd n: rows packed (stride n), so the tile is the signals' own contiguous layout.
  // n a multiple of 4: stride n + 4 keeps every row 16-byte aligned.  Either way a
  // float4 of the signal array is one aligned 16-byte LDS access.  Otherwise n + 1.
  P.stride = (n % 2) ? n : ((n % 4 == 0) ? n + 4 : n + 1);
  P.magic_n = magic_for((uint32_t)n);

  std::vector<int32_t> stages, ops, blocks, items, gidx, sidx;
  std::vector<uint32_t> &frag = out.frag;
  frag.clear();
  P.prec = precision;
  const int KS = precision == GFT_FP32 ? 4 : 16;                  // K per MFMA
  const int WPL = precision == GFT_FP32 ? 1 : (precision == GFT_SPLIT_BF16 ? 4 : 2);

  // Haar stages.  Forward: left stages in plan order before the blocks (node positions),
  // the right stage after them (output positions).  Inverse: the right stage before the
  // blocks, the left stages in reverse order after them.
  auto emit = [&](const HostStage &st) {
    const int off = (int)(ops.size() / 2);
    for (size_t u = 0; u < st.pair_x.size(); ++u) {
      ops.push_back(st.pair_x[u]);
      ops.push_back(st.pair_y[u]);
    }
    for (int32_t c : st.znodes) {
      ops.push_back(c);
      ops.push_back(-1);
    }
    const int cnt = (int)(ops.size() / 2) - off;
    stages.push_back(off);
    stages.push_back(cnt);
    stages.push_back((int32_t)magic_for((uint32_t)std::max(cnt, 1)));
    stages.push_back(0);
  };
  const int ns = (int)p.stages.size();
  const int nr = p.right.pair_x.empty() ? 0 : 1;
  if (direction == 0) {
    for (int q = 0; q < ns; ++q) emit(p.stages[q]);
    if (nr) emit(p.right);
    P.num_pre = ns;
    P.num_post = nr;
  } else {
    if (nr) emit(p.right);
    for (int q = ns - 1; q >= 0; --q) emit(p.stages[q]);
    P.num_pre = nr;
    P.num_post = ns;
  }
  P.total_ops = (int32_t)(ops.size() / 2);

  // Blocks.  Forward: K = block nodes (gather node columns), N = eigenvectors (scatter to
  // output positions), M[j][k] = scale * V[j][k].  Inverse: K = output positions, N = nodes,
  // M[k][j] = scale * V[j][k].
  // Leaf blocks of at most 16 nodes are packed, first fit by decreasing size, into device
  // blocks of at most 16 whose matrix is block diagonal: one 16-column MFMA tile then
  // serves several small blocks (the zero off-diagonal entries add exact zeros).
  std::vector<std::vector<int>> groups;
  {
    std::vector<int> order(p.blocks.size());
    for (size_t b = 0; b < order.size(); ++b) order[b] = (int)b;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return p.blocks[a].size > p.blocks[c].size; });
    std::vector<int> fill;
    for (int b : order) {
      const int sz = p.blocks[b].size;
      int dst = -1;
      if (sz <= 16)
        for (size_t g = 0; g < groups.size(); ++g)
          if (fill[g] + sz <= 16 && fill[g] > 0 && p.blocks[groups[g][0]].size <= 16) {
            dst = (int)g;
            break;
          }
      if (dst < 0) {
        groups.push_back({});
        fill.push_back(0);
        dst = (int)groups.size() - 1;
      }
      groups[dst].push_back(b);
      fill[dst] += sz;
    }
  }
  for (int b = 0; b < (int)groups.size(); ++b) {
    // concatenated nodes / output positions, and the owning leaf block of each index
    std::vector<int32_t> knodes, kout;
    std::vector<const HostBlock *> owner;
    std::vector<int> local;
    for (int lb : groups[b]) {
      const HostBlock &L = p.blocks[lb];
      for (int k = 0; k < L.size; ++k) {
        knodes.push_back(L.nodes[k]);
        kout.push_back(L.out_pos[k]);
        owner.push_back(&L);
        local.push_back(k);
      }
    }
    const int sz = (int)knodes.size();
    const int kchunks = (sz + KS - 1) / KS;
    const int ntiles = (sz + 15) / 16;
    const int g_off = (int)gidx.size(), s_off = (int)sidx.size(), f_off = (int)frag.size();
    const std::vector<int32_t> &kin = direction == 0 ? knodes : kout;
    const std::vector<int32_t> &nout = direction == 0 ? kout : knodes;
    for (int k = 0; k < KS * kchunks; ++k) gidx.push_back(kin[k < sz ? k : 0]);
    for (int c = 0; c < sz; ++c) sidx.push_back(nout[c]);
    auto mat = [&](int k, int c) -> double {   // M[k][c] of this direction, zero padded
      if (k >= sz || c >= sz || owner[k] != owner[c]) return 0.0;
      const HostBlock &B = *owner[k];
      const int lk = local[k], lc = local[c], bs = B.size;
      return B.scale * (direction == 0 ? B.V[(size_t)lk * bs + lc] : B.V[(size_t)lc * bs + lk]);
    };
    frag.resize(frag.size() + (size_t)kchunks * ntiles * 64 * WPL, 0u);
    for (int kc = 0; kc < kchunks; ++kc)
      for (int nt = 0; nt < ntiles; ++nt)
        for (int lane = 0; lane < 64; ++lane) {
          uint32_t *w = &frag[f_off + (((size_t)kc * ntiles + nt) * 64 + lane) * WPL];
          const int c = 16 * nt + lane % 16;
          if (precision == GFT_FP32) {
            const float v = (float)mat(4 * kc + lane / 16, c);
            std::memcpy(w, &v, 4);
            continue;
          }
          uint16_t hi[4], lo[4];
          for (int j = 0; j < 4; ++j) {
            const double v = mat(16 * kc + 4 * (lane / 16) + j, c);
            if (precision == GFT_FP16) {
              hi[j] = to_f16_bits((float)v);
              lo[j] = 0;
            } else {
              hi[j] = to_bf16_bits((float)v);
              lo[j] = to_bf16_bits((float)(v - (double)bf16_to_float(hi[j])));
            }
          }
          w[0] = (uint32_t)hi[0] | ((uint32_t)hi[1] << 16);
          w[1] = (uint32_t)hi[2] | ((uint32_t)hi[3] << 16);
          if (precision == GFT_SPLIT_BF16) {
            w[2] = (uint32_t)lo[0] | ((uint32_t)lo[1] << 16);
            w[3] = (uint32_t)lo[2] | ((uint32_t)lo[3] << 16);
          }
        }
    blocks.insert(blocks.end(), {sz, kchunks, ntiles, g_off, s_off, f_off, 0, 0});
    for (int nt = 0; nt < ntiles; ++nt) items.push_back((b << 16) | nt);
  }
  // Largest blocks first so the waves of a workgroup finish together.
  std::stable_sort(items.begin(), items.end(), [&](int32_t a, int32_t c) {
    return blocks[8 * (a >> 16) + 1] > blocks[8 * (c >> 16) + 1];
  });
  P.num_blocks = (int32_t)groups.size();
  P.num_items = (int32_t)items.size();
  P.gidx_len = (int32_t)gidx.size();
  P.sidx_len = (int32_t)sidx.size();

  std::vector<int32_t> &t = out.table;
  t.clear();
  t.insert(t.end(), stages.begin(), stages.end());
  t.insert(t.end(), ops.begin(), ops.end());
  t.insert(t.end(), blocks.begin(), blocks.end());
  t.insert(t.end(), items.begin(), items.end());
  t.insert(t.end(), gidx.begin(), gidx.end());
  t.insert(t.end(), sidx.begin(), sidx.end());
  P.table_words = (int32_t)t.size();
  P.frag_words = (int32_t)frag.size();
  // Fragments live in LDS when they are small: read from global memory their waits would
  // also drain the in-flight prefetch of the next tile (the load counter is in order).
  P.frag_lds = frag.size() * 4 <= 16 * 1024 ? 1 : 0;

  if (tile_override > 0) {
    P.mt = tile_override / 16;
    if (P.mt != 1 && P.mt != 2 && P.mt != 4 && P.mt != 8) return false;
    return program_lds_bytes(P) <= lds_budget;
  }
  // Prefer tiles whose LDS footprint leaves room for several workgroups per CU (64 KB);
  // larger signals fall back to one M-tile within the full budget.
  for (int mt : {8, 4, 2, 1}) {
    P.mt = mt;
    if (program_lds_bytes(P) <= std::min<size_t>(lds_budget, 64 * 1024)) return true;
  }
  P.mt = 1;
  return program_lds_bytes(P) <= lds_budget;
}

}  // namespace gft

namespace gft {

// One-stage plans that are not uniform hypercubes (fixed nodes V_Z, blocks of unequal size
// or split into components, 8 <= n <= 96): orbit o holds the o-th V_X node (or, past
// the pairs, the V_Z nodes) in slot 0 and its partner in slot 1 (a zero word for V_Z and
// padding), so the register Haar gives the G+ input (x + x') and the G- input (x - x').  G+
// (V_X then V_Z positions) and G- (V_Y positions) are each one zero-padded block of M = 16, 32
// or 48 rows holding their leaf blocks on the diagonal; the sqrt 2 of a V_Z node is folded
// into its G+ row (the kernel's Haar adds a zero to it).  Slot 0 always holds the V_X node, so no
// sign flips.
static bool build_butterfly_one_stage(const GraphPlan &p, int direction, UProgramImage &out,
                                      int precision) {
  const int n = p.n;
  if (p.stages.size() != 1 || !p.right.pair_x.empty() || n < 8) return false;
  const HostStage &st = p.stages[0];
  const int P = (int)st.pair_x.size(), Z = (int)st.znodes.size();
  const int pp = P + Z;                        // |G+|
  const int wide = std::max(pp, P);
  const int M = wide <= 16 ? 16 : (wide <= 32 ? 32 : (wide <= 48 ? 48 : 0));
  if (M == 0 || 2 * P + Z != n) return false;
  std::vector<int> plus_node(pp), minus_node(P), side(n, -1), ppos(n, -1);
  for (int u = 0; u < P; ++u) {
    plus_node[u] = st.pair_x[u];
    minus_node[u] = st.pair_y[u];
  }
  for (int z = 0; z < Z; ++z) plus_node[P + z] = st.znodes[z];
  for (int o = 0; o < pp; ++o) {
    side[plus_node[o]] = 0;
    ppos[plus_node[o]] = o;
  }
  for (int o = 0; o < P; ++o) {
    side[minus_node[o]] = 1;
    ppos[minus_node[o]] = o;
  }
  for (int i = 0; i < n; ++i)
    if (side[i] < 0) return false;
  // super-block matrices Vs[b][o][c] (row = position o, column = output column c) and the
  // output position of each column
  std::vector<std::vector<double>> Vs(2, std::vector<double>((size_t)M * M, 0.0));
  std::vector<std::vector<int>> outp(2, std::vector<int>(M, -1));
  int ncol[2] = {0, 0};
  for (const HostBlock &B : p.blocks) {
    const int b = side[B.nodes[0]];
    for (int k = 0; k < B.size; ++k)
      if (side[B.nodes[k]] != b || B.depth != 1) return false;
    if (ncol[b] + B.size > M) return false;
    for (int k = 0; k < B.size; ++k) {
      const int o = ppos[B.nodes[k]];
      const double zs = (b == 0 && o >= P) ? std::sqrt(2.0) : 1.0;   // V_Z row
      for (int c = 0; c < B.size; ++c) Vs[b][(size_t)o * M + ncol[b] + c] = zs * B.scale * B.V[(size_t)k * B.size + c];
    }
    for (int c = 0; c < B.size; ++c) outp[b][ncol[b] + c] = B.out_pos[c];
    ncol[b] += B.size;
  }
  if (ncol[0] != pp || ncol[1] != P) return false;
  if (precision != GFT_FP32 && precision != GFT_BF16) return false;
  const bool bf = precision == GFT_BF16;
  const int NB = 2, KC = M / 4, NT = M / 16, Q = NB * M / 4;
  auto node_at = [&](int b, int o) { return b == 0 ? (o < pp ? plus_node[o] : -1) : (o < P ? minus_node[o] : -1); };
  // orbit in data register set kc of lane group g (BF16: 4 consecutive k per 16x16x16 MFMA)
  auto orbit = [&](int g, int kc) { return bf ? 16 * (kc / 4) + 4 * g + kc % 4 : 4 * kc + g; };
  UProgramImage im;
  im.prog.S = 1;
  im.prog.M = M;
  im.prog.n = n;
  im.prog.dir = direction;
  im.prog.prec = precision;
  im.prog.gen = 1;
  im.gcol.assign((size_t)4 * Q, -1);
  im.scol.assign((size_t)4 * Q, -1);
  im.flips.assign(8, 0);
  for (int g = 0; g < 4; ++g) {
    for (int kc = 0; kc < KC; ++kc)
      for (int b = 0; b < NB; ++b)
        im.gcol[(size_t)g * Q + kc * NB + b] = direction == 0 ? node_at(b, orbit(g, kc)) : outp[b][orbit(g, kc)];
    for (int nt = 0; nt < NT; ++nt)
      for (int v = 0; v < 4; ++v) {
        const int c = 16 * nt + 4 * g + v;
        for (int b = 0; b < NB; ++b) {
          if (direction == 0)
            im.scol[(size_t)g * Q + (b * NT + nt) * 4 + v] = outp[b][c];
          else
            im.scol[(size_t)g * Q + (nt * 4 + v) * NB + b] = node_at(b, c);
        }
      }
  }
  // forward: A[c][o] = Vs[o][c]; inverse: A[o][k] = Vs[o][k]
  auto aval = [&](int b, int row, int k) {
    const int o = direction == 0 ? k : row;
    const int c = direction == 0 ? row : k;
    return Vs[b][(size_t)o * M + c];
  };
  if (bf) {
    im.afrag.assign((size_t)NB * NT * (KC / 4) * 64 * 2, 0.0f);
    for (int b = 0; b < NB; ++b)
      for (int nt = 0; nt < NT; ++nt)
        for (int k4 = 0; k4 < KC / 4; ++k4)
          for (int lane = 0; lane < 64; ++lane) {
            const int row = 16 * nt + lane % 16, k0 = 16 * k4 + 4 * (lane / 16);
            uint32_t w[2];
            for (int h = 0; h < 2; ++h)
              w[h] = (uint32_t)to_bf16_bits((float)aval(b, row, k0 + 2 * h)) |
                     ((uint32_t)to_bf16_bits((float)aval(b, row, k0 + 2 * h + 1)) << 16);
            std::memcpy(&im.afrag[(((size_t)(b * NT + nt) * (KC / 4) + k4) * 64 + lane) * 2], w, 8);
          }
  } else {
    im.afrag.assign((size_t)NB * NT * KC * 64, 0.0f);
    for (int b = 0; b < NB; ++b)
      for (int nt = 0; nt < NT; ++nt)
        for (int kc = 0; kc < KC; ++kc)
          for (int lane = 0; lane < 64; ++lane)
            im.afrag[((size_t)(b * NT + nt) * KC + kc) * 64 + lane] =
                (float)aval(b, 16 * nt + lane % 16, 4 * kc + lane / 16);
  }
  out = std::move(im);
  return true;
}

// Two-stage plans that are not uniform hypercubes (odd or unequal grids under LR then UD,
// fixed nodes at either stage, leaves split into components), FP32 blocks.  An orbit is led
// by a node a of the first stage's sum side G+ (V_X1 or V_Z1) that is the V_X node or a
// fixed node of the second stage there: slot 0 = a, slot 1 = its second-stage partner a'
// in G+, slot 2 = phi1(a), slot 3 = phi1(a') (the first-stage partners, in G-), with empty
// slots where a node is fixed or absent (a zero word).  The kernel's stage 1 combines slots
// (0, 2) and (1, 3), stage 2 slots (0, 1) and (2, 3), so G-'s second-stage pairs must be
// exactly (phi1(a), phi1(a')), a sign flip orienting them (the difference belongs at
// G-'s V_X2 node).  A slot left empty before a stage receives a copy of its partner's
// value; the layout is accepted only where such copies meet other copies or empty slots,
// never a real value (checked per orbit).  The final slot b of an orbit is leaf block class
// b (++, +-, -+, --); every missing partner along a value's way (a fixed node) leaves out
// a factor sqrt 2, folded into that value's block row.
static bool build_butterfly_two_stage(const GraphPlan &p, int direction, UProgramImage &out) {
  const int n = p.n;
  if (p.stages.size() != 2 || !p.right.pair_x.empty() || n < 8) return false;
  const HostStage &s1 = p.stages[0], &s2 = p.stages[1];
  if ((int)(s2.pair_x.size() * 2 + s2.znodes.size()) != n) return false;   // both sides split
  if ((int)(s1.pair_x.size() * 2 + s1.znodes.size()) != n) return false;
  std::vector<int> phi1(n, -1), phi2(n, -1), is_x2(n, 0), side(n, -1), z1(n, 0), z2(n, 0);
  for (size_t u = 0; u < s1.pair_x.size(); ++u) {
    phi1[s1.pair_x[u]] = s1.pair_y[u];
    phi1[s1.pair_y[u]] = s1.pair_x[u];
    side[s1.pair_x[u]] = 0;
    side[s1.pair_y[u]] = 1;
  }
  for (int z : s1.znodes) {
    side[z] = 0;
    z1[z] = 1;
  }
  for (size_t u = 0; u < s2.pair_x.size(); ++u) {
    phi2[s2.pair_x[u]] = s2.pair_y[u];
    phi2[s2.pair_y[u]] = s2.pair_x[u];
    is_x2[s2.pair_x[u]] = 1;
  }
  for (int z : s2.znodes) z2[z] = 1;
  for (int i = 0; i < n; ++i)
    if (side[i] < 0 || (phi2[i] < 0 && !z2[i]) || (phi2[i] >= 0 && side[phi2[i]] != side[i])) return false;
  // orbits: slots {a, a', phi1(a), phi1(a')}, -1 empty
  std::vector<std::array<int, 4>> orb;
  std::vector<int> seen(n, 0);
  for (int a = 0; a < n; ++a) {
    if (side[a] != 0 || !(is_x2[a] || z2[a])) continue;
    std::array<int, 4> o{a, z2[a] ? -1 : phi2[a], -1, -1};
    if (!z1[a]) o[2] = phi1[a];
    if (o[1] >= 0 && !z1[o[1]]) o[3] = phi1[o[1]];
    // G-'s second-stage structure must match: a pair (phi1 a, phi1 a') or fixed nodes
    if (o[2] >= 0 && o[3] >= 0 && phi2[o[2]] != o[3]) return false;
    if (o[2] >= 0 && o[3] < 0 && !z2[o[2]]) return false;
    if (o[2] < 0 && o[3] >= 0) return false;
    // copies made by stage 1 (slot j empty-partner) must not meet real values at stage 2
    const bool e0 = o[0] < 0, e1 = o[1] < 0, e2 = o[2] < 0, e3 = o[3] < 0;
    if (e2 && !e0 && !e3) return false;
    if (e3 && !e1 && !e2) return false;
    for (int v : o)
      if (v >= 0) {
        if (seen[v]) return false;
        seen[v] = 1;
      }
    orb.push_back(o);
  }
  for (int i = 0; i < n; ++i)
    if (!seen[i]) return false;
  const int O = (int)orb.size();
  // final slot (leaf class) and orbit of every node's value after the two stages: slot 0
  // holds a's label, slot 1 a', slot 2 G-'s V_X2 (or fixed) node, slot 3 its V_Y2 node
  std::vector<int> fslot(n, -1), forb(n, -1), flip(O, 0);
  for (int o = 0; o < O; ++o) {
    const auto &v = orb[o];
    fslot[v[0]] = 0;
    forb[v[0]] = o;
    if (v[1] >= 0) {
      fslot[v[1]] = 1;
      forb[v[1]] = o;
    }
    if (v[2] >= 0) {
      const bool sw = v[3] >= 0 && !is_x2[v[2]];   // G-'s V_X2 node sits in slot 3
      flip[o] = sw;
      const int lx = sw ? v[3] : v[2], ly = sw ? v[2] : v[3];
      fslot[lx] = 2;
      forb[lx] = o;
      if (ly >= 0) {
        fslot[ly] = 3;
        forb[ly] = o;
      }
    }
  }
  // super-blocks: leaf blocks of class b packed by columns, rows = orbit positions
  int maxcol[4] = {0, 0, 0, 0};
  for (const HostBlock &B : p.blocks) {
    const int b = fslot[B.nodes[0]];
    for (int k = 0; k < B.size; ++k)
      if (fslot[B.nodes[k]] != b || B.depth != 2) return false;
    maxcol[b] += B.size;
  }
  const int wide = std::max(O, std::max(std::max(maxcol[0], maxcol[1]), std::max(maxcol[2], maxcol[3])));
  const int M = wide <= 16 ? 16 : (wide <= 32 ? 32 : 0);
  if (M == 0) return false;
  const int NB = 4, KC = M / 4, NT = M / 16, Q = NB * M / 4;
  std::vector<std::vector<double>> Vs(4, std::vector<double>((size_t)M * M, 0.0));
  std::vector<std::vector<int>> outp(4, std::vector<int>(M, -1));
  int ncol[4] = {0, 0, 0, 0};
  for (const HostBlock &B : p.blocks) {
    const int b = fslot[B.nodes[0]];
    for (int k = 0; k < B.size; ++k) {
      const int v = B.nodes[k];
      const double zs = (z1[v] && side[v] == 0 ? std::sqrt(2.0) : 1.0) * (z2[v] ? std::sqrt(2.0) : 1.0);
      for (int c = 0; c < B.size; ++c)
        Vs[b][(size_t)forb[v] * M + ncol[b] + c] = zs * B.scale * B.V[(size_t)k * B.size + c];
    }
    for (int c = 0; c < B.size; ++c) outp[b][ncol[b] + c] = B.out_pos[c];
    ncol[b] += B.size;
  }
  auto node_at = [&](int o, int b) { return o < O ? orb[o][b] : -1; };
  UProgramImage im;
  im.prog.S = 2;
  im.prog.M = M;
  im.prog.n = n;
  im.prog.dir = direction;
  im.prog.prec = GFT_FP32;
  im.prog.gen = 1;
  im.gcol.assign((size_t)4 * Q, -1);
  im.scol.assign((size_t)4 * Q, -1);
  im.flips.assign(8, 0);
  for (int g = 0; g < 4; ++g) {
    uint64_t fw = 0;
    for (int kc = 0; kc < KC; ++kc)
      for (int b = 0; b < NB; ++b)
        im.gcol[(size_t)g * Q + kc * NB + b] = direction == 0 ? node_at(4 * kc + g, b) : outp[b][4 * kc + g];
    for (int nt = 0; nt < NT; ++nt)
      for (int v = 0; v < 4; ++v) {
        const int c = 16 * nt + 4 * g + v;
        for (int b = 0; b < NB; ++b) {
          if (direction == 0)
            im.scol[(size_t)g * Q + (b * NT + nt) * 4 + v] = outp[b][c];
          else
            im.scol[(size_t)g * Q + (nt * 4 + v) * NB + b] = node_at(c, b);
        }
      }
    // flip bit of register set j, stage t = 1, lo-slot rank k = 1 (slots 2, 3): 4 j + 3;
    // j = kc (forward, orbit 4 kc + g) or nt * 4 + v (inverse, orbit 16 nt + 4 g + v)
    if (direction == 0) {
      for (int kc = 0; kc < KC; ++kc)
        if (4 * kc + g < O && flip[4 * kc + g]) fw |= 1ull << (4 * kc + 3);
    } else {
      for (int j = 0; j < NT * 4; ++j) {
        const int o = 16 * (j / 4) + 4 * g + j % 4;
        if (o < O && flip[o]) fw |= 1ull << (4 * j + 3);
      }
    }
    im.flips[2 * g] = (uint32_t)fw;
    im.flips[2 * g + 1] = (uint32_t)(fw >> 32);
  }
  auto aval = [&](int b, int row, int k) {
    const int o = direction == 0 ? k : row;
    const int c = direction == 0 ? row : k;
    return Vs[b][(size_t)o * M + c];
  };
  im.afrag.assign((size_t)NB * NT * KC * 64, 0.0f);
  for (int b = 0; b < NB; ++b)
    for (int nt = 0; nt < NT; ++nt)
      for (int kc = 0; kc < KC; ++kc)
        for (int lane = 0; lane < 64; ++lane)
          im.afrag[((size_t)(b * NT + nt) * KC + kc) * 64 + lane] = (float)aval(b, 16 * nt + lane % 16, 4 * kc + lane / 16);
  out = std::move(im);
  return true;
}

static bool build_butterfly_uniform(const GraphPlan &p, int direction, UProgramImage &out);

bool build_butterfly(const GraphPlan &p, int direction, UProgramImage &out, int precision) {
  // a uniform layout of a shape with no compiled kernel (e.g. two blocks of 48) falls
  // through to the padded layouts, which take every uniform one- and two-stage plan too
  UProgramImage u;
  if (precision == GFT_FP32 && build_butterfly_uniform(p, direction, u) &&
      butterfly_shape_compiled(u.prog.S, u.prog.M, false)) {
    out = std::move(u);
    return true;
  }
  if (build_butterfly_one_stage(p, direction, out, precision)) return true;
  return precision == GFT_FP32 && build_butterfly_two_stage(p, direction, out);
}

static bool build_butterfly_uniform(const GraphPlan &p, int direction, UProgramImage &out) {
  const int n = p.n;
  const int S = (int)p.stages.size();
  if (S < 1 || S > 3 || !p.right.pair_x.empty()) return false;
  const int NB = 1 << S;
  if ((int)p.blocks.size() != NB || n % NB) return false;
  const int M = n / NB;
  if (M % 16) return false;
  for (const HostBlock &B : p.blocks)
    if (B.size != M || B.depth != S) return false;
  for (const HostStage &st : p.stages)
    if (!st.znodes.empty() || (int)st.pair_x.size() * 2 != n) return false;

  // final slot of a node = its leaf block; bit S-1-t of it is the node's side at stage t
  std::vector<int> fslot(n, -1), pos(n, -1);
  for (int b = 0; b < NB; ++b)
    for (int k = 0; k < M; ++k) {
      fslot[p.blocks[b].nodes[k]] = b;
      pos[p.blocks[b].nodes[k]] = k;
    }
  std::vector<std::vector<int>> partner(S, std::vector<int>(n, -1));
  std::vector<std::vector<char>> isx(S, std::vector<char>(n, 0));
  for (int t = 0; t < S; ++t) {
    const HostStage &st = p.stages[t];
    for (size_t u = 0; u < st.pair_x.size(); ++u) {
      partner[t][st.pair_x[u]] = st.pair_y[u];
      partner[t][st.pair_y[u]] = st.pair_x[u];
      isx[t][st.pair_x[u]] = 1;
    }
    for (int i = 0; i < n; ++i)
      if (partner[t][i] < 0 || ((fslot[i] >> (S - 1 - t)) & 1) != (isx[t][i] ? 0 : 1)) return false;
  }
  // Slot bit of each node before stage t (pb[t][i]): stage-t partners differ in it, and
  // partners at any earlier stage agree in it (they must share every bit but their own).
  std::vector<std::vector<int>> pb(S, std::vector<int>(n, -1));
  for (int t = 0; t < S; ++t) {
    std::vector<int> &c = pb[t];
    for (int s0 = 0; s0 < n; ++s0) {
      if (c[s0] >= 0) continue;
      c[s0] = 0;
      std::vector<int> stack{s0};
      while (!stack.empty()) {
        const int v = stack.back();
        stack.pop_back();
        for (int t2 = 0; t2 <= t; ++t2) {
          const int w = partner[t2][v];
          const int want = t2 == t ? 1 - c[v] : c[v];
          if (c[w] < 0) {
            c[w] = want;
            stack.push_back(w);
          } else if (c[w] != want) {
            return false;
          }
        }
      }
    }
  }
  std::vector<int> islot(n, 0);
  for (int i = 0; i < n; ++i)
    for (int t = 0; t < S; ++t) islot[i] |= pb[t][i] << (S - 1 - t);

  // orbits: one node per final slot and per initial slot, numbered by block-0 position
  std::vector<int> parent(n);
  for (int i = 0; i < n; ++i) parent[i] = i;
  auto find = [&](int v) {
    while (parent[v] != v) v = parent[v] = parent[parent[v]];
    return v;
  };
  for (int t = 0; t < S; ++t)
    for (int i = 0; i < n; ++i) parent[find(i)] = find(partner[t][i]);
  std::vector<int> orbit_id(n, -1);
  for (int k = 0; k < M; ++k) orbit_id[find(p.blocks[0].nodes[k])] = k;
  std::vector<int> node_fin((size_t)M * NB, -1), node_ini((size_t)M * NB, -1);
  for (int i = 0; i < n; ++i) {
    const int o = orbit_id[find(i)];
    if (o < 0) return false;
    int &cf = node_fin[(size_t)o * NB + fslot[i]];
    int &ci = node_ini[(size_t)o * NB + islot[i]];
    if (cf >= 0 || ci >= 0) return false;
    cf = ci = i;
  }
  // Sign flips: at stage t the pair (x, y) sits in slots (lo, lo | bit); when x (the V_X
  // node) starts in the upper slot the difference lands negated and is flipped back.
  const int PPS = NB / 2;  // pairs per stage within an orbit
  std::vector<uint64_t> oflip(M, 0);
  for (int t = 0; t < S; ++t) {
    const int bp = S - 1 - t;
    for (int x = 0; x < n; ++x) {
      if (!isx[t][x]) continue;
      // slot of x before stage t: final bits above t, initial bits from t down
      const int hi_mask = ~((1 << (bp + 1)) - 1) & (NB - 1);
      const int pre = (fslot[x] & hi_mask) | (islot[x] & ((1 << (bp + 1)) - 1));
      const int lo = pre & ~(1 << bp);
      const int k = ((lo >> (bp + 1)) << bp) | (lo & ((1 << bp) - 1));
      if (pb[t][x]) oflip[orbit_id[find(x)]] |= (uint64_t)1 << (t * PPS + k);
    }
  }

  const int Q = n / 4, KC = M / 4, NT = M / 16;
  const int FB = S * PPS;  // flip bits per orbit
  if (KC * FB > 64 || NT * 4 * FB > 64) return false;
  UProgramImage im;
  im.prog.S = S;
  im.prog.M = M;
  im.prog.n = n;
  im.prog.dir = direction;
  im.prog.prec = GFT_FP32;
  im.prog.gen = 0;
  im.gcol.assign((size_t)4 * Q, 0);
  im.scol.assign((size_t)4 * Q, 0);
  im.flips.assign(8, 0);
  for (int g = 0; g < 4; ++g) {
    uint64_t fw = 0;
    for (int kc = 0; kc < KC; ++kc)
      for (int b = 0; b < NB; ++b)
        im.gcol[(size_t)g * Q + kc * NB + b] =
            direction == 0 ? node_ini[(size_t)(4 * kc + g) * NB + b]
                           : p.blocks[b].out_pos[4 * kc + g];
    if (direction == 0)
      for (int kc = 0; kc < KC; ++kc) fw |= oflip[4 * kc + g] << (kc * FB);
    for (int nt = 0; nt < NT; ++nt)
      for (int v = 0; v < 4; ++v) {
        const int c = 16 * nt + 4 * g + v;
        for (int b = 0; b < NB; ++b) {
          if (direction == 0)
            im.scol[(size_t)g * Q + (b * NT + nt) * 4 + v] = p.blocks[b].out_pos[c];
          else
            im.scol[(size_t)g * Q + (nt * 4 + v) * NB + b] = node_ini[(size_t)c * NB + b];
        }
        if (direction == 1) fw |= oflip[c] << ((nt * 4 + v) * FB);
      }
    im.flips[2 * g] = (uint32_t)(fw & 0xffffffffu);
    im.flips[2 * g + 1] = (uint32_t)(fw >> 32);
  }
  im.afrag.assign((size_t)NB * NT * KC * 64, 0.0f);
  for (int b = 0; b < NB; ++b) {
    const HostBlock &B = p.blocks[b];
    for (int nt = 0; nt < NT; ++nt)
      for (int kc = 0; kc < KC; ++kc)
        for (int lane = 0; lane < 64; ++lane) {
          const int row = 16 * nt + lane % 16, k = 4 * kc + lane / 16;
          // forward: A[c][o] = V_b[pos(node(o,b))][c]; inverse: A[o][k] = V_b[pos(node(o,b))][k]
          const int o = direction == 0 ? k : row;
          const int c = direction == 0 ? row : k;
          const int node = node_fin[(size_t)o * NB + b];
          im.afrag[((size_t)(b * NT + nt) * KC + kc) * 64 + lane] =
              (float)(B.scale * B.V[(size_t)pos[node] * M + c]);
        }
  }
  out = std::move(im);
  return true;
}

}  // namespace gft

namespace gft {

int64_t large_workspace_cols(const GraphPlan &p) {
  int64_t cols = 0;
  for (const HostBlock &B : p.blocks) cols += (B.size + 7) & ~7;
  return cols;
}

bool build_large(const GraphPlan &p, int direction, LargeImage &out) {
  LargeImage im;
  const int n = p.n;
  if (n > kLargeMaxCols || large_workspace_cols(p) > kLargeMaxCols) return false;
  im.n = n;
  // block-contiguous workspace layout, each block's span padded to a multiple of 8 (16-byte
  // rows of BF16 workspace and matrices)
  // Node order inside each block's span.  With one left stage the nodes follow the order of
  // the Haar units (V_Z nodes after them), so column k of the sum block and column k of the
  // difference block derive from the same pair x_i, x_phi(i): the one-pass form then reads
  // each pair once for both blocks.  Otherwise ascending node labels.
  std::vector<int64_t> rank(n, 0);
  for (int v = 0; v < n; ++v) rank[v] = (int64_t)n + v;
  if (p.stages.size() == 1) {
    const HostStage &S0 = p.stages[0];
    for (size_t u = 0; u < S0.pair_x.size(); ++u) rank[S0.pair_x[u]] = rank[S0.pair_y[u]] = (int64_t)u;
    for (size_t z = 0; z < S0.znodes.size(); ++z) rank[S0.znodes[z]] = (int64_t)(S0.pair_x.size() + z);
  }
  std::vector<std::vector<int32_t>> ords;   // block position k -> index into B.nodes
  std::vector<int32_t> col_node, col_coef;   // per workspace column (or -1 for padding)
  int col = 0;
  size_t mat = 0;
  for (const HostBlock &B : p.blocks) {
    const int ld = (B.size + 7) & ~7;
    std::vector<int32_t> ord(B.size);
    for (int k = 0; k < B.size; ++k) ord[k] = k;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return rank[B.nodes[a]] < rank[B.nodes[b]]; });
    im.blocks.push_back({B.size, col, (int32_t)mat, ld, (int32_t)im.omap.size()});
    // final position of each block output: coefficients (forward) or nodes (inverse)
    for (int k = 0; k < B.size; ++k) im.omap.push_back(direction == 0 ? B.out_pos[k] : B.nodes[ord[k]]);
    im.block_sizes.push_back(B.size);
    for (int k = 0; k < ld; ++k) {
      col_node.push_back(k < B.size ? B.nodes[ord[k]] : -1);
      col_coef.push_back(k < B.size ? B.out_pos[k] : -1);
    }
    col += ld;
    mat += (size_t)B.size * ld;
    ords.push_back(std::move(ord));
  }
  im.ldw = col;
  if (im.ldw > kLargeMaxCols || mat > (size_t)INT32_MAX) return false;
  im.mats.assign(mat, 0.0f);
  for (size_t b = 0; b < p.blocks.size(); ++b) {
    const HostBlock &B = p.blocks[b];
    const LBlock &L = im.blocks[b];
    const std::vector<int32_t> &ord = ords[b];
    for (int k = 0; k < B.size; ++k)
      for (int c = 0; c < B.size; ++c)  // stored transposed: Mt[c][k] = M[k][c], with forward
        // M[k][c] = V[ord k][c] (input k: node ord k) and inverse M[k][c] = V[ord c][k]
        im.mats[(size_t)L.mat + (size_t)c * L.ld + k] =
            (float)(B.scale * (direction == 0 ? B.V[(size_t)ord[k] * B.size + c] : B.V[(size_t)ord[c] * B.size + k]));
  }
  im.mats16.resize(im.mats.size());
  for (size_t i = 0; i < im.mats.size(); ++i) im.mats16[i] = to_bf16_bits(im.mats[i]);
  // Workspace column col holds node col_node[col] (coefficient col_coef[col]) of its block,
  // or padding (-1).
  auto inverse_of = [&](const std::vector<int32_t> &cols, int nvals) {
    std::vector<int32_t> inv(nvals, -1);   // value -> workspace column
    for (int c = 0; c < (int)cols.size(); ++c)
      if (cols[c] >= 0) inv[cols[c]] = c;
    return inv;
  };
  const std::vector<int32_t> wcol_node = inverse_of(col_node, n);
  const std::vector<int32_t> wcol_coef = inverse_of(col_coef, n);
  // Stage programs of the two passes.  Pass 1 works on the input row (tile columns = node
  // positions forward, coefficient positions inverse); pass 3 on the workspace row (tile
  // columns = workspace columns).  Forward: left stages in pass 1, the right stage in pass
  // 3; inverse: the right stage in pass 1, the left stages (reversed) in pass 3.
  auto emit = [&](int k, const HostStage &S, const std::vector<int32_t> *map) {
    auto tcol = [&](int32_t v) { return (uint32_t)(map ? (*map)[v] : v); };
    const int off = (int)im.ops[k].size();
    for (size_t u = 0; u < S.pair_x.size(); ++u)
      im.ops[k].push_back(tcol(S.pair_x[u]) | (tcol(S.pair_y[u]) << 16));
    for (int32_t c : S.znodes) im.ops[k].push_back(tcol(c) | (0xffffu << 16));
    im.stages[k].push_back(off);
    im.stages[k].push_back((int)im.ops[k].size() - off);
  };
  const int ns = (int)p.stages.size();
  const bool has_right = !p.right.pair_x.empty();
  if (direction == 0) {
    for (int q = 0; q < ns; ++q) emit(0, p.stages[q], nullptr);
    if (has_right) emit(1, p.right, &wcol_coef);
  } else {
    if (has_right) emit(0, p.right, nullptr);
    for (int q = ns - 1; q >= 0; --q) emit(1, p.stages[q], &wcol_node);
  }
  for (int k = 0; k < 2; ++k) {
    PermPass &P = im.pass[k];
    P.num_stages = (int32_t)im.stages[k].size() / 2;
    const std::vector<int32_t> &map = (direction == 0) == (k == 0) ? col_node : col_coef;
    if (k == 0) {          // n-wide input -> workspace layout
      P.in_cols = n;
      P.out_cols = im.ldw;
      im.gather[k] = map;                        // node / coefficient of each ws column
    } else {               // workspace layout -> n-wide output
      P.in_cols = im.ldw;
      P.out_cols = n;
      im.gather[k] = inverse_of(map, n);         // ws column of each node / coefficient
    }
  }
  out = std::move(im);
  return true;
}

}  // namespace gft

namespace gft {

// Whether a one-set plan's entries can be loaded as pairs (OnePass::src_mode 5): for every
// lane's entries e = 2m and f = 2m + 1 of the block the kernel reads at that k (block 0
// while it has k steps, then block 1), the pair at entry e's first offset holds e's and f's
// first sources and the pair at entry f's second offset holds f's and e's second sources
// (where those entries use them), both pairs aligned and inside the row.
template <class Src>
static bool onepass_mirror_pairs(const OnePass &P, const std::vector<Src> &src, const std::vector<int32_t> &desc,
                                 int n, int esz) {
  if (n % 2 != 0) return false;   // rows start on pair boundaries
  for (int kt = 0; kt < P.nk; ++kt) {
    const int b = kt < P.nkc[0] || P.nblocks == 1 ? 0 : 1;
    for (int m = 0; m < 16; ++m) {
      const size_t e = (size_t)P.desc_off[b] + 32 * kt + 2 * m, f = e + 1;
      const int32_t *de = &desc[4 * e], *df = &desc[4 * f];
      const int32_t a = de[0], c = df[1];   // the two pairs' byte offsets
      if (a % (2 * esz) != 0 || c % (2 * esz) != 0 || a + 2 * esz > n * esz || c + 2 * esz > n * esz) return false;
      if (src[f].c0 != 0.0f && df[0] != a + esz) return false;   // f's first source follows e's
      if (src[e].c1 != 0.0f && de[1] != c + esz) return false;   // e's second source follows f's
      if (src[e].c0 != 0.0f && de[0] != a) return false;
      if (src[f].c1 != 0.0f && df[1] != c) return false;
    }
  }
  return true;
}

bool build_onepass(const LargeImage &L, int precision, bool in16, OnePassImage &out, bool general) {
  if (precision != GFT_FP32 && precision != GFT_BF16 && precision != GFT_SPLIT_BF16) return false;
  const PermPass &P1 = L.pass[0];
  const int nb = (int)L.blocks.size();
  const int esz = in16 ? 2 : 4;
  if (P1.num_stages > 1 || nb < 1 || nb > 2 || L.ldw > 1024 || L.n > kOnePassMaxN) return false;
  if (L.ops[1].size() > (size_t)kOnePassMaxOps3) return false;
  OnePassImage im;
  OnePass &P = im.P;
  im.mt = precision == GFT_SPLIT_BF16 ? 3 : 4;   // split: two operand planes, fewer rows
  P.n = L.n;
  P.ldw = L.ldw;
  P.slab_stride = L.ldw + 4;
  P.nblocks = nb;
  P.num_stages3 = L.pass[1].num_stages;
  P.ops3_words = (int)L.ops[1].size();
  // source mode 5 also writes the results straight to their output columns: a last pass
  // without stages whose gather takes every workspace column at most once
  bool direct = P.num_stages3 == 0 && (int)L.gather[1].size() == L.n;
  if (direct) {
    im.omap.assign((size_t)L.ldw, -1);
    for (int c = 0; c < L.n && direct; ++c) {
      const int w = L.gather[1][c];
      if (w < 0) continue;
      if (w >= L.ldw || im.omap[w] >= 0) direct = false;
      else im.omap[w] = c;
    }
  }
  // waves: each block's 16-column tiles over the fewest waves of at most 8 tiles each
  int wave = 0, entries = 0, frags = 0;
  for (int w = 0; w < 8; ++w) P.wblk[w] = -1, P.wnt0[w] = 0, P.wcnt[w] = 0;
  for (int b = 0; b < nb; ++b) {
    const LBlock &B = L.blocks[b];
    P.K[b] = B.size;
    P.col[b] = B.col;
    P.nkc[b] = (B.size + 31) / 32;
    P.ntl[b] = (B.size + 15) / 16;
    P.desc_off[b] = entries;
    P.frag_off[b] = frags;
    entries += 32 * P.nkc[b];
    frags += P.nkc[b] * P.ntl[b];
    const int waves = (P.ntl[b] + 7) / 8, per = (P.ntl[b] + waves - 1) / waves;
    if (wave + waves > 8) return false;
    for (int t = 0; t < P.ntl[b]; t += per, ++wave) {
      P.wblk[wave] = b;
      P.wnt0[wave] = t;
      P.wcnt[wave] = std::min(per, P.ntl[b] - t);
    }
    P.nk = std::max(P.nk, P.nkc[b]);
  }
  // first-pass value of each input position: its role in the (single) stage
  std::vector<int32_t> kind(L.n, 0), partner(L.n, -1);
  if (P1.num_stages == 1) {
    const int off = L.stages[0][0], cnt = L.stages[0][1];
    for (int u = 0; u < cnt; ++u) {
      const uint32_t op = L.ops[0][off + u];
      const int i = (int)(op & 0xffffu), j = (int)(op >> 16);
      if (j == 0xffff) {
        kind[i] = 3;
      } else {
        kind[i] = 1, partner[i] = j;   // x_i + x_j
        kind[j] = 2, partner[j] = i;   // x_i - x_j
      }
    }
  }
  // sources (src0, src1: input positions or -1) and coefficients of each entry
  struct Src {
    int32_t s0, s1;
    float c0, c1;
  };
  std::vector<Src> src(entries, Src{-1, -1, 0.0f, 0.0f});
  for (int b = 0; b < nb; ++b)
    for (int k = 0; k < P.K[b]; ++k) {
      const int t = L.gather[0][P.col[b] + k];
      Src &e = src[P.desc_off[b] + k];
      if (t < 0) continue;
      if (kind[t] == 1) e = {t, partner[t], 1.0f, 1.0f};
      else if (kind[t] == 2) e = {partner[t], t, 1.0f, -1.0f};
      else if (kind[t] == 3) e = {t, -1, 1.41421356237309504880f, 0.0f};
      else e = {t, -1, 1.0f, 0.0f};
    }
  // entries: byte offsets of the sources in the input row, coefficients
  im.desc.assign(4 * (size_t)entries, 0);
  for (int e = 0; e < entries; ++e) {
    const Src &x = src[e];
    int32_t *d = &im.desc[4 * (size_t)e];
    d[0] = x.s0 >= 0 ? x.s0 * esz : 0;
    d[1] = x.s1 >= 0 ? x.s1 * esz : d[0];
    std::memcpy(&d[2], &x.c0, 4);
    std::memcpy(&d[3], &x.c1, 4);
  }
  // how a k step's inputs are loaded (OnePass::src_mode): one set for both blocks where
  // every valid entry of the second block has the first block's offsets at the same k;
  // adjacent pairs where both blocks copy and the second block's source follows the first
  // block's (an even position, not the row's last, so that the pair lies in the row);
  // else one set per block, of one value per entry where no entry adds two values
  // (the pair starts at an even position below n - 1, so that it lies in the row; with the
  // second block's source first, block 0's offsets move to the pair's start)
  P.src_mode = nb == 1 ? (!general && direct && onepass_mirror_pairs(P, src, im.desc, L.n, esz) ? 5 : 1) : 2;
  P.pair_swap = 0;
  if (nb == 2 && !general) {
    bool same = true, pair[2] = {true, true};   // pair[s]: block 1's source at block 0's +1 (s = 0) or -1
    for (int k = 0; k < 32 * P.nkc[1] && (same || pair[0] || pair[1]); ++k) {
      const Src &b1 = src[P.desc_off[1] + k];
      if (b1.c0 == 0.0f) continue;   // padding
      if (k >= 32 * P.nkc[0]) {
        same = pair[0] = pair[1] = false;
        break;
      }
      const Src &b0 = src[P.desc_off[0] + k];
      const int32_t *d0 = &im.desc[4 * ((size_t)P.desc_off[0] + k)], *d1 = &im.desc[4 * ((size_t)P.desc_off[1] + k)];
      same = same && d0[0] == d1[0] && d0[1] == d1[1];
      const bool copies = b0.c1 == 0.0f && b1.c1 == 0.0f && b0.s0 >= 0;
      pair[0] = pair[0] && copies && b1.s0 == b0.s0 + 1;
      pair[1] = pair[1] && copies && b1.s0 == b0.s0 - 1;
    }
    for (int s = 0; s < 2; ++s)
      for (int k = 0; k < 32 * P.nkc[0] && pair[s]; ++k) {
        const Src &b0 = src[P.desc_off[0] + k];
        if (b0.c0 == 0.0f) continue;
        const int start = s == 0 ? b0.s0 : b0.s0 - 1;
        pair[s] = b0.c1 == 0.0f && start >= 0 && start % 2 == 0 && start + 1 < L.n;
      }
    // one value per entry in both blocks: copies and sqrt 2 scalings only (no sums or differences)
    bool single = true;
    for (int e = 0; e < entries && single; ++e) single = src[e].c1 == 0.0f;
    if (same) {
      P.src_mode = direct && onepass_mirror_pairs(P, src, im.desc, L.n, esz) ? 5 : 1;
    } else if (pair[0] || pair[1]) {
      P.src_mode = 3;
      P.pair_swap = pair[0] ? 0 : 1;
      if (P.pair_swap)
        for (int k = 0; k < 32 * P.nkc[0]; ++k) {
          int32_t *d0 = &im.desc[4 * ((size_t)P.desc_off[0] + k)];
          if (src[P.desc_off[0] + k].c0 != 0.0f) d0[0] -= esz;
        }
    } else if (single) {
      P.src_mode = 4;
    }
  }
  if (P.src_mode != 5) im.omap.clear();
  P.desc_words = 4 * entries;
  // B fragments (forward and inverse alike: M[k][c] = Mt[c][k] of the stored transpose),
  // rounded as the three-pass GEMM rounds them
  const int PL = precision == GFT_BF16 ? 1 : 2;
  im.frag.assign((size_t)frags * PL * 64 * 4, 0u);
  if (precision == GFT_FP32)
    for (int b = 0; b < nb; ++b) {
      const LBlock &B = L.blocks[b];
      for (int kc = 0; kc < P.nkc[b]; ++kc)
        for (int nt = 0; nt < P.ntl[b]; ++nt)
          for (int h = 0; h < 2; ++h)
            for (int lane = 0; lane < 64; ++lane)
              for (int e = 0; e < 4; ++e) {
                const int k = 32 * kc + 16 * h + 4 * (lane / 16) + e, c = 16 * nt + lane % 16;
                float m = 0.0f;
                if (k < B.size && c < B.size) m = L.mats[(size_t)B.mat + (size_t)c * B.ld + k];
                uint32_t w;
                std::memcpy(&w, &m, 4);
                const size_t f = (size_t)P.frag_off[b] + (size_t)kc * P.ntl[b] + nt;
                im.frag[((f * 2 + h) * 64 + lane) * 4 + e] = w;
              }
    }
  for (int b = 0; b < nb && precision != GFT_FP32; ++b) {
    const LBlock &B = L.blocks[b];
    for (int kc = 0; kc < P.nkc[b]; ++kc)
      for (int nt = 0; nt < P.ntl[b]; ++nt)
        for (int lane = 0; lane < 64; ++lane)
          for (int h = 0; h < 4; ++h) {
            uint32_t hiw = 0, low = 0;
            for (int e = 0; e < 2; ++e) {
              const int k = 32 * kc + 8 * (lane / 16) + 2 * h + e, c = 16 * nt + lane % 16;
              uint16_t hi = 0, lo = 0;
              if (k < B.size && c < B.size) {
                const size_t idx = (size_t)B.mat + (size_t)c * B.ld + k;
                if (precision == GFT_BF16) {
                  hi = L.mats16[idx];
                } else {
                  const float m = L.mats[idx];
                  hi = to_bf16_bits(m);
                  lo = to_bf16_bits(m - bf16_to_float(hi));
                }
              }
              hiw |= (uint32_t)hi << (16 * e);
              low |= (uint32_t)lo << (16 * e);
            }
            const size_t f = (size_t)P.frag_off[b] + (size_t)kc * P.ntl[b] + nt;
            im.frag[((f * PL + 0) * 64 + lane) * 4 + h] = hiw;
            if (PL == 2) im.frag[((f * PL + 1) * 64 + lane) * 4 + h] = low;
          }
  }
  // the kernel's LDS arrays are sized for these limits
  if (entries > kOnePassMaxEntries || P.nk > kOnePassMaxSteps) return false;
  out = std::move(im);
  return true;
}

}  // namespace gft
