// Plan -> device program (host side).
#include "program.hpp"

#include <algorithm>

namespace gft {

namespace {

uint32_t magic_for(uint32_t d) {
  // ceil(2^32 / d): floor(e * magic / 2^32) == e / d whenever e * d < 2^32.
  // d == 1 is encoded as 0 (the kernels divide by 1 directly).
  return d <= 1 ? 0u : (uint32_t)((((uint64_t)1 << 32) + d - 1) / d);
}

}  // namespace

size_t program_lds_bytes(const DevProgram &P) {
  const size_t T = 16 * (size_t)P.mt;
  return 4 * (size_t)((P.table_words + 3) & ~3) + 2 * T * (size_t)P.stride * 4;
}

bool build_program(const GraphPlan &p, int direction, int tile_override, size_t lds_budget,
                   ProgramImage &out) {
  const int n = p.n;
  DevProgram &P = out.prog;
  P = DevProgram{};
  P.n = n;
  P.stride = (n % 2) ? n : n + 1;
  P.magic_n = magic_for((uint32_t)n);

  std::vector<int32_t> stages, ops, blocks, items, gidx, sidx;
  std::vector<float> &frag = out.frag;
  frag.clear();

  // Haar stages: forward in plan order before the blocks; inverse in reverse after them.
  const int ns = (int)p.stages.size();
  for (int q = 0; q < ns; ++q) {
    const HostStage &st = p.stages[direction == 0 ? q : ns - 1 - q];
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
    stages.push_back((int32_t)magic_for((uint32_t)cnt));
    stages.push_back(0);
  }
  P.num_pre = direction == 0 ? ns : 0;
  P.num_post = direction == 0 ? 0 : ns;
  P.total_ops = (int32_t)(ops.size() / 2);

  // Blocks.  Forward: K = block nodes (gather node columns), N = eigenvectors (scatter to
  // output positions), M[j][k] = scale * V[j][k].  Inverse: K = output positions, N = nodes,
  // M[k][j] = scale * V[j][k].
  for (int b = 0; b < (int)p.blocks.size(); ++b) {
    const HostBlock &B = p.blocks[b];
    const int sz = B.size;
    const int kchunks = (sz + 3) / 4;
    const int ntiles = (sz + 15) / 16;
    const int g_off = (int)gidx.size(), s_off = (int)sidx.size(), f_off = (int)frag.size();
    const std::vector<int32_t> &kin = direction == 0 ? B.nodes : B.out_pos;
    const std::vector<int32_t> &nout = direction == 0 ? B.out_pos : B.nodes;
    for (int k = 0; k < 4 * kchunks; ++k) gidx.push_back(kin[k < sz ? k : 0]);
    for (int c = 0; c < sz; ++c) sidx.push_back(nout[c]);
    frag.resize(frag.size() + (size_t)kchunks * ntiles * 64, 0.0f);
    for (int kc = 0; kc < kchunks; ++kc)
      for (int nt = 0; nt < ntiles; ++nt)
        for (int lane = 0; lane < 64; ++lane) {
          const int k = 4 * kc + lane / 16, c = 16 * nt + lane % 16;
          double v = 0.0;
          if (k < sz && c < sz)
            v = direction == 0 ? B.V[(size_t)k * sz + c] : B.V[(size_t)c * sz + k];
          frag[f_off + ((size_t)kc * ntiles + nt) * 64 + lane] = (float)(B.scale * v);
        }
    blocks.insert(blocks.end(), {sz, kchunks, ntiles, g_off, s_off, f_off, 0, 0});
    for (int nt = 0; nt < ntiles; ++nt) items.push_back((b << 16) | nt);
  }
  // Largest blocks first so the waves of a workgroup finish together.
  std::stable_sort(items.begin(), items.end(), [&](int32_t a, int32_t c) {
    return blocks[8 * (a >> 16) + 1] > blocks[8 * (c >> 16) + 1];
  });
  P.num_blocks = (int32_t)p.blocks.size();
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
