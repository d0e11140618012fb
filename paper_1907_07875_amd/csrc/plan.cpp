// Host plan builder: validation, recursive symmetric decomposition, leaf eigensolves,
// output ordering and the FP64 host application of the factorisation.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <numeric>
#include <set>
#include <sstream>
#include <utility>

#include "eigen.hpp"

namespace gft {

namespace {

constexpr double kSqrt2 = 1.41421356237309504880;

[[noreturn]] void fail(gft_status s, const std::string &msg) { throw PlanError{s, msg}; }

// A current sub-graph of the decomposition: node labels (ascending) and its dense
// Laplacian over them (m*m row-major).
struct Sub {
  std::vector<int32_t> nodes;
  std::vector<double> L;
  int32_t depth = 0;
};

void validate_graph(const gft_graph &g) {
  if (g.n <= 0) fail(GFT_ERR_INVALID_ARG, "graph.n must be positive");
  if (g.num_edges < 0) fail(GFT_ERR_INVALID_ARG, "graph.num_edges must be >= 0");
  if (g.num_edges > 0 && (!g.src || !g.dst || !g.weight))
    fail(GFT_ERR_INVALID_ARG, "graph.src/dst/weight must be non-NULL when num_edges > 0");
  std::set<std::pair<int32_t, int32_t>> seen;
  for (int32_t e = 0; e < g.num_edges; ++e) {
    const int32_t a = g.src[e], b = g.dst[e];
    std::ostringstream os;
    if (a < 0 || a >= g.n || b < 0 || b >= g.n) {
      os << "edge " << e << " (" << a << "," << b << ") has a label outside [0," << g.n << ")";
      fail(GFT_ERR_GRAPH, os.str());
    }
    if (a == b) {
      os << "edge " << e << " joins node " << a << " to itself; pass self-loops in self_loop";
      fail(GFT_ERR_GRAPH, os.str());
    }
    if (!std::isfinite(g.weight[e])) {
      os << "edge " << e << " has a non-finite weight";
      fail(GFT_ERR_GRAPH, os.str());
    }
    if (!seen.insert({std::min(a, b), std::max(a, b)}).second) {
      os << "edge " << e << " (" << a << "," << b << ") is listed twice";
      fail(GFT_ERR_GRAPH, os.str());
    }
  }
  if (g.self_loop)
    for (int32_t i = 0; i < g.n; ++i)
      if (!std::isfinite(g.self_loop[i])) {
        std::ostringstream os;
        os << "self_loop[" << i << "] is not finite";
        fail(GFT_ERR_GRAPH, os.str());
      }
}

// L = D - W + S (eqs. def_laplacian, l_from_sw).
std::vector<double> dense_laplacian(const gft_graph &g) {
  const size_t n = (size_t)g.n;
  std::vector<double> L(n * n, 0.0);
  for (int32_t e = 0; e < g.num_edges; ++e) {
    const size_t a = (size_t)g.src[e], b = (size_t)g.dst[e];
    const double w = g.weight[e];
    L[a * n + b] -= w;
    L[b * n + a] -= w;
    L[a * n + a] += w;
    L[b * n + b] += w;
  }
  if (g.self_loop)
    for (size_t i = 0; i < n; ++i) L[i * n + i] += g.self_loop[i];
  return L;
}

double max_abs(const std::vector<double> &v) {
  double m = 0.0;
  for (double x : v) m = std::max(m, std::fabs(x));
  return m;
}

// Split sub-graph H by the local involution lp (Thm. decompose in matrix form, eq. Lpm):
//   L+ over V_X u V_Z:  (L_XX + L_XY J | sqrt2 L_XZ ; sqrt2 L_ZX | L_ZZ)
//   L- over V_Y:        L_YY - J L_XY
// with V_X = {a : lp[a] > a}, V_Y = lp(V_X), V_Z = fixed points.
void split(const Sub &H, const std::vector<int32_t> &lp, Sub &plus, Sub &minus,
           HostStage &stage) {
  const int m = (int)H.nodes.size();
  std::vector<int> pl, mi;
  std::vector<char> kind(m);  // 'x', 'y', 'z'
  for (int a = 0; a < m; ++a) {
    if (lp[a] == a) kind[a] = 'z';
    else kind[a] = lp[a] > a ? 'x' : 'y';
  }
  for (int a = 0; a < m; ++a) {
    if (kind[a] == 'y') mi.push_back(a);
    else pl.push_back(a);
    if (kind[a] == 'x') {
      stage.pair_x.push_back(H.nodes[a]);
      stage.pair_y.push_back(H.nodes[lp[a]]);
    } else if (kind[a] == 'z') {
      stage.znodes.push_back(H.nodes[a]);
    }
  }
  auto Lh = [&](int a, int b) { return H.L[(size_t)a * m + b]; };
  const int mp = (int)pl.size(), mm = (int)mi.size();
  plus.nodes.resize(mp);
  plus.L.assign((size_t)mp * mp, 0.0);
  plus.depth = H.depth + 1;
  for (int p = 0; p < mp; ++p) {
    plus.nodes[p] = H.nodes[pl[p]];
    for (int q = p; q < mp; ++q) {
      const int a = pl[p], b = pl[q];
      double v;
      if (kind[a] == 'x' && kind[b] == 'x') v = Lh(a, b) + Lh(a, lp[b]);
      else if (kind[a] == 'z' && kind[b] == 'z') v = Lh(a, b);
      else v = kSqrt2 * Lh(a, b);
      plus.L[(size_t)p * mp + q] = v;
      plus.L[(size_t)q * mp + p] = v;
    }
  }
  minus.nodes.resize(mm);
  minus.L.assign((size_t)mm * mm, 0.0);
  minus.depth = H.depth + 1;
  for (int p = 0; p < mm; ++p) {
    minus.nodes[p] = H.nodes[mi[p]];
    for (int q = p; q < mm; ++q) {
      const int a = mi[p], b = mi[q];
      const double v = Lh(a, b) - Lh(lp[a], b);
      minus.L[(size_t)p * mm + q] = v;
      minus.L[(size_t)q * mm + p] = v;
    }
  }
}

// Involution search on one sub-graph (Sec. V-F, pruning based on the degree list): a node
// can only be paired with a node of equal invariant (its diagonal entry and the sorted list
// of its off-diagonal entries, the weighted-degree-list generalisation), and a depth-first
// search assigns nodes, most constrained first, either a partner or a fixed point, keeping
// l_ab = l_phi(a)phi(b) against every node already assigned (Definition 2).  It maximises
// the number of pairs (minimising p^2 + (n - p)^2, Sec. V-G), stops at a perfect pairing, and
// gives up after `budget` search steps with the best involution found so far.
std::vector<int32_t> search_involution(const Sub &H, double tol, int64_t budget) {
  const int m = (int)H.nodes.size();
  auto L = [&](int a, int b) { return H.L[(size_t)a * m + b]; };
  std::vector<std::vector<double>> inv(m);
  for (int a = 0; a < m; ++a) {
    for (int b = 0; b < m; ++b)
      if (b != a && std::fabs(L(a, b)) > tol) inv[a].push_back(L(a, b));
    std::sort(inv[a].begin(), inv[a].end());
    inv[a].insert(inv[a].begin(), L(a, a));
  }
  auto same = [&](int a, int b) {
    if (inv[a].size() != inv[b].size()) return false;
    for (size_t i = 0; i < inv[a].size(); ++i)
      if (std::fabs(inv[a][i] - inv[b][i]) > tol) return false;
    return true;
  };
  std::vector<std::vector<int>> cand(m);
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b)
      if (b != a && same(a, b)) cand[a].push_back(b);
  std::vector<int> order(m);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return cand[a].size() < cand[b].size(); });
  std::vector<int32_t> phi(m, -1), best(m);
  std::iota(best.begin(), best.end(), 0);
  std::vector<int> assigned;
  int best_pairs = 0;
  int64_t steps = 0;
  auto consistent = [&](int a, int b) {
    for (int k : assigned) {
      if (std::fabs(L(a, k) - L(b, phi[k])) > tol) return false;
      if (b != a && std::fabs(L(b, k) - L(a, phi[k])) > tol) return false;
    }
    return true;
  };
  std::function<void(int, int, int)> dfs = [&](int pos, int pairs, int open) {
    if (++steps > budget || best_pairs * 2 >= m - 1) return;
    while (pos < m && phi[order[pos]] >= 0) ++pos;
    if (pos == m) {
      if (pairs > best_pairs) {
        best_pairs = pairs;
        best = phi;
      }
      return;
    }
    if (pairs + open / 2 <= best_pairs) return;   // cannot beat the best found
    const int a = order[pos];
    for (int b : cand[a]) {
      if (phi[b] >= 0 || !consistent(a, b)) continue;
      phi[a] = b;
      phi[b] = a;
      assigned.push_back(a);
      assigned.push_back(b);
      dfs(pos + 1, pairs + 1, open - 2);
      assigned.pop_back();
      assigned.pop_back();
      phi[a] = phi[b] = -1;
      if (steps > budget || best_pairs * 2 >= m - 1) return;
    }
    if (consistent(a, a)) {
      phi[a] = a;
      assigned.push_back(a);
      dfs(pos + 1, pairs, open - 1);
      assigned.pop_back();
      phi[a] = -1;
    }
  };
  dfs(0, 0, m);
  return best;
}

// Connected components of a sub-graph (couplings with |l_ab| > tol), each ascending.
// Right Haar split of a connected leaf (Sec. III, eq. right_gft, Thm. right_haar; Lemma
// k-rbg for the eigenvector pairing).  Lb is the leaf's b x b Laplacian.  It qualifies when
// its diagonal is a constant c and its off-diagonal pattern is bipartite (parts part1,
// part2).  From an FP64 eigendecomposition of Lb: every eigenvector (u1; u2) with eigenvalue
// c - s < c gives E's column sqrt2 u1 and F's column sqrt2 u2 (its mirror (u1; -u2) at c + s
// is the difference of the same two columns); the eigenspace of c splits into an
// orthonormal basis of its part-1 halves (E's remaining columns) and of its part-2 halves
// (F's).  Returns false when the leaf does not qualify or the counts do not come out.
struct RightSplit {
  std::vector<int> part1, part2;
  std::vector<double> E, F;          // p x p and q x q, column k of E at E[j * p + k]
  std::vector<double> lamE, lamF;    // eigenvalue carried by each column
  int pairs = 0;                     // leading paired columns
  std::vector<double> U, lamU;       // the b x b eigenbasis they imply (for the checks)
};

// Modified Gram-Schmidt (twice) of candidate vectors of length m; keeps those whose
// remaining norm exceeds keep_tol, appended to `basis` (k vectors of length m, column-major).
void orthonormal_extend(int m, const std::vector<std::vector<double>> &cands, double keep_tol,
                        std::vector<std::vector<double>> &basis) {
  for (std::vector<double> v : cands) {
    for (int pass = 0; pass < 2; ++pass)
      for (const std::vector<double> &w : basis) {
        double d = 0.0;
        for (int i = 0; i < m; ++i) d += w[i] * v[i];
        for (int i = 0; i < m; ++i) v[i] -= d * w[i];
      }
    double nr = 0.0;
    for (int i = 0; i < m; ++i) nr += v[i] * v[i];
    nr = std::sqrt(nr);
    if (nr <= keep_tol) continue;
    for (int i = 0; i < m; ++i) v[i] /= nr;
    basis.push_back(std::move(v));
  }
}

bool right_split(int b, const std::vector<double> &Lb, double tol, RightSplit &rs) {
  if (b < 2) return false;
  const double c = Lb[0];
  for (int i = 0; i < b; ++i)
    if (std::fabs(Lb[(size_t)i * b + i] - c) > tol) return false;
  std::vector<int> side(b, -1), queue{0};
  side[0] = 0;
  for (size_t h = 0; h < queue.size(); ++h) {
    const int i = queue[h];
    for (int j = 0; j < b; ++j) {
      if (j == i || std::fabs(Lb[(size_t)i * b + j]) <= tol) continue;
      if (side[j] < 0) {
        side[j] = 1 - side[i];
        queue.push_back(j);
      } else if (side[j] == side[i]) {
        return false;   // odd cycle: not bipartite
      }
    }
  }
  for (int i = 0; i < b; ++i) {
    if (side[i] < 0) return false;   // not connected (components are, so this is defensive)
    (side[i] == 0 ? rs.part1 : rs.part2).push_back(i);
  }
  const int p = (int)rs.part1.size(), q = (int)rs.part2.size();
  std::vector<double> lam, V;
  if (!symmetric_eigen(b, Lb, lam, V)) return false;
  double lmax = 1.0;
  for (double l : lam) lmax = std::max(lmax, std::fabs(l));
  const double thr = 1e-8 * lmax;
  std::vector<std::vector<double>> e_cols, f_cols, e_null, f_null;
  std::vector<double> pair_lam;
  int above = 0;
  std::vector<std::vector<double>> h1, h2;
  for (int k = 0; k < b; ++k) {
    std::vector<double> u1(p), u2(q);
    for (int a = 0; a < p; ++a) u1[a] = V[(size_t)rs.part1[a] * b + k];
    for (int a = 0; a < q; ++a) u2[a] = V[(size_t)rs.part2[a] * b + k];
    if (lam[k] < c - thr) {
      for (double &x : u1) x *= std::sqrt(2.0);
      for (double &x : u2) x *= std::sqrt(2.0);
      e_cols.push_back(std::move(u1));
      f_cols.push_back(std::move(u2));
      pair_lam.push_back(lam[k]);
    } else if (lam[k] > c + thr) {
      ++above;
    } else {
      h1.push_back(std::move(u1));
      h2.push_back(std::move(u2));
    }
  }
  const int m = (int)e_cols.size();
  if (above != m) return false;
  orthonormal_extend(p, h1, 1e-6, e_null);
  orthonormal_extend(q, h2, 1e-6, f_null);
  if (m + (int)e_null.size() != p || m + (int)f_null.size() != q) return false;
  rs.pairs = m;
  rs.E.assign((size_t)p * p, 0.0);
  rs.F.assign((size_t)q * q, 0.0);
  for (int k = 0; k < p; ++k) {
    const std::vector<double> &col = k < m ? e_cols[k] : e_null[k - m];
    for (int j = 0; j < p; ++j) rs.E[(size_t)j * p + k] = col[j];
    rs.lamE.push_back(k < m ? pair_lam[k] : c);
  }
  for (int k = 0; k < q; ++k) {
    const std::vector<double> &col = k < m ? f_cols[k] : f_null[k - m];
    for (int j = 0; j < q; ++j) rs.F[(size_t)j * q + k] = col[j];
    rs.lamF.push_back(k < m ? 2 * c - pair_lam[k] : c);
  }
  // the implied eigenbasis of Lb: (e; f)/sqrt2 and (e; -f)/sqrt2 per pair, (e0; 0), (0; f0)
  rs.U.assign((size_t)b * b, 0.0);
  int col = 0;
  auto put = [&](const std::vector<double> *e, const std::vector<double> *f, double fs, double sc,
                 double l) {
    for (int a = 0; a < p && e; ++a) rs.U[(size_t)rs.part1[a] * b + col] = sc * (*e)[a];
    for (int a = 0; a < q && f; ++a) rs.U[(size_t)rs.part2[a] * b + col] = sc * fs * (*f)[a];
    rs.lamU.push_back(l);
    ++col;
  };
  const double r2 = 1.0 / std::sqrt(2.0);
  for (int k = 0; k < m; ++k) {
    put(&e_cols[k], &f_cols[k], 1.0, r2, pair_lam[k]);
    put(&e_cols[k], &f_cols[k], -1.0, r2, 2 * c - pair_lam[k]);
  }
  for (const auto &v : e_null) put(&v, nullptr, 1.0, 1.0, c);
  for (const auto &v : f_null) put(nullptr, &v, 1.0, 1.0, c);
  return col == b;
}

std::vector<std::vector<int>> components(const Sub &H, double tol) {
  const int m = (int)H.nodes.size();
  std::vector<int> comp(m, -1);
  std::vector<std::vector<int>> out;
  for (int r = 0; r < m; ++r) {
    if (comp[r] >= 0) continue;
    std::vector<int> stack{r}, members;
    comp[r] = (int)out.size();
    while (!stack.empty()) {
      const int v = stack.back();
      stack.pop_back();
      members.push_back(v);
      for (int u = 0; u < m; ++u)
        if (u != v && comp[u] < 0 && std::fabs(H.L[(size_t)v * m + u]) > tol) {
          comp[u] = comp[r];
          stack.push_back(u);
        }
    }
    std::sort(members.begin(), members.end());
    out.push_back(members);
  }
  return out;
}

// Closed-form leaf bases (Sec. V-C): a leaf whose Laplacian is c I plus the Laplacian of a
// path with one edge weight w > 0 has the DCT-II eigenbasis, node i of the path (from one
// end) carrying sqrt((2 - [k = 0]) / b) cos(pi k (2i + 1) / (2b)) in eigenvector k, with
// eigenvalue c + 2w (1 - cos(pi k / b)); with an extra self-loop 2w at one end (the leaf
// on the difference side of a path's reversal, whose end next to the axis gains it) it is
// DST-IV from that end: sqrt(2 / b) sin(pi (2i + 1)(2k + 1) / (4b)), eigenvalue
// c + 2w (1 - cos(pi (2k + 1) / (2b))).  Entries are compared to `tol`.  Returns the kind
// (1 DCT-II, 2 DST-IV) with the basis (V[j * b + k], j in the leaf's node order) and the
// ascending eigenvalues, or 0.
int closed_form_leaf(int b, const std::vector<double> &L, double tol, std::vector<double> &lambda,
                     std::vector<double> &V) {
  if (b < 2) return 0;
  // path structure: every off-diagonal entry -w or 0, two ends of one neighbour
  double w = 0.0;
  std::vector<std::vector<int>> nb(b);
  for (int i = 0; i < b; ++i)
    for (int j = i + 1; j < b; ++j) {
      const double v = L[(size_t)i * b + j];
      if (std::fabs(v) <= tol) continue;
      if (w == 0.0) w = -v;
      if (!(w > tol) || std::fabs(v + w) > tol) return 0;
      nb[i].push_back(j);
      nb[j].push_back(i);
    }
  int end = -1;
  for (int i = 0; i < b; ++i) {
    if (nb[i].empty() || nb[i].size() > 2) return 0;
    if (nb[i].size() == 1 && end < 0) end = i;
  }
  if (end < 0) return 0;   // a cycle
  std::vector<int> order{end};
  for (int prev = -1, cur = end; (int)order.size() < b;) {
    int next = -1;
    for (int x : nb[cur])
      if (x != prev) next = x;
    if (next < 0) return 0;   // not connected
    order.push_back(next);
    prev = cur;
    cur = next;
  }
  auto d = [&](int i) { return L[(size_t)order[i] * b + order[i]]; };
  // DST-IV from the end with the larger diagonal
  if (d(b - 1) > d(0)) std::reverse(order.begin(), order.end());
  const double c = d(b - 1) - w;   // the free end: w + c
  bool uniform = true;
  for (int i = 1; i + 1 < b; ++i) uniform &= std::fabs(d(i) - (2 * w + c)) <= tol;
  if (!uniform) return 0;
  int kind = 0;
  if (std::fabs(d(0) - (w + c)) <= tol) kind = 1;
  else if (std::fabs(d(0) - (3 * w + c)) <= tol) kind = 2;
  if (!kind) return 0;
  const double pi = 3.14159265358979323846;
  lambda.assign(b, 0.0);
  V.assign((size_t)b * b, 0.0);
  for (int k = 0; k < b; ++k) {
    lambda[k] = kind == 1 ? c + 2 * w * (1 - std::cos(pi * k / b)) : c + 2 * w * (1 - std::cos(pi * (2 * k + 1) / (2.0 * b)));
    for (int i = 0; i < b; ++i)
      V[(size_t)order[i] * b + k] =
          kind == 1 ? std::sqrt((k == 0 ? 1.0 : 2.0) / b) * std::cos(pi * k * (2 * i + 1) / (2.0 * b))
                    : std::sqrt(2.0 / b) * std::sin(pi * (2 * i + 1) * (2 * k + 1) / (4.0 * b));
  }
  return kind;
}

// A graph read as a row-major Cartesian product G_a x G_b (node (i, j) = i * nb + j): the
// factors' edges, weights and self-loops, and the given stages sorted by axis.
struct ProductSplit {
  int32_t na = 0, nb = 0;
  std::vector<int32_t> src[2], dst[2];
  std::vector<double> w[2], loop[2];
  std::vector<int32_t> phi[2];   // stages along axis a (rows) and axis b (columns)
  int32_t stages[2] = {0, 0};
};

// Is g, with its stages, such a product for this (na, nb)?  Every edge must join two nodes
// of one row (an axis-b edge) or of one column (an axis-a edge), with the same weight in
// every row (column); self-loops must split as s(i, j) = s_a(i) + s_b(j); every stage must
// move one coordinate only, by the same involution in every row (column).  Weights and
// loops are compared to `tol` (relative to the largest magnitude).
bool product_split(const gft_graph &g, const gft_pairing *pairing, int32_t na, int32_t nb, double tol,
                   ProductSplit &ps) {
  const int32_t n = g.n;
  double wmax = 0.0;
  for (int32_t e = 0; e < g.num_edges; ++e) wmax = std::max(wmax, std::fabs(g.weight[e]));
  if (g.self_loop)
    for (int32_t i = 0; i < n; ++i) wmax = std::max(wmax, std::fabs(g.self_loop[i]));
  const double eps = tol * std::max(wmax, 1e-300);
  // factor weight matrices and, per factor edge, how many rows (columns) carry it
  const int32_t m[2] = {na, nb};
  std::vector<double> W[2];
  std::vector<int32_t> cnt[2];
  for (int a = 0; a < 2; ++a) {
    W[a].assign((size_t)m[a] * m[a], 0.0);
    cnt[a].assign((size_t)m[a] * m[a], 0);
  }
  for (int32_t e = 0; e < g.num_edges; ++e) {
    const int32_t u = g.src[e], v = g.dst[e];
    const int32_t iu = u / nb, ju = u % nb, iv = v / nb, jv = v % nb;
    int ax;
    int32_t p, q;
    if (iu == iv) {
      ax = 1;
      p = std::min(ju, jv);
      q = std::max(ju, jv);
    } else if (ju == jv) {
      ax = 0;
      p = std::min(iu, iv);
      q = std::max(iu, iv);
    } else {
      return false;
    }
    const size_t k = (size_t)p * m[ax] + q;
    if (cnt[ax][k] == 0) W[ax][k] = g.weight[e];
    else if (!(std::fabs(W[ax][k] - g.weight[e]) <= eps)) return false;
    ++cnt[ax][k];
  }
  for (int a = 0; a < 2; ++a) {
    ps.src[a].clear();
    ps.dst[a].clear();
    ps.w[a].clear();
    for (int32_t p = 0; p < m[a]; ++p)
      for (int32_t q = p + 1; q < m[a]; ++q) {
        const int32_t c = cnt[a][(size_t)p * m[a] + q];
        if (c == 0) continue;
        if (c != m[1 - a]) return false;   // the edge must repeat in every row (column)
        ps.src[a].push_back(p);
        ps.dst[a].push_back(q);
        ps.w[a].push_back(W[a][(size_t)p * m[a] + q]);
      }
  }
  ps.loop[0].assign(na, 0.0);
  ps.loop[1].assign(nb, 0.0);
  if (g.self_loop) {
    for (int32_t j = 0; j < nb; ++j) ps.loop[1][j] = g.self_loop[j];
    for (int32_t i = 0; i < na; ++i) ps.loop[0][i] = g.self_loop[(size_t)i * nb] - g.self_loop[0];
    for (int32_t i = 0; i < na; ++i)
      for (int32_t j = 0; j < nb; ++j)
        if (!(std::fabs(g.self_loop[(size_t)i * nb + j] - ps.loop[0][i] - ps.loop[1][j]) <= eps)) return false;
  }
  ps.na = na;
  ps.nb = nb;
  ps.phi[0].clear();
  ps.phi[1].clear();
  ps.stages[0] = ps.stages[1] = 0;
  const int32_t k = pairing ? pairing->num_stages : 0;
  for (int32_t s = 0; s < k; ++s) {
    const int32_t *phi = pairing->phi + (size_t)s * n;
    bool ident = true, along_a = true, along_b = true;
    for (int32_t v = 0; v < n; ++v) {
      const int32_t t = phi[v];
      if (t < 0 || t >= n) return false;
      ident &= t == v;
      const int32_t i = v / nb, j = v % nb, ti = t / nb, tj = t % nb;
      along_a &= tj == j && ti == phi[(size_t)i * nb] / nb && phi[(size_t)i * nb] % nb == 0;
      along_b &= ti == i && tj == phi[j] % nb && phi[j] / nb == 0;
    }
    if (ident) continue;
    const int ax = along_a ? 0 : (along_b ? 1 : -1);
    if (ax < 0) return false;
    for (int32_t c = 0; c < m[ax]; ++c)
      ps.phi[ax].push_back(ax == 0 ? phi[(size_t)c * nb] / nb : phi[c] % nb);
    ++ps.stages[ax];
  }
  return true;
}

}  // namespace

GraphPlan build_graph_plan(const gft_graph &g, const gft_pairing *pairing,
                           const gft_options &opts, bool recognize_products) {
  validate_graph(g);
  const int32_t n = g.n;
  const int32_t num_stages = pairing ? pairing->num_stages : 0;
  if (num_stages < 0) fail(GFT_ERR_INVALID_ARG, "pairing.num_stages must be >= 0");
  if (num_stages > 0 && !pairing->phi)
    fail(GFT_ERR_INVALID_ARG, "pairing.phi must be non-NULL when num_stages > 0");
  const double sym_tol = opts.sym_tol > 0 ? opts.sym_tol : 1e-12;

  GraphPlan plan;
  plan.n = n;
  plan.num_stages_given = num_stages;

  std::vector<Sub> subs(1);
  subs[0].nodes.resize(n);
  std::iota(subs[0].nodes.begin(), subs[0].nodes.end(), 0);
  subs[0].L = dense_laplacian(g);
  if (opts.laplacian == GFT_LAPLACIAN_NORMALIZED) {
    // D^{-1/2} L D^{-1/2} with the degrees of eq. l_from_sw (self-loops excluded)
    std::vector<double> d(n, 0.0);
    for (int32_t e = 0; e < g.num_edges; ++e) {
      d[g.src[e]] += g.weight[e];
      d[g.dst[e]] += g.weight[e];
    }
    for (int32_t i = 0; i < n; ++i)
      if (!(d[i] > 0.0)) {
        std::ostringstream os;
        os << "the normalized Laplacian needs a positive degree at every node; node " << i
           << " has degree " << d[i];
        fail(GFT_ERR_GRAPH, os.str());
      }
    for (int32_t i = 0; i < n; ++i)
      for (int32_t j = 0; j < n; ++j) subs[0].L[(size_t)i * n + j] /= std::sqrt(d[i] * d[j]);
  }
  const double scale_L = std::max(max_abs(subs[0].L), 1e-300);

  // Cartesian product with stages along the axes: plan the two factors (their leaves give
  // the leaf blocks' Kronecker bases below).  Only the combinatorial Laplacian is a
  // Kronecker sum.  The factors are planned without right Haar units (their leaves stay
  // dense blocks), and a Kronecker leaf is preferred to a right Haar split of the product
  // leaf: it is applied separably.
  std::shared_ptr<GraphPlan> kfa, kfb;
  int32_t kna = 0, knb = 0;
  if (recognize_products && opts.laplacian == GFT_LAPLACIAN_COMBINATORIAL && n >= 4) {
    ProductSplit ps;
    for (int32_t na = std::max<int32_t>(2, (n + 63) / 64); na <= 64 && na * 2 <= n && !kfa; ++na) {
      if (n % na != 0 || n / na > 64) continue;
      if (!product_split(g, pairing, na, n / na, sym_tol, ps)) continue;
      std::shared_ptr<GraphPlan> f[2];
      try {
        for (int a = 0; a < 2; ++a) {
          gft_graph fg{a == 0 ? ps.na : ps.nb, (int32_t)ps.src[a].size(), ps.src[a].data(), ps.dst[a].data(),
                       ps.w[a].data(), ps.loop[a].data()};
          gft_pairing fp{ps.stages[a], ps.phi[a].data()};
          gft_options fo = opts;
          fo.order = GFT_ORDER_EIGENVALUE;
          fo.right_haar = GFT_RIGHT_HAAR_OFF;
          f[a] = std::make_shared<GraphPlan>(build_graph_plan(fg, &fp, fo, false));
        }
      } catch (const PlanError &) {
        continue;   // a factor's stages are not valid on their own: plan the graph as given
      }
      if (f[0] && f[1]) {
        kfa = f[0];
        kfb = f[1];
        kna = ps.na;
        knb = ps.nb;
      }
    }
  }
  // factor block and local index of every factor node
  std::vector<int32_t> kblk[2], kpos[2];
  for (int a = 0; a < 2 && kfa; ++a) {
    const GraphPlan &F = a == 0 ? *kfa : *kfb;
    kblk[a].assign(F.n, -1);
    kpos[a].assign(F.n, -1);
    for (int32_t b = 0; b < (int32_t)F.blocks.size(); ++b)
      for (int32_t p = 0; p < F.blocks[b].size; ++p) {
        kblk[a][F.blocks[b].nodes[p]] = b;
        kpos[a][F.blocks[b].nodes[p]] = p;
      }
  }
  struct KronBlock {
    int32_t ba, bb;
    std::vector<int32_t> ka, kb;   // factor local indices of each local eigenvector
  };
  std::vector<KronBlock> kron_blocks;
  bool all_kron = (bool)kfa;
  int32_t num_closed = 0;   // leaves with a closed-form (DCT-II / DST-IV) basis

  std::vector<int32_t> owner(n, 0), local(n, 0);
  for (int32_t s = 0; s < num_stages; ++s) {
    const int32_t *phi = pairing->phi + (size_t)s * n;
    for (int32_t i = 0; i < n; ++i) {
      if (phi[i] < 0 || phi[i] >= n || phi[phi[i]] != i) {
        std::ostringstream os;
        os << "stage " << s << ": pairing is not an involution at node " << i
           << " (phi = " << phi[i] << ")";
        fail(GFT_ERR_NOT_INVOLUTION, os.str());
      }
    }
    for (size_t h = 0; h < subs.size(); ++h)
      for (size_t a = 0; a < subs[h].nodes.size(); ++a) {
        owner[subs[h].nodes[a]] = (int32_t)h;
        local[subs[h].nodes[a]] = (int32_t)a;
      }
    HostStage stage;
    std::vector<Sub> next;
    next.reserve(subs.size() * 2);
    for (size_t h = 0; h < subs.size(); ++h) {
      Sub &H = subs[h];
      const int m = (int)H.nodes.size();
      bool moves = false;
      std::vector<int32_t> lp(m);
      for (int a = 0; a < m; ++a) {
        const int32_t i = H.nodes[a], j = phi[i];
        if (owner[j] != (int32_t)h) {
          std::ostringstream os;
          os << "stage " << s << ": node " << i << " is paired with node " << j
             << ", which lies in a different sub-graph";
          fail(GFT_ERR_PAIRING_CROSSES_SUBGRAPH, os.str());
        }
        lp[a] = local[j];
        moves |= (j != i);
      }
      if (!moves) {
        next.push_back(std::move(H));
        continue;
      }
      // Definition 2 on the sub-graph: l_ab = l_{phi a, phi b} for all a, b
      const double tol = sym_tol * std::max(max_abs(H.L), 1e-300 * scale_L);
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
          const double d = H.L[(size_t)a * m + b] - H.L[(size_t)lp[a] * m + lp[b]];
          if (!(std::fabs(d) <= tol)) {
            std::ostringstream os;
            os << "stage " << s << ": sub-graph is not phi-symmetric at nodes (" << H.nodes[a]
               << "," << H.nodes[b] << ") vs (" << H.nodes[lp[a]] << "," << H.nodes[lp[b]]
               << "), difference " << d;
            fail(GFT_ERR_NOT_SYMMETRIC, os.str());
          }
        }
      Sub plus, minus;
      split(H, lp, plus, minus, stage);
      next.push_back(std::move(plus));
      if (!minus.nodes.empty()) next.push_back(std::move(minus));
    }
    subs = std::move(next);
    if (!stage.pair_x.empty()) plan.stages.push_back(std::move(stage));
  }

  // Leaves -> connected components -> dense blocks with FP64 eigensolves, or block pairs
  // (E, F) with right Haar units for leaves that qualify.
  double max_res = 0.0, max_orth = 0.0;
  struct RightPair {
    int32_t e, f, pairs;
  };
  std::vector<RightPair> right_pairs;
  for (const Sub &H : subs) {
    const int m = (int)H.nodes.size();
    const double tol = sym_tol * std::max(max_abs(H.L), 1e-300 * scale_L);
    for (const std::vector<int> &comp : components(H, tol)) {
      HostBlock B;
      B.size = (int32_t)comp.size();
      B.depth = H.depth;
      B.scale = std::pow(0.5, 0.5 * H.depth);
      const int b = B.size;
      std::vector<double> Lb((size_t)b * b);
      for (int p = 0; p < b; ++p) {
        B.nodes.push_back(H.nodes[comp[p]]);
        for (int q = 0; q < b; ++q) Lb[(size_t)p * b + q] = H.L[(size_t)comp[p] * m + comp[q]];
      }
      // Kronecker leaf: the block's nodes are exactly rows(B_a) x columns(B_b) of one block
      // of each factor plan; its basis V_a (x) V_b, ordered by lambda + mu (ties by the
      // factor indices).
      bool kron = false;
      KronBlock kb{-1, -1, {}, {}};
      if (all_kron) {
        const int32_t i0 = B.nodes[0] / knb, j0 = B.nodes[0] % knb;
        kb.ba = kblk[0][i0];
        kb.bb = kblk[1][j0];
        const HostBlock &A = kfa->blocks[kb.ba], &C = kfb->blocks[kb.bb];
        kron = A.size * C.size == b;
        for (int p = 0; p < b && kron; ++p) {
          const int32_t i = B.nodes[p] / knb, j = B.nodes[p] % knb;
          // nodes ascend: p = (local row) * |B_b| + local column
          kron = kblk[0][i] == kb.ba && kblk[1][j] == kb.bb && kpos[0][i] * C.size + kpos[1][j] == p;
        }
        if (kron) {
          std::vector<int32_t> idx((size_t)b);
          std::iota(idx.begin(), idx.end(), 0);
          std::stable_sort(idx.begin(), idx.end(), [&](int32_t u, int32_t v) {
            return A.lambda[u / C.size] + C.lambda[u % C.size] < A.lambda[v / C.size] + C.lambda[v % C.size];
          });
          B.lambda.resize(b);
          B.V.assign((size_t)b * b, 0.0);
          for (int k = 0; k < b; ++k) {
            const int32_t ka = idx[k] / C.size, kc = idx[k] % C.size;
            kb.ka.push_back(ka);
            kb.kb.push_back(kc);
            B.lambda[k] = A.lambda[ka] + C.lambda[kc];
            for (int pa = 0; pa < A.size; ++pa)
              for (int pc = 0; pc < C.size; ++pc)
                B.V[(size_t)(pa * C.size + pc) * b + k] = A.V[(size_t)pa * A.size + ka] * C.V[(size_t)pc * C.size + kc];
          }
        } else {
          all_kron = false;
        }
      }
      // a right Haar split is cheaper than any dense basis of the leaf (two-node leaves
      // with a constant diagonal are both a uniform path and a right Haar unit: Sec. III)
      RightSplit rs;
      const bool right = !kron && opts.right_haar == GFT_RIGHT_HAAR_AUTO && right_split(b, Lb, tol, rs);
      const int closed = kron || right ? 0 : closed_form_leaf(b, Lb, tol, B.lambda, B.V);
      if (closed) ++num_closed;
      if (kron || closed) {
        // basis set above; checked below like any leaf basis
      } else if (right) {
        B.lambda = rs.lamU;
        B.V = rs.U;            // checked below as any leaf basis
      } else if (!symmetric_eigen(b, Lb, B.lambda, B.V)) {
        std::ostringstream os;
        os << "eigensolver did not converge on a leaf block of size " << b;
        fail(GFT_ERR_EIGENSOLVE, os.str());
      }
      // plan-time checks: residual ||L V - V Lambda||_F / ||L||_F and orthogonality
      double res2 = 0.0, nrm2 = 0.0, orth = 0.0;
      for (int i = 0; i < b; ++i)
        for (int k = 0; k < b; ++k) {
          double s = 0.0, o = 0.0;
          for (int j = 0; j < b; ++j) {
            s += Lb[(size_t)i * b + j] * B.V[(size_t)j * b + k];
            o += B.V[(size_t)j * b + i] * B.V[(size_t)j * b + k];
          }
          const double r = s - B.lambda[k] * B.V[(size_t)i * b + k];
          res2 += r * r;
          nrm2 += Lb[(size_t)i * b + k] * Lb[(size_t)i * b + k];
          orth = std::max(orth, std::fabs(o - (i == k ? 1.0 : 0.0)));
        }
      const double res = std::sqrt(res2) / std::max(std::sqrt(nrm2), 1e-300);
      max_res = std::max(max_res, nrm2 > 0 ? res : std::sqrt(res2));
      max_orth = std::max(max_orth, orth);
      if (orth > 1e-10 || (nrm2 > 0 ? res : std::sqrt(res2)) > 1e-10) {
        std::ostringstream os;
        os << "leaf block of size " << b << " failed the plan-time check (orthogonality "
           << orth << ", residual " << res << ")";
        fail(GFT_ERR_ORTHOGONALITY, os.str());
      }
      if (right) {
        // E on part 1, F on part 2; the paired columns carry the 1/sqrt2 of their Haar unit
        HostBlock E, F;
        E.depth = F.depth = B.depth;
        E.scale = F.scale = B.scale;
        E.size = (int32_t)rs.part1.size();
        F.size = (int32_t)rs.part2.size();
        for (int a : rs.part1) E.nodes.push_back(B.nodes[a]);
        for (int a : rs.part2) F.nodes.push_back(B.nodes[a]);
        E.V = rs.E;
        F.V = rs.F;
        E.lambda = rs.lamE;
        F.lambda = rs.lamF;
        const double r2 = 1.0 / std::sqrt(2.0);
        for (int k = 0; k < rs.pairs; ++k) {
          for (int j = 0; j < E.size; ++j) E.V[(size_t)j * E.size + k] *= r2;
          for (int j = 0; j < F.size; ++j) F.V[(size_t)j * F.size + k] *= r2;
        }
        right_pairs.push_back({(int32_t)plan.blocks.size(), (int32_t)plan.blocks.size() + 1, rs.pairs});
        plan.blocks.push_back(std::move(E));
        plan.blocks.push_back(std::move(F));
        all_kron = false;
        continue;
      }
      if (kron) kron_blocks.push_back(std::move(kb));
      plan.blocks.push_back(std::move(B));
    }
  }

  // Output order: ascending eigenvalue; eigenvalues within tau of their neighbour form
  // one cluster, ordered by (block, local index).  Block order keeps block order.
  struct Ent {
    double lam;
    int32_t b, k;
  };
  std::vector<Ent> ents;
  double lam_max = 1.0;
  for (int32_t b = 0; b < (int32_t)plan.blocks.size(); ++b)
    for (int32_t k = 0; k < plan.blocks[b].size; ++k) {
      ents.push_back({plan.blocks[b].lambda[k], b, k});
      lam_max = std::max(lam_max, std::fabs(plan.blocks[b].lambda[k]));
    }
  if (opts.order == GFT_ORDER_EIGENVALUE) {
    std::stable_sort(ents.begin(), ents.end(),
                     [](const Ent &a, const Ent &b) { return a.lam < b.lam; });
    const double tau = 1e-9 * lam_max;
    size_t c0 = 0;
    for (size_t i = 1; i <= ents.size(); ++i) {
      if (i == ents.size() || ents[i].lam - ents[i - 1].lam > tau) {
        std::sort(ents.begin() + c0, ents.begin() + i, [](const Ent &a, const Ent &b) {
          return a.b != b.b ? a.b < b.b : a.k < b.k;
        });
        c0 = i;
      }
    }
  } else if (opts.order != GFT_ORDER_BLOCK) {
    fail(GFT_ERR_INVALID_ARG, "options.order must be 0 (eigenvalue) or 1 (block)");
  }
  for (auto &B : plan.blocks) B.out_pos.assign(B.size, -1);
  plan.lambda_out.resize(n);
  for (int32_t p = 0; p < (int32_t)ents.size(); ++p) {
    plan.blocks[ents[p].b].out_pos[ents[p].k] = p;
    plan.lambda_out[p] = ents[p].lam;
  }

  for (const RightPair &rp : right_pairs)
    for (int k = 0; k < rp.pairs; ++k) {
      plan.right.pair_x.push_back(plan.blocks[rp.e].out_pos[k]);   // c - s: the sum
      plan.right.pair_y.push_back(plan.blocks[rp.f].out_pos[k]);   // c + s: the difference
    }

  gft_plan_stats &st = plan.stats;
  st.n = n;
  st.num_stages = num_stages;
  st.num_units = 0;
  st.num_z_scalings = 0;
  for (const HostStage &S : plan.stages) {
    st.num_units += (int32_t)S.pair_x.size();
    st.num_z_scalings += (int32_t)S.znodes.size();
  }
  st.num_right_units = (int32_t)plan.right.pair_x.size();
  st.num_right_leaves = (int32_t)right_pairs.size();
  st.num_units += st.num_right_units;
  st.num_blocks = (int32_t)plan.blocks.size();
  st.max_block = 0;
  int64_t sum_b2 = 0, sum_bb1 = 0;
  for (const HostBlock &B : plan.blocks) {
    st.max_block = std::max(st.max_block, B.size);
    sum_b2 += (int64_t)B.size * B.size;
    sum_bb1 += (int64_t)B.size * (B.size - 1);
  }
  st.adds = 2 * (int64_t)st.num_units + sum_bb1;
  st.mults = sum_b2 + st.num_z_scalings;
  st.max_residual = max_res;
  st.max_orth_error = max_orth;
  st.num_kron_leaves = 0;
  st.num_closed_form_leaves = num_closed;
  st.separable_mults = st.mults;
  if (all_kron && kron_blocks.size() == plan.blocks.size()) {
    // coefficient (block b, local k) is factor coefficient pair (p, q): the factors'
    // output positions of (B_a, ka) and (B_b, kb)
    auto K = std::make_shared<KronPlan>();
    K->na = kna;
    K->nb = knb;
    K->fa = kfa;
    K->fb = kfb;
    K->order.assign(n, -1);
    int64_t sep = 0;
    for (size_t b = 0; b < plan.blocks.size(); ++b) {
      const KronBlock &kb = kron_blocks[b];
      const HostBlock &A = kfa->blocks[kb.ba], &C = kfb->blocks[kb.bb];
      sep += (int64_t)A.size * C.size * (A.size + C.size);
      for (int32_t k = 0; k < plan.blocks[b].size; ++k)
        K->order[plan.blocks[b].out_pos[k]] = A.out_pos[kb.ka[k]] * knb + C.out_pos[kb.kb[k]];
    }
    K->separable_mults = sep;
    st.num_kron_leaves = (int32_t)plan.blocks.size();
    st.separable_mults = sep + st.num_z_scalings;
    plan.kron = std::move(K);
  }
  return plan;
}

int find_pairing(const gft_graph &g, const gft_options &opts, int max_stages, int64_t budget,
                 std::vector<int32_t> &phi_out) {
  validate_graph(g);
  const int32_t n = g.n;
  const double sym_tol = opts.sym_tol > 0 ? opts.sym_tol : 1e-12;
  std::vector<Sub> subs(1);
  subs[0].nodes.resize(n);
  std::iota(subs[0].nodes.begin(), subs[0].nodes.end(), 0);
  subs[0].L = dense_laplacian(g);
  if (opts.laplacian == GFT_LAPLACIAN_NORMALIZED) {
    std::vector<double> d(n, 0.0);
    for (int32_t e = 0; e < g.num_edges; ++e) {
      d[g.src[e]] += g.weight[e];
      d[g.dst[e]] += g.weight[e];
    }
    for (int32_t i = 0; i < n; ++i)
      if (!(d[i] > 0.0)) fail(GFT_ERR_GRAPH, "the normalized Laplacian needs a positive degree at every node");
    for (int32_t i = 0; i < n; ++i)
      for (int32_t j = 0; j < n; ++j) subs[0].L[(size_t)i * n + j] /= std::sqrt(d[i] * d[j]);
  }
  const double scale_L = std::max(max_abs(subs[0].L), 1e-300);
  phi_out.clear();
  int stages = 0;
  for (; stages < max_stages; ++stages) {
    std::vector<int32_t> phi(n);
    std::iota(phi.begin(), phi.end(), 0);
    std::vector<Sub> next;
    bool any = false;
    HostStage unused;
    for (Sub &H : subs) {
      const double tol = sym_tol * std::max(max_abs(H.L), 1e-300 * scale_L);
      const std::vector<int32_t> lp = search_involution(H, tol, budget);
      bool moves = false;
      for (size_t a = 0; a < lp.size(); ++a) {
        phi[H.nodes[a]] = H.nodes[lp[a]];
        moves |= lp[a] != (int32_t)a;
      }
      if (!moves) {
        next.push_back(std::move(H));
        continue;
      }
      any = true;
      Sub plus, minus;
      split(H, lp, plus, minus, unused);
      next.push_back(std::move(plus));
      if (!minus.nodes.empty()) next.push_back(std::move(minus));
    }
    if (!any) break;
    phi_out.insert(phi_out.end(), phi.begin(), phi.end());
    subs = std::move(next);
  }
  return stages;
}

void apply_host(const GraphPlan &p, int direction, const double *x, double *y, int64_t S) {
  const int n = p.n;
  std::vector<double> z(n), w(n);
  for (int64_t s = 0; s < S; ++s) {
    const double *xs = x + s * n;
    double *ys = y + s * n;
    if (direction == 0) {
      std::copy(xs, xs + n, z.begin());
      for (const HostStage &st : p.stages) {
        for (size_t u = 0; u < st.pair_x.size(); ++u) {
          const double a = z[st.pair_x[u]], b = z[st.pair_y[u]];
          z[st.pair_x[u]] = a + b;
          z[st.pair_y[u]] = a - b;
        }
        for (int32_t c : st.znodes) z[c] *= kSqrt2;
      }
      for (const HostBlock &B : p.blocks)
        for (int k = 0; k < B.size; ++k) {
          double acc = 0.0;
          for (int j = 0; j < B.size; ++j) acc += B.V[(size_t)j * B.size + k] * z[B.nodes[j]];
          ys[B.out_pos[k]] = B.scale * acc;
        }
      for (size_t u = 0; u < p.right.pair_x.size(); ++u) {   // right Haar units
        const double a = ys[p.right.pair_x[u]], b = ys[p.right.pair_y[u]];
        ys[p.right.pair_x[u]] = a + b;
        ys[p.right.pair_y[u]] = a - b;
      }
    } else {
      std::copy(xs, xs + n, z.begin());
      for (size_t u = 0; u < p.right.pair_x.size(); ++u) {   // right Haar units (own inverse)
        const double a = z[p.right.pair_x[u]], b = z[p.right.pair_y[u]];
        z[p.right.pair_x[u]] = a + b;
        z[p.right.pair_y[u]] = a - b;
      }
      for (const HostBlock &B : p.blocks)
        for (int j = 0; j < B.size; ++j) {
          double acc = 0.0;
          for (int k = 0; k < B.size; ++k) acc += B.V[(size_t)j * B.size + k] * z[B.out_pos[k]];
          w[B.nodes[j]] = B.scale * acc;
        }
      for (auto it = p.stages.rbegin(); it != p.stages.rend(); ++it) {
        for (int32_t c : it->znodes) w[c] *= kSqrt2;
        for (size_t u = 0; u < it->pair_x.size(); ++u) {
          const double a = w[it->pair_x[u]], b = w[it->pair_y[u]];
          w[it->pair_x[u]] = a + b;
          w[it->pair_y[u]] = a - b;
        }
      }
      std::copy(w.begin(), w.end(), ys);
    }
  }
}

}  // namespace gft
