"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only builds inputs: graphs as edge lists (Sec. II-B: undirected weighted
graph with self-loops), node pairings (involutions, Sec. IV-A, one array per butterfly
stage) and batches of graph signals.  It holds none of the transform's arithmetic: no
Laplacian, no eigenvectors, no Haar units.  Both the library under test and the oracle
consume exactly what it returns.

Node labels are 0-based.  A pairing stage ``phi`` is an int32 array with ``phi[i]`` the
partner of node ``i`` (``phi[i] == i`` for a node on the axis of symmetry).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 190707875


def rng_for(config: int, *sub: int) -> np.random.Generator:
    """PCG64 stream for configuration ``config`` (1-based), with optional sub-streams."""
    return np.random.default_rng([SEED_BASE, int(config), *[int(s) for s in sub]])


@dataclass
class Graph:
    n: int
    src: np.ndarray            # int32 [E]
    dst: np.ndarray            # int32 [E]
    weight: np.ndarray         # float64 [E]
    self_loop: Optional[np.ndarray] = None   # float64 [n] or None
    stages: List[np.ndarray] = field(default_factory=list)   # pairings, each int32 [n]
    name: str = ""

    @property
    def num_edges(self) -> int:
        return int(self.src.shape[0])

    def pairing(self) -> np.ndarray:
        if not self.stages:
            return np.zeros((0, self.n), dtype=np.int32)
        return np.ascontiguousarray(np.stack(self.stages).astype(np.int32))


def _graph(n, edges, weights=None, loops=None, stages=None, name=""):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    w = np.ones(len(e)) if weights is None else np.asarray(weights, dtype=np.float64)
    s = None if loops is None else np.asarray(loops, dtype=np.float64)
    return Graph(n=int(n), src=e[:, 0].astype(np.int32), dst=e[:, 1].astype(np.int32),
                 weight=w.astype(np.float64), self_loop=s,
                 stages=[np.asarray(p, dtype=np.int32) for p in (stages or [])], name=name)


# ----------------------------------------------------------------------------- pairings

def reversal(n: int) -> np.ndarray:
    """Order reversal i <-> n-1-i (the J matrix of the notation section)."""
    return np.arange(n - 1, -1, -1, dtype=np.int32)


def identity(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.int32)


def reversal_on(n: int, nodes) -> np.ndarray:
    """Reverse the listed nodes among themselves, fix every other node."""
    phi = identity(n)
    nodes = np.asarray(nodes, dtype=np.int32)
    phi[nodes] = nodes[::-1]
    return phi


# ----------------------------------------------------------------------------- families

def path(n: int, weights=None, loops=None, name="path") -> Graph:
    """Line graph 0-1-...-(n-1); one reversal stage (symmetric line graphs, Sec. V-B)."""
    edges = [(i, i + 1) for i in range(n - 1)]
    return _graph(n, edges, weights, loops, [reversal(n)] if n > 1 else [], name)


def cycle(n: int, name="cycle") -> Graph:
    """Unit-weight n-cycle; one reversal stage (steerable DFTs, Sec. V-C)."""
    edges = [(i, (i + 1) % n) for i in range(n)]
    return _graph(n, edges, None, None, [reversal(n)], name)


def grid_edges(N1: int, N2: int):
    edges = []
    for k in range(N1):
        for l in range(N2):
            v = k * N2 + l
            if l + 1 < N2:
                edges.append((v, v + 1))
            if k + 1 < N1:
                edges.append((v, v + N2))
    return edges


def grid_lr(N1: int, N2: int, cols=None) -> np.ndarray:
    """LR symmetry (k,l) <-> (k, N2-1-l) of Table 2, restricted to columns ``cols``."""
    cols = list(range(N2)) if cols is None else list(cols)
    phi = identity(N1 * N2)
    for k in range(N1):
        for a, b in zip(cols, cols[::-1]):
            phi[k * N2 + a] = k * N2 + b
    return phi


def grid_ud(N1: int, N2: int, rows=None) -> np.ndarray:
    """UD symmetry (k,l) <-> (N1-1-k, l) of Table 2, restricted to rows ``rows``."""
    rows = list(range(N1)) if rows is None else list(rows)
    phi = identity(N1 * N2)
    for l in range(N2):
        for a, b in zip(rows, rows[::-1]):
            phi[a * N2 + l] = b * N2 + l
    return phi


def grid(N1: int, N2: Optional[int] = None, name="grid") -> Graph:
    """Unit-weight 4-connected N1 x N2 grid, node (k,l) -> k*N2+l; stages LR then UD."""
    N2 = N1 if N2 is None else N2
    stages = [grid_lr(N1, N2), grid_ud(N1, N2)]
    return _graph(N1 * N2, grid_edges(N1, N2), None, None, stages, name)


def grid3d(A: int, B: int, C: int, name="grid3d") -> Graph:
    """Unit-weight 6-connected A x B x C grid, node (a,b,c) -> (a*B + b)*C + c; one
    reversal stage per axis (c, then b, then a)."""
    def v(a, b, c):
        return (a * B + b) * C + c
    edges = []
    for a in range(A):
        for b in range(B):
            for c in range(C):
                if c + 1 < C:
                    edges.append((v(a, b, c), v(a, b, c + 1)))
                if b + 1 < B:
                    edges.append((v(a, b, c), v(a, b + 1, c)))
                if a + 1 < A:
                    edges.append((v(a, b, c), v(a + 1, b, c)))
    n = A * B * C
    stages = []
    for axis in range(3):
        phi = identity(n)
        for a in range(A):
            for b in range(B):
                for c in range(C):
                    t = [a, b, c]
                    t[2 - axis] = [A, B, C][2 - axis] - 1 - t[2 - axis]
                    phi[v(a, b, c)] = v(*t)
        stages.append(phi)
    return _graph(n, edges, None, None, stages, name)


def cycle_two_stage(n: int, name="cycle2") -> Graph:
    """n-cycle (4 | n) with the reversal and then a reversal inside each half: both halves
    are symmetric paths (the + half plain, the - half with a self-loop 2 at each end)."""
    g = cycle(n, name)
    h = n // 2
    phi = identity(n)
    phi[:h] = np.arange(h - 1, -1, -1)
    phi[h:] = np.arange(n - 1, h - 1, -1)
    g.stages.append(phi)
    return g


def bidiagonal_grid(N: int, a: float = 0.5, name="grid6conn") -> Graph:
    """6-connected N x N grid: unit horizontal/vertical edges plus diagonal edges
    (k,l)-(k+1,l+1) of weight a.  Symmetric about both diagonals (Fig. grid_bidiag).
    Stages: diagonal symmetry (k,l) <-> (l,k), then anti-diagonal (k,l) <-> (N-1-l, N-1-k)."""
    edges = grid_edges(N, N)
    w = [1.0] * len(edges)
    for k in range(N - 1):
        for l in range(N - 1):
            edges.append((k * N + l, (k + 1) * N + l + 1))
            w.append(a)
    diag = identity(N * N)
    anti = identity(N * N)
    for k in range(N):
        for l in range(N):
            diag[k * N + l] = l * N + k
            anti[k * N + l] = (N - 1 - l) * N + (N - 1 - k)
    return _graph(N * N, edges, w, None, [diag, anti], name)


def zshaped_grid(N: int, w: float = 2.0, name="zgrid") -> Graph:
    """N x N grid with unit horizontal edges and anti-diagonal edges (k,l)-(k+1,l-1) of
    weight w (Fig. z4x4); centrosymmetric, one stage phi(i) = n-1-i."""
    edges, ws = [], []
    for k in range(N):
        for l in range(N):
            if l + 1 < N:
                edges.append((k * N + l, k * N + l + 1))
                ws.append(1.0)
            if k + 1 < N and l >= 1:
                edges.append((k * N + l, (k + 1) * N + l - 1))
                ws.append(w)
    return _graph(N * N, edges, ws, None, [reversal(N * N)], name)


def skeleton(spine: int, arm: int, leg: int, arm_at: int, leg_at: int, name="skeleton") -> Graph:
    """Skeleton tree: a spine path 0..spine-1 and two mirror-symmetric arms (attached at
    spine node arm_at) and legs (attached at leg_at); labels: spine, left arm, left leg,
    right arm, right leg.  One stage swaps left and right limbs (Fig. Gsk)."""
    edges = [(i, i + 1) for i in range(spine - 1)]
    n, limbs = spine, []
    for length, at in ((arm, arm_at), (leg, leg_at), (arm, arm_at), (leg, leg_at)):
        edges.append((at, n))
        edges += [(n + i, n + i + 1) for i in range(length - 1)]
        limbs.append((n, length))
        n += length
    phi = identity(n)
    for (b1, l1), (b2, _) in ((limbs[0], limbs[2]), (limbs[1], limbs[3])):
        for i in range(l1):
            phi[b1 + i], phi[b2 + i] = b2 + i, b1 + i
    return _graph(n, edges, None, None, [phi], name)


def _halving_chain(m: int):
    """Nested index ranges [0, m), [0, m/2), ... used by the recursive reversal stages."""
    ranges = []
    size = m
    while size >= 2:
        ranges.append(list(range(size)))
        size //= 2
    return ranges


def grid_recursive(N: int, name="grid_recursive") -> Graph:
    """N x N grid (N a power of two) with LR and UD reversals recursed on the + branch.

    Each axis contributes log2(N) stages; a stage reverses the first ``m`` columns (or
    rows) among themselves and fixes the rest, m = N, N/2, ..., 2.  Stages alternate
    LR, UD.
    """
    stages = []
    for r in _halving_chain(N):
        stages.append(grid_lr(N, N, r))
        stages.append(grid_ud(N, N, r))
    return _graph(N * N, grid_edges(N, N), None, None, stages, name)


def path_recursive(N: int, name="path_recursive") -> Graph:
    """Path of N nodes (N a power of two) with the reversal recursed on the + branch:
    stage t reverses the first N / 2^t nodes among themselves (log2 N stages); one axis
    of :func:`grid_recursive`."""
    g = path(N, name=name)
    g.stages = [reversal_on(N, r) for r in _halving_chain(N)]
    return g


def cartesian_product(ga: Graph, gb: Graph, name="product") -> Graph:
    """Cartesian product of two graphs: node (i, j) has label i * gb.n + j; edges
    (i, j)-(i', j) carry ga's weights, (i, j)-(i, j') gb's; self-loop s_a(i) + s_b(j).
    No stages (the product is planned from its factors)."""
    na, nb = ga.n, gb.n
    edges, w = [], []
    for e in range(ga.num_edges):
        for j in range(nb):
            edges.append((int(ga.src[e]) * nb + j, int(ga.dst[e]) * nb + j))
            w.append(float(ga.weight[e]))
    for e in range(gb.num_edges):
        for i in range(na):
            edges.append((i * nb + int(gb.src[e]), i * nb + int(gb.dst[e])))
            w.append(float(gb.weight[e]))
    loops = None
    if ga.self_loop is not None or gb.self_loop is not None:
        sa = np.zeros(na) if ga.self_loop is None else np.asarray(ga.self_loop, dtype=np.float64)
        sb = np.zeros(nb) if gb.self_loop is None else np.asarray(gb.self_loop, dtype=np.float64)
        loops = (sa[:, None] + sb[None, :]).reshape(-1)
    return _graph(na * nb, edges, w, loops, None, name)


def product_with_stages(ga: Graph, gb: Graph, name="product_staged") -> Graph:
    """Cartesian product of ga and gb (labels as :func:`cartesian_product`) carrying the
    factors' stages lifted to their axes, alternating axis b then axis a while both last:
    ga's stage phi_a becomes (i, j) -> (phi_a(i), j), gb's phi_b becomes (i, j) -> (i, phi_b(j))."""
    g = cartesian_product(ga, gb, name=name)
    na, nb = ga.n, gb.n
    i, j = np.divmod(np.arange(na * nb), nb)
    lifted_a = [(np.asarray(p)[i] * nb + j).astype(np.int32) for p in ga.stages]
    lifted_b = [(i * nb + np.asarray(p)[j]).astype(np.int32) for p in gb.stages]
    stages = []
    for t in range(max(len(lifted_a), len(lifted_b))):
        if t < len(lifted_b):
            stages.append(lifted_b[t])
        if t < len(lifted_a):
            stages.append(lifted_a[t])
    g.stages = stages
    return g


def skeleton25(name="skeleton25") -> Graph:
    """25-node skeleton tree: 5-node spine plus mirror-symmetric arms and legs of 5 nodes.

    Labels: spine 0-4 (0 = hip node, 3 = shoulder node, 4 = head), left arm 5-9,
    left leg 10-14, right arm 15-19, right leg 20-24.  Arm roots attach to node 3, leg
    roots to node 0.  One stage swaps left and right limbs node by node; the spine is
    fixed (skeletal graphs, Sec. V-E).
    """
    edges = [(0, 1), (1, 2), (2, 3), (3, 4)]
    for base, root in ((5, 3), (10, 0), (15, 3), (20, 0)):
        edges.append((root, base))
        edges += [(base + i, base + i + 1) for i in range(4)]
    phi = identity(25)
    for i in range(10):
        phi[5 + i] = 15 + i
        phi[15 + i] = 5 + i
    return _graph(25, edges, None, None, [phi], name)


def symmetric_bipartite(n: int, rng: np.random.Generator, p_edge=0.2, name="bipartite") -> Graph:
    """Random bipartite graph with an imposed part-preserving involution.

    Parts S1 = first floor(n/2) labels, S2 = the rest.  Within each part nodes are
    paired at random, leaving 0-2 nodes fixed.  For each orbit {(i,j),(phi i,phi j)}
    of cross-part node pairs both edges are added with probability ``p_edge`` and one
    shared weight U(0.5, 1.5).
    """
    n1 = n // 2
    parts = [np.arange(0, n1), np.arange(n1, n)]
    phi = identity(n)
    for part in parts:
        perm = rng.permutation(part)
        nfix = int(rng.integers(0, 3))
        if (len(perm) - nfix) % 2:
            nfix += 1
        nfix = min(nfix, len(perm))
        paired = perm[nfix:]
        for a, b in zip(paired[0::2], paired[1::2]):
            phi[a], phi[b] = b, a
    seen = set()
    edges, weights = [], []
    for i in parts[0]:
        for j in parts[1]:
            key = tuple(sorted([(int(i), int(j)), (int(phi[i]), int(phi[j]))]))
            if key in seen:
                continue
            seen.add(key)
            if rng.random() < p_edge:
                w = rng.uniform(0.5, 1.5)
                for (a, b) in set(key):
                    edges.append((a, b))
                    weights.append(w)
    if not edges:
        edges, weights = [(int(parts[0][0]), int(parts[1][0]))], [1.0]
        if phi[parts[0][0]] != parts[0][0] or phi[parts[1][0]] != parts[1][0]:
            a, b = int(phi[parts[0][0]]), int(phi[parts[1][0]])
            if (a, b) != edges[0]:
                edges.append((a, b))
                weights.append(1.0)
    return _graph(n, edges, weights, None, [phi], name)


def weighted_symmetric_path(N: int, rng: np.random.Generator, name="wpath") -> Graph:
    """Path with mirrored weights w_i = w_{N-2-i} ~ U(0.1,1) and mirrored loops ~ U(0,0.5)."""
    w = np.empty(N - 1)
    half = (N - 1) // 2
    w[:half] = rng.uniform(0.1, 1.0, half)
    w[N - 2 - np.arange(half)] = w[:half]
    if (N - 1) % 2:
        w[half] = rng.uniform(0.1, 1.0)
    s = np.empty(N)
    s[: N // 2] = rng.uniform(0.0, 0.5, N // 2)
    s[N - 1 - np.arange(N // 2)] = s[: N // 2]
    if N % 2:
        s[N // 2] = rng.uniform(0.0, 0.5)
    return path(N, w, s, name)


# ----------------------------------------------------------------------------- signals

def gaussian(S: int, n: int, rng: np.random.Generator, dtype=np.float32) -> np.ndarray:
    """i.i.d. N(0,1) signals, drawn in FP64 then rounded to ``dtype``."""
    return rng.standard_normal((S, n)).astype(dtype)


def ar1_field(S: int, N1: int, N2: int, rho: float, rng: np.random.Generator,
              dtype=np.float32, chunk: int = 1 << 16) -> np.ndarray:
    """Separable 2-D Gaussian AR(1) field, unit variance, node label k*N2+l.

    Per signal Z ~ N(0,1)^{N1 x N2}; along rows and then along columns
    y_0 = z_0, y_k = rho*y_{k-1} + sqrt(1-rho^2)*z_k.
    """
    out = np.empty((S, N1 * N2), dtype=dtype)
    c = np.sqrt(1.0 - rho * rho)
    for a in range(0, S, chunk):
        b = min(S, a + chunk)
        z = rng.standard_normal((b - a, N1, N2))
        for l in range(1, N2):
            z[:, :, l] = rho * z[:, :, l - 1] + c * z[:, :, l]
        for k in range(1, N1):
            z[:, k, :] = rho * z[:, k - 1, :] + c * z[:, k, :]
        out[a:b] = z.reshape(b - a, N1 * N2).astype(dtype)
    return out


def skeleton_walks_chunked(seqs: int, channels: int = 3, frames: int = 300, chunk: int = 512,
                           dtype=np.float32) -> np.ndarray:
    """Config 3 signals [seqs, channels, frames, 25], generated in chunks of ``chunk``
    sequences, chunk k from its own stream rng_for(3, 100 + k) (any chunk can be rebuilt)."""
    out = np.empty((seqs, channels, frames, 25), dtype=dtype)
    for k, a in enumerate(range(0, seqs, chunk)):
        b = min(seqs, a + chunk)
        out[a:b] = skeleton_walks(b - a, channels, frames, rng_for(3, 100 + k), dtype)
    return out


def skeleton_walks(seqs: int, channels: int, frames: int, rng: np.random.Generator,
                   dtype=np.float32) -> np.ndarray:
    """Smooth random-walk motion on the 25-joint skeleton, shape [seqs, channels, frames, 25].

    Per (sequence, channel) a pose is drawn down the tree (root ~ N(0,1), child = parent
    + N(0, 0.1^2)); each joint then follows a random walk over frames with N(0, 0.01^2)
    increments, smoothed by a 5-tap moving average.
    """
    g = skeleton25()
    parent = np.full(25, -1)
    for a, b in zip(g.src, g.dst):
        parent[b] = a
    pose = np.empty((seqs, channels, 25))
    pose[..., 0] = rng.standard_normal((seqs, channels))
    for j in range(1, 25):   # labels are in topological order: parents precede children
        pose[..., j] = pose[..., parent[j]] + 0.1 * rng.standard_normal((seqs, channels))
    steps = 0.01 * rng.standard_normal((seqs, channels, frames + 4, 25))
    walk = pose[:, :, None, :] + np.cumsum(steps, axis=2)
    k = np.ones(5) / 5.0
    cs = np.cumsum(np.concatenate([np.zeros((seqs, channels, 1, 25)), walk], axis=2), axis=2)
    smooth = (cs[:, :, 5:, :] - cs[:, :, :-5, :]) * k[0]
    return smooth[:, :, :frames, :].astype(dtype)


# ----------------------------------------------------------------------------- configs

def config1_graph() -> Graph:
    return path(8, name="path8")


def config2_graph() -> Graph:
    return grid(8, 8, name="grid8x8")


def config3_graph() -> Graph:
    return skeleton25()


def config4_graphs(rng: Optional[np.random.Generator] = None) -> List[Graph]:
    """Mixed batch: paths 4..64, cycles 8..64, square grids 4..16, bipartite 16..128."""
    rng = rng_for(4) if rng is None else rng
    gs = [path(n, name=f"path{n}") for n in range(4, 65)]
    gs += [cycle(n, name=f"cycle{n}") for n in range(8, 65)]
    gs += [grid(s, s, name=f"grid{s}x{s}") for s in range(4, 17)]
    gs += [symmetric_bipartite(n, rng, name=f"bip{n}") for n in range(16, 129, 8)]
    return gs


def config4_signal_counts(num_graphs: int, rng: np.random.Generator, lo=256, hi=65536):
    """Log-uniform integer signal counts in [lo, hi]."""
    u = rng.uniform(np.log(lo), np.log(hi + 1), num_graphs)
    return np.minimum(np.floor(np.exp(u)).astype(np.int64), hi)


def config5a_graph() -> Graph:
    return grid_recursive(64, name="grid64x64")


def config5b_graph() -> Graph:
    return weighted_symmetric_path(1024, rng_for(5, 1), name="wpath1024")
