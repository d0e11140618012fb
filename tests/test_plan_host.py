"""Host-side tests of the C ABI: exports, plan algebra vs the oracle, op counts, errors.

No GPU is used: gft_plan is host-only and gft_plan_apply_host / gft_plan_basis run the
plan's factorisation in FP64 on the host.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1907_07875_amd as G
import workloads as wl
from oracle import gft_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = G.load_library()
    header = open(os.path.join(ROOT, "include", "gft.h")).read()
    declared = set(re.findall(r"\b(gft_[a-z_]+)\s*\(", header))
    assert declared, "no declarations parsed"
    assert declared == set(G.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
    assert "gfx950" in G.version()


GRAPHS = [wl.config1_graph(), wl.config2_graph(), wl.config3_graph(), wl.cycle(12),
          wl.cycle(13), wl.cycle(80), wl.grid(5, 5), wl.grid(4, 6), wl.path(33),
          wl.symmetric_bipartite(48, wl.rng_for(4, 48)), wl.config5b_graph()]


@pytest.mark.parametrize("g", GRAPHS, ids=lambda g: f"{g.name}{g.n}")
def test_plan_basis_is_an_oracle_eigenbasis(g):
    plan = G.Plan.from_graph(g)
    lam, U = O.gft(O.laplacian_of(g))
    lam_p = plan.eigenvalues()
    scale = max(1.0, np.abs(lam).max())
    np.testing.assert_allclose(lam_p, lam, atol=1e-10 * scale)
    Uh = plan.basis()
    np.testing.assert_allclose(Uh.T @ Uh, np.eye(g.n), atol=1e-12)
    Ua, min_sv = O.align(U, Uh, lam)
    assert min_sv > 1 - 1e-9
    assert np.abs(Ua - Uh).max() < 1e-9
    X = wl.gaussian(17, g.n, wl.rng_for(9, g.n), dtype=np.float64)
    np.testing.assert_allclose(plan.apply_host(X, 0), O.forward(X, Ua), atol=1e-10)
    np.testing.assert_allclose(plan.apply_host(O.forward(X, Ua), 1), X, atol=1e-10)
    st = plan.info()
    assert st["max_orth_error"] < 1e-12 and st["max_residual"] < 1e-12


@pytest.mark.parametrize("g", [wl.path(8), wl.cycle(12), wl.config2_graph(), wl.config3_graph(),
                               wl.weighted_symmetric_path(16, wl.rng_for(9, 16)),
                               wl.symmetric_bipartite(40, wl.rng_for(4, 41)), wl.cycle_two_stage(16)],
                         ids=lambda g: f"{g.name}{g.n}")
def test_normalized_laplacian_plan_is_an_oracle_eigenbasis(g):
    """Same stages on D^{-1/2} L D^{-1/2}: symmetric graphs have d_i = d_phi(i), so the
    normalized Laplacian keeps every phi-symmetry and the left Haar decomposition applies.
    Every graph here has positive degrees (the bipartite draw is one without isolated nodes)."""
    assert np.all(O.degrees(g.n, g.src, g.dst, g.weight) > 0)
    plan = G.Plan.from_graph(g, laplacian="normalized")
    lam, U = O.gft(O.normalized_laplacian_of(g))
    np.testing.assert_allclose(plan.eigenvalues(), lam, atol=1e-10 * max(1.0, np.abs(lam).max()))
    Uh = plan.basis()
    np.testing.assert_allclose(Uh.T @ Uh, np.eye(g.n), atol=1e-12)
    Ua, min_sv = O.align(U, Uh, lam)
    assert min_sv > 1 - 1e-9
    X = wl.gaussian(9, g.n, wl.rng_for(9, g.n, 1), dtype=np.float64)
    np.testing.assert_allclose(plan.apply_host(X, 0), O.forward(X, Ua), atol=1e-10)
    assert plan.info()["num_stages"] == len(g.stages)


def test_normalized_laplacian_rejects_isolated_nodes():
    g = wl._graph(4, [(0, 1), (1, 2)])
    assert _status(lambda: G.gft_plan(4, g.src, g.dst, g.weight, laplacian="normalized")) == "GFT_ERR_GRAPH"


def test_config_op_counts():
    """Fast op counts (Table tab:runtime convention) of the benchmark graphs."""
    want = {"path8": (1, 4, 2, 32, 32), "grid8x8": (2, 64, 4, 1088, 1024),
            "skeleton25": (1, 10, 3, 270, 280)}
    for g in (wl.config1_graph(), wl.config2_graph(), wl.config3_graph()):
        st = G.Plan.from_graph(g).info()
        assert (st["num_stages"], st["num_units"], st["num_blocks"], st["adds"], st["mults"]) == want[g.name]


def test_skeleton_minus_graph_splits_into_limbs():
    """G- of the skeleton has two connected components (arm, leg), as in Fig. Gsk."""
    plan = G.Plan.from_graph(wl.config3_graph())
    sizes = sorted(len(b) for b in plan.blocks())
    assert sizes == [5, 5, 15]


def test_grid_recursive_64x64_blocks():
    """64x64 grid, LR/UD reversals recursed on the + branch: 49 blocks b_i * b_j."""
    g = wl.config5a_graph()
    plan = G.Plan.from_graph(g)
    st = plan.info()
    assert st["num_blocks"] == 49 and st["max_block"] == 1024
    sizes = sorted(len(b) for b in plan.blocks())
    axis = [32, 16, 8, 4, 2, 1, 1]
    assert sizes == sorted(a * b for a in axis for b in axis)
    assert st["mults"] - st["num_z_scalings"] == 1366 ** 2


def test_block_order_option():
    g = wl.config2_graph()
    p_eig = G.Plan.from_graph(g)
    p_blk = G.Plan.from_graph(g, order=G.ORDER_BLOCK)
    assert np.all(np.diff(p_eig.eigenvalues()) >= -1e-12)
    lb = p_blk.eigenvalues()
    assert not np.all(np.diff(lb) >= -1e-12)
    np.testing.assert_allclose(np.sort(lb), p_eig.eigenvalues(), atol=1e-12)


# ----------------------------------------------------------------------------- errors

def _status(fn):
    with pytest.raises(G.GFTError) as e:
        fn()
    return e.value.status_name


def test_error_not_involution():
    g = wl.path(6)
    assert _status(lambda: G.gft_plan(6, g.src, g.dst, g.weight, None, [np.array([1, 2, 0, 3, 4, 5])])) \
        == "GFT_ERR_NOT_INVOLUTION"
    assert _status(lambda: G.gft_plan(6, g.src, g.dst, g.weight, None, [np.array([0, 1, 2, 3, 4, 9])])) \
        == "GFT_ERR_NOT_INVOLUTION"


def test_error_not_symmetric_names_stage_and_nodes():
    g = wl.path(6, weights=[1, 2, 3, 4, 5])
    with pytest.raises(G.GFTError) as e:
        G.Plan.from_graph(g)
    assert e.value.status_name == "GFT_ERR_NOT_SYMMETRIC"
    assert "stage 0" in str(e.value)


def test_error_pairing_crosses_subgraph():
    g = wl.path(8)
    # after the reversal, {0..3} and {4..7} are separate sub-graphs; pairing 3 <-> 4 crosses
    bad = wl.identity(8)
    bad[3], bad[4] = 4, 3
    assert _status(lambda: G.gft_plan(8, g.src, g.dst, g.weight, None, [wl.reversal(8), bad])) \
        == "GFT_ERR_PAIRING_CROSSES_SUBGRAPH"


def test_error_bad_graphs():
    assert _status(lambda: G.gft_plan(3, [0, 1], [1, 5], [1.0, 1.0])) == "GFT_ERR_GRAPH"
    assert _status(lambda: G.gft_plan(3, [0, 1], [1, 1], [1.0, 1.0])) == "GFT_ERR_GRAPH"
    assert _status(lambda: G.gft_plan(3, [0, 1], [1, 0], [1.0, 1.0])) == "GFT_ERR_GRAPH"
    assert _status(lambda: G.gft_plan(3, [0], [1], [np.nan])) == "GFT_ERR_GRAPH"
    assert _status(lambda: G.gft_plan(3, [0], [1], [1.0], [0, np.inf, 0])) == "GFT_ERR_GRAPH"
    assert _status(lambda: G.gft_plan(0, [], [], [])) == "GFT_ERR_INVALID_ARG"


def test_error_bad_options():
    g = wl.path(4)
    assert _status(lambda: G.gft_plan(4, g.src, g.dst, g.weight, precision=7)) == "GFT_ERR_INVALID_ARG"
    assert _status(lambda: G.gft_plan(4, g.src, g.dst, g.weight, order=3)) == "GFT_ERR_INVALID_ARG"
    assert _status(lambda: G.gft_plan(4, g.src, g.dst, g.weight, tile=24)) == "GFT_ERR_INVALID_ARG"
    # storage types: only FP32 / BF16 values; batch plans run FP32 storage only
    o = G._options()
    o.in_dtype = 2
    h = ctypes.c_void_p()
    keep = []
    gs = G._graph_struct(4, g.src, g.dst, g.weight, None, keep)
    ps = G._pairing_struct(4, g.stages, keep)
    assert G.load_library().gft_plan(ctypes.byref(gs), ctypes.byref(ps), ctypes.byref(o), ctypes.byref(h)) == 1
    assert _status(lambda: G.gft_plan_batch([g, wl.path(6)], in_dtype="bf16")) == "GFT_ERR_UNSUPPORTED"
    p = G.gft_plan(4, g.src, g.dst, g.weight, stages=g.stages, in_dtype="bf16", out_dtype="bf16")
    assert (p.in_dtype, p.out_dtype) == ("bf16", "bf16")


def test_wide_signals_beyond_one_lds_row_rejected_at_planning():
    """Signals wider than a generic-engine tile run on the large-signal engine, which stages
    whole FP32 rows (input and block-padded workspace) in 160 KB of LDS: at most 40960
    columns.  An edgeless graph has one block per node, each padded to 8 workspace
    columns: 5120 nodes fill exactly 40960, 5121 exceed it and no engine can run the plan."""
    ok = G.gft_plan(5120, [], [], [])
    assert ok.info()["num_blocks"] == 5120
    e = None
    try:
        G.gft_plan(5121, [], [], [])
    except G.GFTError as err:
        e = err
    assert e is not None and e.status_name == "GFT_ERR_UNSUPPORTED" and "40960" in str(e)
    assert _status(lambda: G.gft_plan(40961, [], [], [])) == "GFT_ERR_UNSUPPORTED"


def test_null_arguments_rejected():
    lib = G.load_library()
    h = ctypes.c_void_p()
    assert lib.gft_plan(None, None, None, ctypes.byref(h)) == 1
    assert lib.gft_forward(None, None, None, 1, None) == 1
    assert lib.gft_plan_info(None, 0, None) == 1
    assert lib.gft_plan_destroy(None) == 0


def test_negative_weights_accepted():
    """Sub-graphs carry negative weights (Sec. IV-C); the input graph may too."""
    g = wl.path(6, weights=[1.0, -0.5, 2.0, -0.5, 1.0])
    plan = G.Plan.from_graph(g)
    lam, U = O.gft(O.laplacian_of(g))
    np.testing.assert_allclose(plan.eigenvalues(), lam, atol=1e-12)


def test_single_node_and_no_edges():
    for n, src, dst, w in ((1, [], [], []), (5, [], [], [])):
        plan = G.gft_plan(n, src, dst, w)
        X = np.arange(3 * n, dtype=np.float64).reshape(3, n)
        np.testing.assert_allclose(np.abs(plan.apply_host(X, 0)).sum(axis=1), np.abs(X).sum(axis=1))


def test_two_sparse_transposition_stage():
    """A single transposition (Lemma 2sparse) is a one-unit stage; U- is 1x1."""
    n = 6
    g = wl._graph(n, [(0, j) for j in range(1, n)])
    phi = wl.identity(n)
    phi[2], phi[5] = 5, 2
    plan = G.gft_plan(n, g.src, g.dst, g.weight, None, [phi])
    st = plan.info()
    assert st["num_units"] == 1 and sorted(len(b) for b in plan.blocks())[0] == 1
    lam, U = O.gft(O.laplacian_of(g))
    Ua, sv = O.align(U, plan.basis(), lam)
    assert sv > 1 - 1e-10


# ------------------------------------------------------------------ right Haar units

def _golden_c4():
    rows, scale = [], 1.0
    for line in open(os.path.join(ROOT, "tests", "golden", "c4_cycle.txt")):
        line = line.split("#")[0].strip()
        if not line or line.startswith("eigenvalues"):
            continue
        if line.startswith("scale"):
            scale = float(line.split()[1])
        else:
            rows.append([float(v) for v in line.split()])
    return scale * np.array(rows)


def _assert_oracle_basis(plan, g, laplacian="combinatorial"):
    L = O.laplacian_of(g) if laplacian == "combinatorial" else O.normalized_laplacian_of(g)
    lam, U = O.gft(L)
    np.testing.assert_allclose(plan.eigenvalues(), lam, atol=1e-10 * max(1.0, np.abs(lam).max()))
    Uh = plan.basis()
    np.testing.assert_allclose(Uh.T @ Uh, np.eye(g.n), atol=1e-12)
    Ua, min_sv = O.align(U, Uh, lam)
    assert min_sv > 1 - 1e-9
    X = wl.gaussian(7, g.n, wl.rng_for(9, g.n, 2), dtype=np.float64)
    np.testing.assert_allclose(plan.apply_host(X, 0), O.forward(X, Ua), atol=1e-10)
    np.testing.assert_allclose(plan.apply_host(O.forward(X, Ua), 1), X, atol=1e-10)


def test_c4_left_and_right_haar_reproduce_the_printed_gft():
    """Sec. III: the 4-cycle GFT factors into a left and a right butterfly stage.  With the
    reversal pairing, both leaves (L+ = [[1,-1],[-1,1]], L- = [[3,-1],[-1,3]]) have a
    constant diagonal and one edge, so each becomes two 1 x 1 blocks and a right Haar unit;
    the basis is the printed C4 matrix up to column signs."""
    g = wl.cycle(4)
    g.stages = [np.array([3, 2, 1, 0], dtype=np.int32)]
    plan = G.Plan.from_graph(g)
    st = plan.info()
    assert (st["num_right_leaves"], st["num_right_units"], st["num_blocks"], st["max_block"]) == (2, 2, 4, 1)
    assert (st["num_units"], st["mults"], st["adds"]) == (4, 4, 8)
    Uc4 = _golden_c4()
    np.testing.assert_allclose(np.abs(plan.basis().T @ Uc4), np.eye(4), atol=1e-14)
    _assert_oracle_basis(plan, g)
    dense = G.Plan.from_graph(g, right_haar=False).info()
    assert (dense["num_right_leaves"], dense["num_blocks"], dense["mults"]) == (0, 2, 8)


@pytest.mark.parametrize("n", [8, 12, 30])
def test_even_cycle_is_two_regular_bipartite(n):
    """Without left stages an even cycle is one 2-regular bipartite leaf: blocks n/2 + n/2
    and n/2 right Haar units (Thm. right_haar), (n/2)^2 * 2 multiplications instead of n^2."""
    g = wl.cycle(n)
    g.stages = []
    plan = G.Plan.from_graph(g)
    st = plan.info()
    assert (st["num_right_leaves"], st["num_blocks"], st["max_block"], st["mults"]) == (1, 2, n // 2, n * n // 2)
    # eigenvalue c = 2 (singular value 0, cos(2 pi k / n) = 0) occurs twice exactly when 4 | n;
    # those two columns pass through unpaired
    assert st["num_right_units"] == n // 2 - (1 if n % 4 == 0 else 0)
    _assert_oracle_basis(plan, g)


def _k_regular_bipartite(m, weights, loop=0.0):
    """Parts {0..m-1}, {m..2m-1}; node i joins m + (i + r) mod m with weight weights[r]:
    every node has weighted degree sum(weights) (a weighted k-regular bipartite graph)."""
    edges, w = [], []
    for r, wr in enumerate(weights):
        for i in range(m):
            edges.append((i, m + (i + r) % m))
            w.append(wr)
    return wl._graph(2 * m, edges, w, loops=np.full(2 * m, loop) if loop else None)


@pytest.mark.parametrize("m,weights,loop", [(5, [1.0, 1.0, 1.0], 0.0), (7, [0.3, 1.7, 0.9], 0.25),
                                            (16, [1.0, 0.5], 0.0)])
def test_weighted_k_regular_bipartite(m, weights, loop):
    g = _k_regular_bipartite(m, weights, loop)
    plan = G.Plan.from_graph(g)
    st = plan.info()
    assert (st["num_right_leaves"], st["num_blocks"], st["max_block"]) == (1, 2, m)
    _assert_oracle_basis(plan, g)


def test_normalized_laplacian_of_any_bipartite_graph():
    """Normalized Laplacian of a bipartite graph with parts of 5 and 9 nodes: diagonal 1, so
    the leaf takes right Haar units with p != n - p; the 4 extra part-2 columns are null
    vectors of the cross block (eigenvalue 1) and pass through."""
    rng = wl.rng_for(9, 3)
    p, q = 5, 9
    edges, w = [], []
    for j in range(q):
        for i in range(p):
            if rng.random() < 0.45 or i == j % p:
                edges.append((i, p + j))
                w.append(rng.uniform(0.5, 1.5))
    g = wl._graph(p + q, edges, w)
    plan = G.Plan.from_graph(g, laplacian="normalized")
    st = plan.info()
    assert (st["num_right_leaves"], st["num_blocks"], st["max_block"], st["num_right_units"]) == (1, 2, q, p)
    _assert_oracle_basis(plan, g, laplacian="normalized")
    assert G.Plan.from_graph(g).info()["num_right_leaves"] == 0     # combinatorial: degrees differ


def test_right_haar_leaves_benchmark_plans_alone():
    """Leaves of the benchmark graphs have varying diagonals: no right Haar units there."""
    for g in (wl.config1_graph(), wl.config2_graph(), wl.config3_graph(), wl.config5b_graph()):
        assert G.Plan.from_graph(g).info()["num_right_leaves"] == 0


# ------------------------------------------------------------------ pairing search

def _sym_graph(phi, rng, p=0.6):
    """Random phi-symmetric weighted graph with self-loops (Definition 2)."""
    n = len(phi)
    W = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            if W[i, j] == 0 and rng.random() < p:
                w = rng.uniform(0.1, 2.0)
                for a, b in ((i, j), (phi[i], phi[j])):
                    if a != b:
                        W[a, b] = W[b, a] = w
    s = rng.uniform(0.0, 1.0, n)
    return W, 0.5 * (s + s[phi])


def _graph_from_weights(W, s):
    n = len(W)
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if W[i, j] != 0]
    return wl._graph(n, edges, [W[i, j] for i, j in edges], loops=s)


def _find(g, **kw):
    return G.gft_find_pairing(g.n, g.src, g.dst, g.weight, g.self_loop, **kw)


def test_find_pairing_matches_brute_force_optimum():
    """Sec. V-F: the search returns a valid involution (Definition 2, checked by the oracle)
    with as many pairs as the best of all T(n) involutions, found by brute force."""
    rng = np.random.default_rng(21)
    for n in (3, 4, 5, 6, 7, 8):
        invs = O.involutions(n)
        for trial in range(5):
            phi0 = invs[rng.integers(len(invs))]
            W, s = _sym_graph(phi0, rng, p=0.6)
            g = _graph_from_weights(W, s)
            best = max(O.p_phi(phi) for phi in invs if O.is_phi_symmetric(W, s, phi, tol=1e-12))
            st = _find(g, max_stages=1)
            assert (O.p_phi(st[0]) if st else 0) == best, (n, phi0)
            if st:
                assert O.is_phi_symmetric(W, s, st[0], tol=1e-12)


@pytest.mark.parametrize("g", [wl.path(16), wl.cycle(12), wl.grid(8, 8), wl.config3_graph(),
                               wl.weighted_symmetric_path(24, wl.rng_for(9, 24))],
                         ids=lambda g: f"{g.name}{g.n}")
def test_found_stages_plan_an_exact_gft(g):
    """Stages found stage by stage inside the current sub-graphs: gft_plan accepts them (it
    checks Definition 2 on every sub-graph), the plan is an oracle eigenbasis, and it needs
    no more multiplications than the dense GFT."""
    st = _find(g, max_stages=8)
    assert len(st) >= 1
    assert O.p_phi(st[0]) == {"path": 8, "cycle": 6, "grid": 32, "skeleton25": 10, "wpath": 12}[g.name]
    plan = G.gft_plan(g.n, g.src, g.dst, g.weight, g.self_loop, stages=st)
    assert plan.info()["mults"] <= g.n * g.n
    _assert_oracle_basis(plan, g)


def test_find_pairing_on_paths_is_the_reversal_then_recursion():
    """A path's only non-trivial symmetry is the reversal; G+ is again a path with both end
    diagonals 1, so the next stage reverses it, and so on (the recursion of Sec. V)."""
    st = _find(wl.path(16), max_stages=8)
    np.testing.assert_array_equal(st[0], np.arange(15, -1, -1))
    assert [O.p_phi(p) for p in st] == [8, 4, 2, 1]


def test_find_pairing_no_symmetry():
    g = wl._graph(5, [(0, 1), (1, 2), (2, 3), (3, 4), (0, 2)], [1.0, 2.0, 3.0, 4.0, 5.0])
    assert _find(g) == []
    st = _find(wl.path(6), laplacian="normalized", max_stages=1)
    np.testing.assert_array_equal(st[0], np.arange(5, -1, -1))


def test_stream_copy_argument_checks_launch_nothing():
    """gft_stream_copy rejects bad arguments before it touches a device (so this runs on a
    host without a GPU); only invalid calls and the zero-byte no-op are made here."""
    lib = G.load_library()
    V = ctypes.c_void_p
    cases = [
        ((4096, 8192, 100), "GFT_ERR_INVALID_ARG"),     # not a multiple of 16
        ((4096, 8192, -16), "GFT_ERR_INVALID_ARG"),
        ((0, 8192, 4096), "GFT_ERR_INVALID_ARG"),       # NULL source
        ((4096, 0, 4096), "GFT_ERR_INVALID_ARG"),       # NULL destination
        ((4100, 8192, 1024), "GFT_ERR_ALIGNMENT"),
        ((4096, 4096 + 2048, 4096), "GFT_ERR_ALIGNMENT"),   # overlap
    ]
    for (a, b, nb), want in cases:
        st = lib.gft_stream_copy(V(a), V(b), nb, V(0))
        assert G.STATUS[st] == want, (a, b, nb, G.STATUS[st])
    assert lib.gft_stream_copy(V(4096), V(8192), 0, V(0)) == 0


def test_closed_form_leaves_are_dct2_and_dst4():
    """Leaves that are uniform paths (plus a constant self-loop) take the DCT-II basis in
    closed form, those with an extra self-loop 2w at one end DST-IV, instead of an
    eigensolve (Sec. V-C).  Pinned by the oracle's closed forms: the 8-node path with its
    reversal stage (leaves DCT-II(4) and DST-IV(4)) has the DCT-II(8) basis up to sign; a
    6-node path of weight 0.3 with self-loops 0.7 everywhere has the DCT-II(6) basis and the
    eigenvalues 0.7 + 0.3 (2 - 2 cos(pi k / 6)); weighted or odd-length leaves (a V_Z node
    scales edges by sqrt 2) keep the eigensolver."""
    plan = G.Plan.from_graph(wl.config1_graph())
    assert plan.info()["num_closed_form_leaves"] == 2
    U = plan.basis()
    np.testing.assert_allclose(np.abs(U.T @ O.dct2_matrix(8)), np.eye(8), atol=1e-14)
    np.testing.assert_allclose(plan.eigenvalues(), O.path_eigenvalues(8), atol=1e-14)
    g = wl.path(6, weights=[0.3] * 5)
    p = G.gft_plan(6, g.src, g.dst, g.weight, np.full(6, 0.7))
    assert p.info()["num_closed_form_leaves"] == 1
    np.testing.assert_allclose(p.eigenvalues(), 0.7 + 0.3 * O.path_eigenvalues(6), atol=1e-14)
    np.testing.assert_allclose(np.abs(p.basis().T @ O.dct2_matrix(6)), np.eye(6), atol=1e-14)
    # the halving recursion of a 64-path: every leaf of two or more nodes is DST-IV
    pr = G.Plan.from_graph(wl.path_recursive(64))
    assert pr.info()["num_closed_form_leaves"] == 5
    lam, U64 = O.gft(O.laplacian_of(wl.path_recursive(64)))
    Ua, sv = O.align(U64, pr.basis(), lam)
    assert sv > 1 - 1e-12 and np.abs(pr.basis() - Ua).max() <= 1e-12
    assert G.Plan.from_graph(wl.path(9)).info()["num_closed_form_leaves"] == 0
    assert G.Plan.from_graph(wl.config5b_graph()).info()["num_closed_form_leaves"] == 0
