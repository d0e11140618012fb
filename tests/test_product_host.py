"""Product-graph plans on the host (no GPU): the Kronecker factorisation of the GFT of a
Cartesian product, checked against the FP64 oracle of the explicit product graph.

The Laplacian of G_a x G_b is L_a (x) I + I (x) L_b (self-loops add), so its eigenvalues are
the sums lambda_p + mu_q and U_a (x) U_b is an eigenbasis.  The pins below do not use the
plan's own algebra: eigenvalues against the oracle's eigendecomposition of the explicit
product Laplacian and, for unit paths, against the closed form of the path spectrum; the
basis through the residual of that Laplacian and orthogonality; the forward through the
oracle's coefficients after rotating its basis inside each eigenvalue cluster.
"""
import numpy as np
import pytest

import paper_1907_07875_amd as G
import workloads as wl
from oracle import gft_oracle as O

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")

PRODUCTS = [
    (wl.path(6), wl.path(5)),
    (wl.path(8), wl.path(8)),
    (wl.weighted_symmetric_path(12, wl.rng_for(9, 12)), wl.cycle(7)),
    (wl.path_recursive(16), wl.config3_graph()),
    (wl.symmetric_bipartite(24, wl.rng_for(4, 24)), wl.path(3)),
]


def _ids(pair):
    return f"{pair[0].name}{pair[0].n}x{pair[1].name}{pair[1].n}"


@pytest.mark.parametrize("pair", PRODUCTS, ids=_ids)
def test_product_spectrum_and_basis_match_explicit_product(pair):
    ga, gb = pair
    plan = G.Plan.from_product(ga, gb)
    g = wl.cartesian_product(ga, gb)
    L = O.laplacian_of(g)
    lam_o, U_o = O.gft(L)
    lam = plan.eigenvalues()
    np.testing.assert_allclose(lam, lam_o, atol=1e-10 * max(1.0, np.abs(lam_o).max()))
    U = plan.basis()
    n = g.n
    np.testing.assert_allclose(U.T @ U, np.eye(n), atol=1e-12)
    assert np.abs(L @ U - U * lam[None, :]).max() <= 1e-11 * max(1.0, np.abs(L).max())
    # forward on the host equals the oracle's coefficients in the plan's eigenbasis choice
    X = wl.gaussian(40, n, wl.rng_for(9, n, 11), dtype=np.float64)
    Ua, min_sv = O.align(U_o, U, lam_o)
    assert min_sv > 1 - 1e-9
    Y = plan.apply_host(X, 0)
    # eigh resolves near-degenerate clusters of the explicit product only to ~eps ||L|| / gap
    assert O.relative_error(Y, O.forward(X, Ua)) <= 1e-9
    assert O.relative_error(plan.apply_host(Y, 1), X) <= 1e-12


def test_product_of_unit_paths_is_the_2d_dct_spectrum():
    """Unit paths: the spectrum is the closed form 2 - 2cos(pi k/N) summed over the axes, and
    the basis spans the 2-D DCT-II eigenspaces (grid GFT = Kronecker of DCT-IIs)."""
    plan = G.Plan.from_product(wl.path(9), wl.path(6))
    la, lb = O.path_eigenvalues(9), O.path_eigenvalues(6)
    expect = np.sort((la[:, None] + lb[None, :]).reshape(-1))
    np.testing.assert_allclose(plan.eigenvalues(), expect, atol=1e-12)
    D = np.kron(O.dct2_matrix(9), O.dct2_matrix(6))       # columns: DCT-II basis vectors
    lam_d = (la[:, None] + lb[None, :]).reshape(-1)
    Ua, min_sv = O.align(D[:, np.argsort(lam_d, kind="stable")], plan.basis(), expect)
    assert min_sv > 1 - 1e-9


def test_product_order_block_is_row_major_kronecker():
    """GFT_ORDER_BLOCK: coefficient p * n_b + q is basis vector (p, q) of the factors, each
    factor in its own block order."""
    ga, gb = wl.path(5), wl.cycle(6)
    plan = G.Plan.from_product(ga, gb, order=G.ORDER_BLOCK)
    fa, fb = G.Plan.from_graph(ga, order=G.ORDER_BLOCK), G.Plan.from_graph(gb, order=G.ORDER_BLOCK)
    np.testing.assert_allclose(plan.basis(), np.kron(fa.basis(), fb.basis()), atol=1e-14)
    la, lb = fa.eigenvalues(), fb.eigenvalues()
    np.testing.assert_allclose(plan.eigenvalues(), (la[:, None] + lb[None, :]).reshape(-1), atol=1e-14)


def test_product_info_and_errors():
    plan = G.Plan.from_product(wl.path(10), wl.path(4))
    st = plan.info()
    assert st["n"] == 40 and st["num_blocks"] == 2 and st["max_block"] == 10
    assert st["mults"] == 40 * 14
    with pytest.raises(G.GFTError) as e:
        plan.blocks()
    assert e.value.status_name == "GFT_ERR_UNSUPPORTED"
    for kwargs in ({"precision": "fp16"}, {"laplacian": "normalized"}, {"engine": "generic"}):
        with pytest.raises(G.GFTError) as e:
            G.gft_plan_product(wl.path(4), wl.path(4), **kwargs)
        assert e.value.status_name == "GFT_ERR_UNSUPPORTED", kwargs
    with pytest.raises(G.GFTError) as e:
        G.gft_plan_product(wl.path(65), wl.path(2))
    assert e.value.status_name == "GFT_ERR_UNSUPPORTED"
    bad = wl.path(6)
    bad.stages = [np.array([1, 0, 2, 3, 4, 5], dtype=np.int32)]   # not a symmetry of the path
    with pytest.raises(G.GFTError):
        G.gft_plan_product(wl.path(4), bad)


def test_product_basis_is_the_grid_eigenbasis_at_4096():
    """The 64 x 64 grid as path64 x path64 (each axis with its halving reversal stages, the
    benchmark's product plan): residual and orthogonality of the product basis against the
    explicit 4096-node grid Laplacian, and the closed-form spectrum."""
    ga = wl.path_recursive(64)
    plan = G.Plan.from_product(ga, ga)
    U = plan.basis()
    lam = plan.eigenvalues()
    lp = O.path_eigenvalues(64)
    np.testing.assert_allclose(lam, np.sort((lp[:, None] + lp[None, :]).reshape(-1)), atol=1e-12)
    L = O.laplacian_of(wl.cartesian_product(ga, ga))
    assert np.abs(L @ U - U * lam[None, :]).max() <= 1e-10
    assert np.abs(U.T @ U - np.eye(4096)).max() <= 1e-10


# ---------------------------------------------------------------- Kronecker leaves in gft_plan

STAGED_PRODUCTS = [
    (wl.path(8), wl.path(8)),                                              # the 8x8 grid
    (wl.path_recursive(16), wl.path_recursive(16)),                        # 8 stages
    (wl.weighted_symmetric_path(12, wl.rng_for(9, 12)), wl.path(7)),       # weights, self-loops
    (wl.config3_graph(), wl.weighted_symmetric_path(9, wl.rng_for(9, 9))),
    (wl.path(5), wl.cycle(12)),                                            # V_Z nodes on axis a
]


@pytest.mark.parametrize("pair", STAGED_PRODUCTS, ids=_ids)
def test_gft_plan_recognises_products_and_gives_separable_leaves(pair):
    """gft_plan on a row-major Cartesian product whose stages act along one axis each: every
    leaf block gets a Kronecker basis, and the plan is an exact GFT of the product graph
    (oracle eigenvalues, Laplacian residual, orthogonality, aligned coefficients); every
    basis vector, reshaped to na x nb, is the outer product of one eigenvector of each
    factor Laplacian (checked against the oracle's factor eigendecompositions)."""
    ga, gb = pair
    g = wl.product_with_stages(ga, gb)
    plan = G.Plan.from_graph(g)
    st = plan.info()
    assert st["num_kron_leaves"] == st["num_blocks"] > 0
    L = O.laplacian_of(g)
    lam_o, U_o = O.gft(L)
    lam = plan.eigenvalues()
    np.testing.assert_allclose(lam, lam_o, atol=1e-10 * max(1.0, np.abs(lam_o).max()))
    U = plan.basis()
    np.testing.assert_allclose(U.T @ U, np.eye(g.n), atol=1e-12)
    assert np.abs(L @ U - U * lam[None, :]).max() <= 1e-11 * max(1.0, np.abs(L).max())
    X = wl.gaussian(30, g.n, wl.rng_for(9, g.n, 12), dtype=np.float64)
    Ua, min_sv = O.align(U_o, U, lam_o)
    assert min_sv > 1 - 1e-9
    assert O.relative_error(plan.apply_host(X, 0), O.forward(X, Ua)) <= 1e-9
    # separability: each basis vector is u_a (x) u_b with L_a u_a = l_a u_a, L_b u_b = l_b u_b
    La, Lb = O.laplacian_of(ga), O.laplacian_of(gb)
    for k in range(g.n):
        M = U[:, k].reshape(ga.n, gb.n)
        sv = np.linalg.svd(M, compute_uv=False)
        assert sv[0] == pytest.approx(1.0, abs=1e-10) and (len(sv) < 2 or sv[1] <= 1e-10)
        A, _, Bt = np.linalg.svd(M)
        ua, ub = A[:, 0], Bt[0]
        la, lb = ua @ La @ ua, ub @ Lb @ ub
        assert np.abs(La @ ua - la * ua).max() <= 1e-10 and np.abs(Lb @ ub - lb * ub).max() <= 1e-10
        assert la + lb == pytest.approx(lam[k], abs=1e-10)


def test_grid64_recursive_plan_has_separable_leaf_count():
    """The 64x64 grid with 12 halving stages: 49 leaf blocks, each b_i x b_j with b in
    (32, 16, 8, 4, 2, 1, 1) per axis.  Dense leaf products cost sum (b_i b_j)^2 =
    (sum b^2)^2 = 1366^2 multiplications per signal (Table tab:runtime convention); applied
    separably, b_i b_j (b_i + b_j) summed, 2 * 1366 * 64 = 174848."""
    plan = G.Plan.from_graph(wl.config5a_graph())
    st = plan.info()
    assert st["num_blocks"] == st["num_kron_leaves"] == 49
    assert st["mults"] - st["num_z_scalings"] == 1366 ** 2
    assert st["separable_mults"] - st["num_z_scalings"] == 2 * 1366 * 64 == 174848


def test_non_products_and_cross_axis_stages_keep_dense_leaves():
    """A stage that mixes the axes (the transposition (k, l) -> (l, k) of a square grid),
    edge weights that differ between rows, a non-product graph: no Kronecker leaves, the plan
    as given."""
    g = wl.grid(6, 6)
    tr = np.arange(36).reshape(6, 6).T.reshape(-1).astype(np.int32)
    g.stages = [tr]
    plan = G.Plan.from_graph(g)
    assert plan.info()["num_kron_leaves"] == 0
    lam_o, _ = O.gft(O.laplacian_of(g))
    np.testing.assert_allclose(plan.eigenvalues(), lam_o, atol=1e-10)
    h = wl.grid(4, 4)
    w = h.weight.copy()
    w[0] = 2.0                                # one row's edge differs from the other rows'
    h = wl._graph(16, np.stack([h.src, h.dst], 1), w, stages=[], name="grid_w")
    assert G.Plan.from_graph(h).info()["num_kron_leaves"] == 0
    assert G.Plan.from_graph(wl.config3_graph()).info()["num_kron_leaves"] == 0
    assert G.Plan.from_graph(wl.cycle(16)).info()["num_kron_leaves"] == 0


def test_normalized_laplacian_of_regular_products():
    """Sec. II-B: D^{-1/2} L D^{-1/2} of a product of regular factors (cycles: every node of
    weighted degree 2w) is L / (d_a + d_b): the product plan's basis with the eigenvalues
    scaled, pinned against the oracle's normalized Laplacian of the explicit product graph;
    a product with a non-regular factor (a path) is refused."""
    ga = wl.cycle(6)
    gb = wl._graph(8, [(i, (i + 1) % 8) for i in range(8)], [0.5] * 8, stages=[wl.reversal(8)], name="cycle_w")
    plan = G.gft_plan_product(ga, gb, laplacian="normalized")
    g = wl.cartesian_product(ga, gb)
    lam, U = O.gft(O.normalized_laplacian_of(g))
    np.testing.assert_allclose(plan.eigenvalues(), lam, atol=1e-12)
    Uh = plan.basis()
    Ua, sv = O.align(U, Uh, lam)
    assert sv > 1 - 1e-9
    X = wl.gaussian(9, g.n, wl.rng_for(9, g.n, 5), dtype=np.float64)
    assert O.relative_error(plan.apply_host(X, 0), O.forward(X, Ua)) <= 1e-10
    with pytest.raises(G.GFTError) as e:
        G.gft_plan_product(wl.path(5), ga, laplacian="normalized")
    assert e.value.status_name == "GFT_ERR_UNSUPPORTED"
