"""GPU parity of product-graph plans (separable GFT of Cartesian products) against the FP64
oracle of the explicit product graph, through the C ABI.

The oracle's eigenbasis of the product Laplacian is rotated onto the plan's basis inside
each eigenvalue cluster (products of symmetric factors have many repeated eigenvalues
lambda_p + mu_q = lambda_q + mu_p); every coefficient of every signal is compared.  FP32
tolerance: relative error <= 1e-5.  The 64 x 64 grid at the benchmark's 65536 signals is
checked on sampled signals against the oracle's eigenbasis of the 4096-node grid.
"""
import numpy as np
import pytest

import paper_1907_07875_amd as G
import workloads as wl
from oracle import gft_oracle as O
from tests.gpu_helpers import aligned_oracle_basis, device, gpu_basis, to_np, torch

pytestmark = pytest.mark.gpu

TOL = 1e-5

PRODUCTS = [
    (wl.path(8), wl.path(8)),                                              # 16 x 16 tiles
    (wl.path(6), wl.path(5)),                                              # n = 30: scalar I/O
    (wl.weighted_symmetric_path(12, wl.rng_for(9, 12)), wl.cycle(7)),      # self-loops
    (wl.path_recursive(16), wl.config3_graph()),                           # 16 x 32
    (wl.path(40), wl.path(24)),                                            # 64 x 32
    (wl.cycle(20), wl.path(50)),                                           # 32 x 64
    (wl.symmetric_bipartite(24, wl.rng_for(4, 24)), wl.path(3)),           # 32 x 16
]


def _ids(pair):
    return f"{pair[0].name}{pair[0].n}x{pair[1].name}{pair[1].n}"


@pytest.mark.parametrize("S", [1, 7, 1000])
@pytest.mark.parametrize("pair", PRODUCTS, ids=_ids)
def test_product_parity(pair, S):
    dev = device()
    ga, gb = pair
    plan = G.Plan.from_product(ga, gb)
    assert plan.engine() == "product" and plan.tiles() == (1, 1)
    g = wl.cartesian_product(ga, gb)
    lam_o, U_o = O.gft(O.laplacian_of(g))
    Uplan = plan.basis()
    Ua, min_sv = O.align(U_o, Uplan, lam_o)
    assert min_sv > 1 - 1e-9
    assert np.abs(gpu_basis(plan, dev) - Uplan).max() <= 2e-6
    X = wl.gaussian(S, g.n, wl.rng_for(9, g.n, S, 3))
    x = torch.from_numpy(X).to(dev)
    y = plan.forward(x)
    C_ref = O.forward(X.astype(np.float64), Ua)
    err = O.relative_error(to_np(y), C_ref)
    assert err <= TOL, f"forward relative error {err:.3e}"
    C32 = C_ref.astype(np.float32)
    xr = plan.inverse(torch.from_numpy(C32).to(dev))
    err_i = O.relative_error(to_np(xr), O.inverse(C32.astype(np.float64), Ua))
    assert err_i <= TOL, f"inverse relative error {err_i:.3e}"
    assert O.relative_error(to_np(plan.inverse(y)), X.astype(np.float64)) <= 2 * TOL


@pytest.mark.parametrize("precision,tol", [("split_bf16", 1e-5), ("bf16", 2e-2)])
@pytest.mark.parametrize("pair", [PRODUCTS[0], PRODUCTS[2], PRODUCTS[4], (wl.path_recursive(64), wl.path_recursive(64))],
                         ids=_ids)
def test_product_reduced_precision(pair, precision, tol):
    """BF16 and split-BF16 factor products (16x16x16 BF16 MFMA, FP32 accumulation) against
    the oracle; the split form reaches the FP32 tolerance."""
    dev = device()
    ga, gb = pair
    plan = G.Plan.from_product(ga, gb, precision=precision)
    g = wl.cartesian_product(ga, gb)
    _, Ua = aligned_oracle_basis(g, plan.basis(), sv_tol=1e-8)
    ref = lambda X: O.forward(X, Ua)          # noqa: E731
    X = wl.gaussian(333, g.n, wl.rng_for(9, g.n, 21))
    y = plan.forward(torch.from_numpy(X).to(dev))
    err = O.relative_error(to_np(y), ref(X.astype(np.float64)))
    assert err <= tol, f"{precision}: forward relative error {err:.3e}"
    if precision == "bf16":
        assert err > 1e-5, "BF16 error suspiciously small: products may not run in BF16"
    xr = plan.inverse(y)
    assert O.relative_error(to_np(xr), X.astype(np.float64)) <= 2 * tol


def test_product_grid64_full_size_sampled():
    """64 x 64 grid as path64 x path64 (each axis with its halving reversal stages), 65536
    signals in one launch: sampled rows against the aligned oracle, round trip on all."""
    dev = device()
    ga = wl.path_recursive(64)
    plan = G.Plan.from_product(ga, ga)
    S, n = 65536, 4096
    _, Ua = aligned_oracle_basis(wl.cartesian_product(ga, ga), plan.basis(), sv_tol=1e-8)
    X = wl.gaussian(S, n, wl.rng_for(5, 7))
    x = torch.from_numpy(X).to(dev)
    y = plan.forward(x)
    rows = np.sort(wl.rng_for(5, 8).choice(S, 256, replace=False))
    Yh = O.forward(X[rows].astype(np.float64), Ua)
    assert O.relative_error(to_np(y[torch.from_numpy(rows).to(dev)]), Yh) <= TOL
    xr = plan.inverse(y)
    assert O.relative_error(to_np(xr[torch.from_numpy(rows).to(dev)]), X[rows].astype(np.float64)) <= 2 * TOL
    # energy of every signal is kept (U orthogonal)
    e_in = (x.double() ** 2).sum(dim=1)
    e_out = (y.double() ** 2).sum(dim=1)
    assert torch.max(torch.abs(e_out - e_in) / e_in).item() <= 1e-5


# ------------------------------------------------- gft_plan with Kronecker leaves (separable)

@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("split_bf16", 1e-5), ("bf16", 2e-2)])
def test_grid64_twelve_stage_plan_runs_separably(precision, tol):
    """The 64 x 64 grid planned by gft_plan with its 12 halving stages: its 49 leaf blocks
    have Kronecker bases, so the automatic engine choice runs it separably (U_a^T X U_b) in
    place of the large engine's dense leaf GEMMs.  Sampled signals of a 65536-signal launch
    against the aligned oracle of the 4096-node grid, forward and inverse."""
    dev = device()
    g = wl.config5a_graph()
    plan = G.Plan.from_graph(g, precision=precision)
    assert plan.engine() == "product" and plan.info()["num_kron_leaves"] == 49
    _, Ua = aligned_oracle_basis(g, plan.basis(), sv_tol=1e-8)
    S = 65536
    X = wl.gaussian(S, g.n, wl.rng_for(5, 17))
    x = torch.from_numpy(X).to(dev)
    y = plan.forward(x)
    rows = np.unique(np.r_[0, S - 1, wl.rng_for(5, 18).choice(S, 190, replace=False)])
    ri = torch.from_numpy(rows).to(dev)
    ref = O.forward(X[rows].astype(np.float64), Ua)
    err = O.relative_error(to_np(y[ri]), ref)
    assert err <= tol, f"{precision}: forward relative error {err:.3e}"
    if precision == "bf16":
        assert err > 1e-5, "BF16 error suspiciously small: products may not run in BF16"
    yi = y[ri].contiguous()
    xr = to_np(plan.inverse(yi))
    assert O.relative_error(xr, O.inverse(to_np(yi), Ua)) <= tol
    # the same plan on the large engine applies the same basis
    big = G.Plan.from_graph(g, precision=precision, engine="large")
    assert big.engine() == "large"
    yl = to_np(big.forward(x[ri].contiguous()))
    assert O.relative_error(yl, ref) <= tol


@pytest.mark.parametrize("S", [1, 37, 1000])
@pytest.mark.parametrize("pair", [(wl.path(8), wl.path(8)), (wl.path_recursive(16), wl.path_recursive(16)),
                                  (wl.weighted_symmetric_path(12, wl.rng_for(9, 12)), wl.path(7)),
                                  (wl.config3_graph(), wl.weighted_symmetric_path(9, wl.rng_for(9, 9))),
                                  (wl.path(5), wl.cycle(12))], ids=_ids)
def test_separable_engine_forced_on_staged_products(pair, S):
    """Staged products planned by gft_plan, forced onto the separable engine (engine 4):
    every coefficient against the aligned oracle, forward, inverse and round trip; the
    engine's basis equals the plan's FP64 basis."""
    dev = device()
    ga, gb = pair
    g = wl.product_with_stages(ga, gb)
    plan = G.gft_plan(g.n, g.src, g.dst, g.weight, g.self_loop, g.stages, engine=4)
    assert plan.engine() == "product"
    Uplan = plan.basis()
    _, Ua = aligned_oracle_basis(g, Uplan, sv_tol=1e-9)
    assert np.abs(gpu_basis(plan, dev) - Uplan).max() <= 2e-6
    X = wl.gaussian(S, g.n, wl.rng_for(9, g.n, S, 31))
    x = torch.from_numpy(X).to(dev)
    y = plan.forward(x)
    C_ref = O.forward(X.astype(np.float64), Ua)
    assert O.relative_error(to_np(y), C_ref) <= TOL
    C32 = C_ref.astype(np.float32)
    xr = plan.inverse(torch.from_numpy(C32).to(dev))
    assert O.relative_error(to_np(xr), O.inverse(C32.astype(np.float64), Ua)) <= TOL
    assert O.relative_error(to_np(plan.inverse(y)), X.astype(np.float64)) <= 2 * TOL


def test_separable_engine_refused_without_kronecker_leaves():
    dev = device()
    g = wl.config3_graph()
    plan = G.gft_plan(g.n, g.src, g.dst, g.weight, g.self_loop, g.stages, engine=4)
    with pytest.raises(G.GFTError) as e:
        plan.forward(torch.zeros((4, g.n), device=dev))
    assert e.value.status_name == "GFT_ERR_UNSUPPORTED"
    # the 8x8 grid has Kronecker leaves but keeps the register butterfly when not forced
    assert G.Plan.from_graph(wl.config2_graph()).engine() == "butterfly"


FORM_PAIRS = [(wl.path_recursive(64), wl.path_recursive(64)),         # one fragment set, 6 of 16 tiles
              (wl.path_recursive(32), wl.path_recursive(64)),
              (wl.path_recursive(16), wl.weighted_symmetric_path(40, wl.rng_for(9, 40))),
              (wl.path(5), wl.cycle(12))]                               # V_Z nodes, padded 16 x 16


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("split_bf16", 1e-5), ("bf16", 2e-2)])
@pytest.mark.parametrize("form", ["dense", "staged"])
@pytest.mark.parametrize("pair", FORM_PAIRS, ids=_ids)
def test_separable_factor_forms(pair, form, precision, tol, monkeypatch):
    """Both forms of the factors on the separable engine: dense factor GFTs, and staged
    factors (Haar stages as add/sub on the tile, leaf blocks as block-diagonal matrices
    whose zero tiles are skipped), forced through GFT_PRODUCT_FORM; every coefficient
    against the aligned oracle, forward, inverse of the oracle's coefficients, round trip."""
    monkeypatch.setenv("GFT_PRODUCT_FORM", form)
    dev = device()
    ga, gb = pair
    g = wl.product_with_stages(ga, gb)
    plan = G.gft_plan(g.n, g.src, g.dst, g.weight, g.self_loop, g.stages, engine="product",
                      precision=precision)
    plan.prepare()
    assert plan.engine() == "product"
    _, Ua = aligned_oracle_basis(g, plan.basis(), sv_tol=1e-8)
    X = wl.gaussian(517, g.n, wl.rng_for(9, g.n, 41))
    x = torch.from_numpy(X).to(dev)
    y = plan.forward(x)
    C_ref = O.forward(X.astype(np.float64), Ua)
    err = O.relative_error(to_np(y), C_ref)
    assert err <= tol, f"{form} {precision}: forward relative error {err:.3e}"
    C32 = C_ref.astype(np.float32)
    xr = plan.inverse(torch.from_numpy(C32).to(dev))
    err_i = O.relative_error(to_np(xr), O.inverse(C32.astype(np.float64), Ua))
    assert err_i <= tol, f"{form} {precision}: inverse relative error {err_i:.3e}"
    assert O.relative_error(to_np(plan.inverse(y)), X.astype(np.float64)) <= 2 * tol
