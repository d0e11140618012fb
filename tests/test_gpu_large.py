"""Large-signal engine (Haar passes + grouped MFMA GEMM over leaf blocks) against the oracle.

Config 5: the 64 x 64 grid with LR/UD reversals recursed on the + branch (n = 4096, 12
stages, 49 leaf blocks up to 1024 nodes) and the weighted symmetric path (n = 1024, leaf
blocks 512 + 512).  Tolerances: FP32 <= 1e-5, BF16 <= 2e-2, split BF16 <= 1e-5.
"""
import numpy as np
import pytest

import paper_1907_07875_amd as G
import workloads as wl
from oracle import gft_oracle as O
from tests.gpu_helpers import device, to_np, torch
from tests.test_gpu_parity import _check_graph

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16": 2e-2, "split_bf16": 1e-5}
BASIS_TOL = {"fp32": 2e-6, "bf16": 1e-2, "split_bf16": 5e-6}


@pytest.mark.parametrize("precision", ["fp32", "bf16", "split_bf16"])
def test_config5b_weighted_path(precision):
    g = wl.config5b_graph()
    X = wl.gaussian(1500, g.n, wl.rng_for(5, 2))
    plan = G.Plan.from_graph(g, precision=precision)
    assert plan.engine() == "large"
    _check_graph(g, X, tol=TOL[precision], precision=precision, basis_tol=BASIS_TOL[precision])


@pytest.mark.parametrize("g", [wl.config3_graph(), wl.grid(8, 8), wl.cycle(13), wl.grid_recursive(8),
                               wl.symmetric_bipartite(72, wl.rng_for(4, 72))],
                         ids=lambda g: f"{g.name}{g.n}")
def test_large_engine_small_graphs(g):
    """The large engine forced on graphs the other engines also serve."""
    X = wl.gaussian(777, g.n, wl.rng_for(5, g.n))
    assert G.Plan.from_graph(g, engine="large").engine() == "large"
    _check_graph(g, X, engine="large")


def test_config5a_grid64_sampled():
    """64 x 64 grid (n = 4096): sampled signals, every coefficient compared."""
    dev = device()
    g = wl.config5a_graph()
    plan = G.Plan.from_graph(g)
    st = plan.info()
    assert st["num_blocks"] == 49 and st["max_block"] == 1024 and st["num_stages"] == 12
    assert plan.engine() == "large"
    X = wl.gaussian(384, g.n, wl.rng_for(5, 1))
    L = O.laplacian_of(g)
    lam, U = O.gft(L)
    Uplan = plan.basis()
    Ua, min_sv = O.align(U, Uplan, lam)
    assert min_sv > 1 - 1e-8
    x = torch.from_numpy(X).to(dev)
    y = plan.forward(x)
    err = O.relative_error(to_np(y), O.forward(X.astype(np.float64), Ua))
    assert err <= 1e-5, err
    xr = plan.inverse(y)
    assert O.relative_error(to_np(xr), X.astype(np.float64)) <= 2e-5
    # the GPU applies the plan's basis: spot-check 64 unit vectors
    idx = np.arange(0, g.n, 64)
    E = torch.zeros((len(idx), g.n), device=dev)
    E[torch.arange(len(idx)), torch.from_numpy(idx).to(dev)] = 1.0
    rows = to_np(plan.forward(E))
    assert np.abs(rows - Uplan[idx]).max() <= 2e-6


def test_large_engine_ragged_and_empty():
    dev = device()
    g = wl.config5b_graph()
    plan = G.Plan.from_graph(g)
    for S in (1, 127, 129):
        X = wl.gaussian(S, g.n, wl.rng_for(5, 3, S))
        y = to_np(plan.forward(torch.from_numpy(X).to(dev)))
        np.testing.assert_allclose(y, X.astype(np.float64) @ plan.basis(), atol=2e-5)
    assert plan.forward(torch.zeros((0, g.n), device=dev)).shape == (0, g.n)
