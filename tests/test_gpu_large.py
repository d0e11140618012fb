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
from tests.gpu_helpers import aligned_oracle_basis, device, to_np, torch
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


@pytest.mark.parametrize("precision", ["fp32", "bf16", "split_bf16"])
def test_config5a_grid64_sampled(precision):
    """64 x 64 grid (n = 4096, 12 stages, 49 leaf blocks) on the large engine in every block
    precision: sampled signals, every coefficient compared with the aligned oracle."""
    dev = device()
    g = wl.config5a_graph()
    plan = G.Plan.from_graph(g, engine="large", precision=precision)
    st = plan.info()
    assert st["num_blocks"] == 49 and st["max_block"] == 1024 and st["num_stages"] == 12
    assert plan.engine() == "large"
    X = wl.gaussian(384, g.n, wl.rng_for(5, 1))
    Uplan = plan.basis()
    _, Ua = aligned_oracle_basis(g, Uplan, sv_tol=1e-8)
    x = torch.from_numpy(X).to(dev)
    y = plan.forward(x)
    ref = O.forward(X.astype(np.float64), Ua)
    err = O.relative_error(to_np(y), ref)
    assert err <= TOL[precision], f"{precision}: forward relative error {err:.3e}"
    if precision == "bf16":
        assert err > 1e-5, "BF16 error suspiciously small: blocks may not run in BF16"
    C32 = ref.astype(np.float32)
    xr = plan.inverse(torch.from_numpy(C32).to(dev))
    err_i = O.relative_error(to_np(xr), O.inverse(C32.astype(np.float64), Ua))
    assert err_i <= TOL[precision], f"{precision}: inverse relative error {err_i:.3e}"
    # the GPU applies the plan's basis: spot-check 64 unit vectors
    idx = np.arange(0, g.n, 64)
    E = torch.zeros((len(idx), g.n), device=dev)
    E[torch.arange(len(idx)), torch.from_numpy(idx).to(dev)] = 1.0
    rows = to_np(plan.forward(E))
    assert np.abs(rows - Uplan[idx]).max() <= BASIS_TOL[precision]


def test_large_engine_ragged_and_empty():
    """Signal counts that leave partial GEMM tiles (1, 127, 129) against the aligned oracle."""
    dev = device()
    g = wl.config5b_graph()
    plan = G.Plan.from_graph(g)
    _, Ua = aligned_oracle_basis(g, plan.basis(), sv_tol=1e-9)
    for S in (1, 127, 129):
        X = wl.gaussian(S, g.n, wl.rng_for(5, 3, S))
        y = to_np(plan.forward(torch.from_numpy(X).to(dev)))
        ref = O.forward(X.astype(np.float64), Ua)
        assert O.relative_error(y, ref) <= TOL["fp32"]
        assert O.max_row_relative_error(y, ref) <= 4 * TOL["fp32"]
        xr = to_np(plan.inverse(torch.from_numpy(ref.astype(np.float32)).to(dev)))
        assert O.relative_error(xr, O.inverse(ref.astype(np.float32).astype(np.float64), Ua)) <= TOL["fp32"]
    assert plan.forward(torch.zeros((0, g.n), device=dev)).shape == (0, g.n)
