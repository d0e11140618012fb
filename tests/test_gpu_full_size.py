"""Parity at the benchmark's full sizes, in the launch the bench times: the 25-node skeleton
with 16384 x 3 x 300 = 14,745,600 signals (one launch over 1.47 GB) and the 1024-node
weighted path with 65536 signals on the large engine.  Every signal is computed on the GPU;
a seeded sample of rows is checked against the FP64 oracle (basis aligned per eigenvalue
cluster), and properties that hold for every row are checked on all of them (FP32 blocks:
per-signal energy, U being orthogonal).  Inputs are i.i.d. N(0,1) of the workloads' shapes:
parity does not depend on the value distribution."""
import numpy as np
import pytest

import paper_1907_07875_amd as G
import workloads as wl
from oracle import gft_oracle as O
from tests.gpu_helpers import aligned_oracle_basis, device, torch

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16": 2e-2, "split_bf16": 1e-5}


def _gaussian_chunked(S, n, rng, chunk=1 << 20):
    X = np.empty((S, n), dtype=np.float32)
    for i in range(0, S, chunk):
        X[i:i + chunk] = rng.standard_normal((min(chunk, S - i), n)).astype(np.float32)
    return X


def _sampled_parity(g, plan, X, y, xr, tol, nrows, seed):
    lam, Ua = aligned_oracle_basis(g, plan.basis(), sv_tol=1e-9)
    rows = np.sort(wl.rng_for(*seed).choice(X.shape[0], nrows, replace=False))
    ri = torch.from_numpy(rows).to(y.device)
    Xs = X[rows].astype(np.float64)
    err = O.relative_error(y[ri].double().cpu().numpy(), O.forward(Xs, Ua))
    assert err <= tol, f"{g.name}: forward relative error {err:.3e} on {nrows} sampled rows"
    rt = O.relative_error(xr[ri].double().cpu().numpy(), Xs)
    assert rt <= 2 * tol, f"{g.name}: round trip error {rt:.3e}"
    return err


def _energy_all_rows(x, y, tol):
    # per-signal ||y||^2 against ||x||^2, in FP64 chunk by chunk
    worst = 0.0
    for i in range(0, x.shape[0], 1 << 21):
        ex = (x[i:i + (1 << 21)].double() ** 2).sum(dim=1)
        ey = (y[i:i + (1 << 21)].double() ** 2).sum(dim=1)
        worst = max(worst, torch.max(torch.abs(ey - ex) / ex).item())
    assert worst <= tol, f"energy not kept: worst relative change {worst:.3e}"


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_config3_skeleton_full_size(precision):
    dev = device()
    g = wl.config3_graph()
    plan = G.Plan.from_graph(g, precision=precision)
    S = 16384 * 3 * 300
    X = _gaussian_chunked(S, g.n, wl.rng_for(3, 7))
    x = torch.from_numpy(X).to(dev)
    y = plan.forward(x)
    xr = plan.inverse(y)
    torch.cuda.synchronize()
    _sampled_parity(g, plan, X, y, xr, TOL[precision], 4096, (3, 8))
    if precision == "fp32":
        _energy_all_rows(x, y, 1e-5)
    del x, y, xr
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", ["fp32", "split_bf16", "bf16"])
def test_config5b_weighted_path_full_size(precision):
    dev = device()
    g = wl.config5b_graph()
    plan = G.Plan.from_graph(g, precision=precision)
    assert plan.engine() == "large"
    S = 65536
    X = _gaussian_chunked(S, g.n, wl.rng_for(5, 9))
    x = torch.from_numpy(X).to(dev)
    y = plan.forward(x)
    xr = plan.inverse(y)
    torch.cuda.synchronize()
    _sampled_parity(g, plan, X, y, xr, TOL[precision], 512, (5, 10))
    if precision != "bf16":
        _energy_all_rows(x, y, 1e-5)


def test_grid8x8_beyond_32bit_offsets():
    """The 8x8 grid on 2^26 + 5 signals: 4,294,967,616 values per array (byte offsets past
    16 GiB, element offsets past 2^32) in one butterfly launch.  Inputs come from torch's
    seeded generator on the device (no library code involved); sampled rows are read back
    and checked against the oracle, the last (partial) tile included, and the energy of
    every signal is checked on the device."""
    dev = device()
    g = wl.grid(8, 8)
    plan = G.Plan.from_graph(g)
    assert plan.engine() == "butterfly"
    S = (1 << 26) + 5
    gen = torch.Generator(device=dev).manual_seed(26)
    x = torch.randn((S, g.n), device=dev, dtype=torch.float32, generator=gen)
    y = plan.forward(x)
    torch.cuda.synchronize()
    lam, Ua = aligned_oracle_basis(g, plan.basis(), sv_tol=1e-9)
    rows = np.unique(np.r_[wl.rng_for(26, 1).choice(S, 1024, replace=False), np.arange(S - 40, S)])
    ri = torch.from_numpy(rows).to(dev)
    Xs = x[ri].double().cpu().numpy()
    err = O.relative_error(y[ri].double().cpu().numpy(), O.forward(Xs, Ua))
    assert err <= TOL["fp32"], f"forward relative error {err:.3e}"
    _energy_all_rows(x, y, 1e-5)
    xr = plan.inverse(y)
    rt = O.relative_error(xr[ri].double().cpu().numpy(), Xs)
    assert rt <= 2 * TOL["fp32"], f"round trip error {rt:.3e}"
    del x, y, xr
    torch.cuda.empty_cache()


def test_batch_beyond_32bit_offsets():
    """One batch launch over 4.97 G values per array (8x8 grid and 48-node path on the
    register phase, then a 12x12 grid on its LDS program whose data runs past element
    2^32): sampled rows of every graph, its last rows included, against the oracle."""
    dev = device()
    graphs = [wl.grid(8, 8), wl.path(48), wl.grid(12, 12)]
    counts = [1 << 25, 1 << 25, (1 << 23) + 3]
    bp = G.gft_plan_batch(graphs)
    total = sum(c * g.n for c, g in zip(counts, graphs))
    gen = torch.Generator(device=dev).manual_seed(32)
    x = torch.randn(total, device=dev, dtype=torch.float32, generator=gen)
    off = torch.from_numpy(np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)).to(dev)
    y = G.gft_forward_batch(bp, x, off)
    xr = G.gft_inverse_batch(bp, y, off)
    torch.cuda.synchronize()
    base = 0
    for k, (g, c) in enumerate(zip(graphs, counts)):
        lam, Ua = aligned_oracle_basis(g, G.Plan.from_graph(g).basis(), sv_tol=1e-9)
        rows = np.unique(np.r_[wl.rng_for(32, k).choice(c, 256, replace=False), np.arange(c - 20, c)])
        idx = torch.from_numpy(base + rows[:, None] * g.n + np.arange(g.n)[None, :]).to(dev)
        Xs = x[idx].double().cpu().numpy()
        err = O.relative_error(y[idx].double().cpu().numpy(), O.forward(Xs, Ua))
        assert err <= TOL["fp32"], f"{g.name}{g.n}: forward relative error {err:.3e}"
        rt = O.relative_error(xr[idx].double().cpu().numpy(), Xs)
        assert rt <= 2 * TOL["fp32"], f"{g.name}{g.n}: round trip error {rt:.3e}"
        base += c * g.n
    assert base > 1 << 32
    del x, y, xr
    torch.cuda.empty_cache()


@pytest.mark.parametrize("which", ["large_wpath1024", "product_grid64"])
def test_large_and_product_beyond_32bit_offsets(which):
    """The large engine (1024-node weighted path, 2^21 + 3 signals: 2.1 G values, byte
    offsets past 8 GiB) and the product engine (64 x 64 grid, 2^20 + 1 signals: 4.3 G values)
    in one launch each: sampled rows and the last signals against the oracle."""
    dev = device()
    if which == "large_wpath1024":
        g = wl.config5b_graph()
        plan = G.Plan.from_graph(g)
        assert plan.engine() == "large"
        S = (1 << 21) + 3
    else:
        ga = wl.path_recursive(64)
        g = wl.cartesian_product(ga, ga)
        plan = G.Plan.from_product(ga, ga)
        S = (1 << 20) + 1
    gen = torch.Generator(device=dev).manual_seed(33)
    x = torch.randn((S, g.n), device=dev, dtype=torch.float32, generator=gen)
    y = plan.forward(x)
    xr = plan.inverse(y)
    torch.cuda.synchronize()
    rows = np.unique(np.r_[wl.rng_for(33, S).choice(S, 128, replace=False), np.arange(S - 4, S)])
    ri = torch.from_numpy(rows).to(dev)
    Xs = x[ri].double().cpu().numpy()
    lam, Ua = aligned_oracle_basis(g, plan.basis(), sv_tol=1e-8)
    ref = O.forward(Xs, Ua)
    err = O.relative_error(y[ri].double().cpu().numpy(), ref)
    assert err <= TOL["fp32"], f"{which}: forward relative error {err:.3e}"
    rt = O.relative_error(xr[ri].double().cpu().numpy(), Xs)
    assert rt <= 2 * TOL["fp32"], f"{which}: round trip error {rt:.3e}"
    del x, y, xr
    torch.cuda.empty_cache()
