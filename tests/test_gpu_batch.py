"""Mixed batches of uneven graphs in one persistent launch (gft_forward_batch / _inverse_batch).

Config 4's families (paths, cycles, grids, random bipartite with an imposed pairing), each
graph with its own signal count, packed back to back in one buffer.  Every graph's slice
is checked against the FP64 oracle; the batch must also match single-graph plans of the
generic engine, leave memory past `total_elements` untouched, skip empty graphs, and give
the same result when replayed from a captured graph.
"""
import numpy as np
import pytest

import paper_1907_07875_amd as G
import workloads as wl
from oracle import gft_oracle as O
from tests.gpu_helpers import aligned_oracle_basis, device, to_np, torch

pytestmark = pytest.mark.gpu


def _pack(graphs, counts, rng):
    xs = [wl.gaussian(int(s), g.n, rng) for g, s in zip(graphs, counts)]
    flat = np.concatenate([x.reshape(-1) for x in xs]) if xs else np.zeros(0, np.float32)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return xs, flat, off


def _slices(graphs, counts):
    pos = 0
    for g, s in zip(graphs, counts):
        yield pos, pos + int(s) * g.n
        pos += int(s) * g.n


def _check_against_oracle(plan, graphs, counts, xs, y, tol=1e-5):
    worst = 0.0
    for i, ((a, b), g, x) in enumerate(zip(_slices(graphs, counts), graphs, xs)):
        if b == a:
            continue
        _, Ua = aligned_oracle_basis(g, plan.basis(i), sv_tol=1e-9)
        err = O.relative_error(y[a:b].reshape(-1, g.n), O.forward(x.astype(np.float64), Ua))
        worst = max(worst, err)
        assert err <= tol, f"graph {i} ({g.name}{g.n}): relative error {err:.3e}"
    return worst


def test_config4_mixed_batch_forward_inverse():
    dev = device()
    rng = wl.rng_for(4, 1)
    graphs = wl.config4_graphs(wl.rng_for(4))
    counts = wl.config4_signal_counts(len(graphs), rng, lo=16, hi=600)
    counts[[3, 50, 100]] = 0                       # empty graphs inside the batch
    plan = G.gft_plan_batch(graphs)
    xs, flat, off = _pack(graphs, counts, rng)
    x = torch.from_numpy(flat).to(dev)
    offs = torch.from_numpy(off).to(dev)
    y = G.gft_forward_batch(plan, x, offs)
    yn = to_np(y)
    _check_against_oracle(plan, graphs, counts, xs, yn)
    xr = to_np(G.gft_inverse_batch(plan, y, offs))
    assert O.relative_error(xr, flat.astype(np.float64)) <= 2e-5


def test_config4_bench_counts_sampled():
    """The benchmark's mixed batch as timed: all 146 graphs with their log-uniform counts of
    256..65536 signals (about 67 M values), one forward and one inverse launch.  Per graph,
    sampled rows (first, last and 28 drawn) against the aligned oracle, forward and inverse
    (the inverse of the GPU's own coefficients against the oracle's inverse of them), and the
    energy of every graph's slice."""
    dev = device()
    graphs = wl.config4_graphs(wl.rng_for(4))
    counts = wl.config4_signal_counts(len(graphs), wl.rng_for(4, 1))
    assert counts.min() >= 256 and counts.max() <= 65536
    rng = wl.rng_for(4, 2)
    xs = [wl.gaussian(int(s), g.n, rng) for g, s in zip(graphs, counts)]
    flat = np.concatenate([x.reshape(-1) for x in xs])
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    plan = G.gft_plan_batch(graphs)
    x = torch.from_numpy(flat).to(dev)
    offs = torch.from_numpy(off).to(dev)
    y = G.gft_forward_batch(plan, x, offs)
    xr = G.gft_inverse_batch(plan, y, offs)
    torch.cuda.synchronize()
    pick = wl.rng_for(4, 8)
    for i, ((a, b), g, X) in enumerate(zip(_slices(graphs, counts), graphs, xs)):
        S = int(counts[i])
        rows = np.unique(np.r_[0, 1, S - 2, S - 1, pick.choice(S, 28, replace=False)])
        yv = y[a:b].view(S, g.n)
        Yg = to_np(yv[torch.from_numpy(rows).to(dev)])
        Xg = to_np(xr[a:b].view(S, g.n)[torch.from_numpy(rows).to(dev)])
        _, Ua = aligned_oracle_basis(g, plan.basis(i), sv_tol=1e-9)
        ref = O.forward(X[rows].astype(np.float64), Ua)
        err = O.relative_error(Yg, ref)
        assert err <= 1e-5 and O.max_row_relative_error(Yg, ref) <= 1e-5, f"graph {i} ({g.name}{g.n}): {err:.3e}"
        ref_i = O.inverse(Yg, Ua)
        assert O.relative_error(Xg, ref_i) <= 1e-5, f"graph {i} ({g.name}{g.n}): inverse"
        e_in = float(torch.sum(x[a:b].double() ** 2))
        e_out = float(torch.sum(y[a:b].double() ** 2))
        assert abs(e_out - e_in) <= 1e-5 * e_in, f"graph {i}: energy {e_in} -> {e_out}"


def _batch_engine(g):
    """The engine a batch plan runs graph g on: the register-butterfly forms the batch kernel
    compiles (one stage with sides of at most 48 nodes, or two stages on 16- or 32-slot
    sides: the test's two-stage graphs have n <= 100 exactly then), else the LDS program."""
    try:
        p = G.Plan.from_graph(g, engine="butterfly")
        p.prepare()
    except G.GFTError:
        return "generic"
    if len(g.stages) == 1:
        phi = np.asarray(g.stages[0])
        fixed = int(np.sum(phi == np.arange(g.n)))
        pairs = (g.n - fixed) // 2
        return "butterfly" if pairs + fixed <= 48 else "generic"
    return "butterfly" if len(g.stages) == 2 and g.n <= 100 else "generic"   # <= 32-slot sides


@pytest.mark.parametrize("direction", ["forward", "inverse"])
def test_batch_matches_single_graph_plans(direction):
    """Each graph's slice of a mixed batch equals its single-graph plan: bit for bit on the
    register-butterfly engine (the same tile loop), to rounding on the LDS-program engine;
    with the generic engine forced the whole batch runs LDS programs and matches too."""
    dev = device()
    rng = wl.rng_for(4, 2)
    graphs = [wl.path(7), wl.path(8), wl.grid(8, 8), wl.config3_graph(), wl.cycle(13), wl.path(64),
              wl.symmetric_bipartite(72, wl.rng_for(4, 72)), wl.grid(5, 5), wl.cycle(48), wl.path(44),
              wl.symmetric_bipartite(40, wl.rng_for(4, 40)), wl.cycle(22), wl.path(90),
              wl.symmetric_bipartite(120, wl.rng_for(4, 120)), wl.grid(7, 7), wl.grid(9, 9)]
    counts = np.array([1, 17, 300, 47, 16, 1000, 33, 5, 129, 77, 250, 3, 61, 40, 45, 70])
    engines = [_batch_engine(g) for g in graphs]
    assert engines.count("butterfly") >= 12 and engines.count("generic") >= 2, engines
    xs, flat, off = _pack(graphs, counts, rng)
    offs = torch.from_numpy(off).to(dev)
    apply = G.gft_forward_batch if direction == "forward" else G.gft_inverse_batch
    for forced in ("auto", "generic"):
        plan = G.gft_plan_batch(graphs, engine=forced)
        y = to_np(apply(plan, torch.from_numpy(flat).to(dev), offs))
        for (a, b), g, xg, eng in zip(_slices(graphs, counts), graphs, xs, engines):
            eng = "generic" if forced == "generic" else eng
            single = G.Plan.from_graph(g, engine=eng)
            xt = torch.from_numpy(xg).to(dev)
            ys = to_np(single.forward(xt) if direction == "forward" else single.inverse(xt)).reshape(-1)
            if eng == "butterfly":
                assert np.array_equal(y[a:b], ys), f"{g.name}{g.n}: batch register phase differs"
            else:
                np.testing.assert_allclose(y[a:b], ys, rtol=0, atol=1e-6 * max(1.0, np.abs(ys).max()))


def test_batch_respects_total_elements_and_empty():
    dev = device()
    rng = wl.rng_for(4, 3)
    graphs = [wl.path(8), wl.grid(4, 4), wl.cycle(12)]
    counts = np.array([40, 0, 30])
    plan = G.gft_plan_batch(graphs)
    xs, flat, off = _pack(graphs, counts, rng)
    x = torch.from_numpy(flat).to(dev)
    sentinel = 12345.0
    y = torch.full_like(x, sentinel)
    # claim a buffer that ends inside the last graph: that graph must be skipped
    short = 40 * 8 + 10
    assert G.load_library().gft_forward_batch(
        plan.handle, G.ctypes.c_void_p(x.data_ptr()), G.ctypes.c_void_p(y.data_ptr()),
        G.ctypes.c_void_p(torch.from_numpy(off).to(dev).data_ptr()), short,
        G._stream_ptr(None)) == 0
    torch.cuda.synchronize()
    yn = to_np(y)
    assert np.all(yn[40 * 8:] == sentinel)
    _, Ua = aligned_oracle_basis(graphs[0], plan.basis(0), sv_tol=1e-9)
    assert O.relative_error(yn[:320].reshape(-1, 8), O.forward(xs[0].astype(np.float64), Ua)) <= 1e-5
    # zero elements is a no-op
    assert G.load_library().gft_forward_batch(plan.handle, None, None, None, 0, None) == 0


def test_batch_plan_rejected_by_single_apply_and_vice_versa():
    dev = device()
    plan = G.gft_plan_batch([wl.path(8), wl.path(9)])
    with pytest.raises(ValueError):
        G.gft_forward(plan, torch.zeros((4, 8), device=dev))
    single = G.Plan.from_graph(wl.path(8))
    with pytest.raises(ValueError):
        G.gft_forward_batch(single, torch.zeros(32, device=dev),
                            torch.zeros(2, dtype=torch.int64, device=dev))


@pytest.mark.parametrize("precision", ["bf16", "split_bf16"])
def test_batch_reduced_precision(precision):
    dev = device()
    rng = wl.rng_for(4, 4)
    graphs = [wl.config3_graph(), wl.grid(8, 8), wl.cycle(31), wl.symmetric_bipartite(56, wl.rng_for(4, 56))]
    counts = np.array([500, 300, 200, 100])
    plan = G.gft_plan_batch(graphs, precision=precision)
    xs, flat, off = _pack(graphs, counts, rng)
    y = to_np(G.gft_forward_batch(plan, torch.from_numpy(flat).to(dev), torch.from_numpy(off).to(dev)))
    _check_against_oracle(plan, graphs, counts, xs, y, tol=2e-2 if precision == "bf16" else 1e-5)


def test_captured_graph_replays_equal_eager():
    """hipGraph capture of batch and single-graph applies; every replay equals eager."""
    dev = device()
    rng = wl.rng_for(4, 5)
    graphs = [wl.path(16), wl.grid(8, 8), wl.config3_graph()]
    counts = np.array([100, 2000, 333])
    bplan = G.gft_plan_batch(graphs)
    splan = G.Plan.from_graph(wl.grid(8, 8))
    bplan.prepare()
    splan.prepare()
    _, flat, off = _pack(graphs, counts, rng)
    x = torch.from_numpy(flat).to(dev)
    offs = torch.from_numpy(off).to(dev)
    xs = torch.from_numpy(wl.gaussian(5000, 64, rng)).to(dev)
    yb = torch.empty_like(x)
    ys = torch.empty_like(xs)
    xr = torch.empty_like(xs)
    eager_b = G.gft_forward_batch(bplan, x, offs).clone()
    eager_s = splan.forward(xs).clone()
    eager_r = splan.inverse(eager_s).clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        G.gft_forward_batch(bplan, x, offs, out=yb)      # warm-up on the side stream
        splan.forward(xs, out=ys)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        G.gft_forward_batch(bplan, x, offs, out=yb)
        splan.forward(xs, out=ys)
        splan.inverse(ys, out=xr)
    for _ in range(3):
        yb.zero_()
        ys.zero_()
        xr.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(yb, eager_b)
        assert torch.equal(ys, eager_s)
        assert torch.equal(xr, eager_r)
        _ = (xs * 2).sum().item()                        # unrelated eager work between replays


def test_captured_graph_other_engines():
    """hipGraph capture of the generic engine, the padded one-stage butterfly with BF16
    blocks and a product plan in one graph; eager work between replays, every replay equals
    the eager result bit for bit."""
    dev = device()
    rng = wl.rng_for(4, 6)
    gen_plan = G.Plan.from_graph(wl.grid(11, 11), engine="generic")
    bf_plan = G.Plan.from_graph(wl.config3_graph(), precision="bf16")
    pr_plan = G.Plan.from_product(wl.path(16), wl.path_recursive(16))
    plans = [gen_plan, bf_plan, pr_plan]
    for p in plans:
        p.prepare()
    assert gen_plan.engine() == "generic" and bf_plan.engine() == "butterfly" and pr_plan.engine() == "product"
    xs = [torch.from_numpy(wl.gaussian(S, p.n, rng)).to(dev) for S, p in zip((1234, 4000, 777), plans)]
    ys = [torch.empty_like(x) for x in xs]
    eager = [p.forward(x).clone() for p, x in zip(plans, xs)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for p, x, y in zip(plans, xs, ys):
            p.forward(x, out=y)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for p, x, y in zip(plans, xs, ys):
            p.forward(x, out=y)
    for _ in range(3):
        for y in ys:
            y.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for y, e in zip(ys, eager):
            assert torch.equal(y, e)
        # eager work between replays, on the same buffers' neighbours
        for p, x in zip(plans, xs):
            p.inverse(p.forward(x))
        torch.cuda.synchronize()
