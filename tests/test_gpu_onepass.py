"""One-pass form of the large-signal engine: the first pass's values staged straight from
the input rows, the leaf-block MFMA products, and the last pass (its Haar stages and the
output order) in LDS, all in one kernel with no workspace array.

The one-pass form computes every value with the operations of the three-pass form in the
same order, so the forms agree bit for bit (GFT_LARGE_FORM forces a form); both agree with
the aligned FP64 oracle within the block precision's bound (FP32 and split BF16 <= 1e-5,
BF16 <= 2e-2).  Cases: the weighted symmetric 1024-path (two 512-node blocks of the sums and
differences of the same Haar units; the forward loads each lane's two units as two pairs of
neighbouring values, the inverse one coefficient per entry), the 1023-path (a V_Z node scaled by
sqrt 2, blocks of 512 and 511), a uniform 1000-path (its inverse loads the two blocks'
alternating coefficients in pairs), a 1000-cycle, and a 600-node path planned without a
stage (one dense block); the inverse directions stage coefficients (a copy per block) and
run the Haar stage on the results in LDS.
"""
import ctypes

import numpy as np
import pytest

import paper_1907_07875_amd as G
import workloads as wl
from oracle import gft_oracle as O
from tests.gpu_helpers import aligned_oracle_basis, device, to_np, torch

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16": 2e-2, "split_bf16": 1e-5}


def _nostage_path(n):
    rng = wl.rng_for(5, 9, n)
    edges = [(i, i + 1) for i in range(n - 1)]
    return wl._graph(n, edges, rng.uniform(0.1, 1.0, n - 1), None, [], "wpath_nostage")


GRAPHS = {
    "wpath1024": wl.config5b_graph,
    # uniform path: the sum and difference blocks' eigenvalues alternate strictly, so the
    # inverse reads each pair of neighbouring coefficients with one load (pair mode)
    "path1000": lambda: wl.path(1000),
    "wpath1023": lambda: wl.weighted_symmetric_path(1023, wl.rng_for(5, 8)),
    "cycle1000": lambda: wl.cycle(1000),
    "nostage600": lambda: _nostage_path(600),
}


def _plan(g, precision, form, monkeypatch, **kw):
    monkeypatch.setenv("GFT_LARGE_FORM", form)
    plan = G.Plan.from_graph(g, engine="large", precision=precision, autotune=False, **kw)
    plan.prepare()
    monkeypatch.delenv("GFT_LARGE_FORM")
    return plan


@pytest.mark.parametrize("precision", ["fp32", "bf16", "split_bf16"])
@pytest.mark.parametrize("name", list(GRAPHS))
def test_onepass_bit_equal_to_three_passes_and_oracle(name, precision, monkeypatch):
    dev = device()
    g = GRAPHS[name]()
    one = _plan(g, precision, "onepass", monkeypatch)
    three = _plan(g, precision, "passes", monkeypatch)
    assert one.engine() == three.engine() == "large"
    assert one.tuning()["variant"] == 2, "the plan should fit the one-pass form"
    assert three.tuning()["variant"] == 0
    S = 1001                      # not a multiple of the 64- or 48-row panels
    X = wl.gaussian(S, g.n, wl.rng_for(5, g.n, 61))
    x = torch.from_numpy(X).to(dev)
    y = one.forward(x)
    assert torch.equal(y, three.forward(x))
    xr = one.inverse(y)
    assert torch.equal(xr, three.inverse(y))
    _, Ua = aligned_oracle_basis(g, one.basis(), sv_tol=1e-8)
    ref = O.forward(X.astype(np.float64), Ua)
    assert O.relative_error(to_np(y), ref) <= TOL[precision]
    assert O.max_row_relative_error(to_np(y), ref) <= 4 * TOL[precision]
    assert O.relative_error(to_np(xr), O.inverse(to_np(y).astype(np.float64), Ua)) <= TOL[precision]


def test_onepass_source_modes():
    """The specialised ways the kernel loads a k step's inputs (OnePass::src_mode 1, 3, 4,
    5, reported by gft_plan_tuning) are exercised by the graphs above, in one direction or
    the other (mode 2, the general two-block mode, by GFT_ONEPASS_GENERAL below); the
    symmetric 1024-path loads its forward as pairs of neighbours and its inverse one
    coefficient per entry."""
    device()
    seen = {}
    cases = dict(GRAPHS)
    cases["bipartite_nosym"] = _bipartite_nosym
    for name, make in cases.items():
        kw = {"laplacian": "normalized"} if name == "bipartite_nosym" else {}
        plan = G.Plan.from_graph(make(), engine="large", precision="bf16", autotune=False, **kw)
        plan.prepare()
        t = plan.tuning()
        seen[name] = (t["onepass_fwd"], t["onepass_inv"])
    assert seen["wpath1024"] == (5, 4), seen
    modes = {m for pair in seen.values() for m in pair}
    assert {1, 3, 4, 5} <= modes, seen


@pytest.mark.parametrize("precision", ["fp32", "bf16", "split_bf16"])
def test_onepass_general_modes_agree(precision, monkeypatch):
    """GFT_ONEPASS_GENERAL=1 builds the one-pass form with its general source modes only
    (each entry's sources loaded as they are: mode 2 with two blocks); the specialised modes
    compute the same values with fewer loads, so the two agree bit for bit."""
    dev = device()
    for name in ("wpath1024", "path1000", "bipartite_nosym"):
        g = _bipartite_nosym() if name == "bipartite_nosym" else GRAPHS[name]()
        kw = {"laplacian": "normalized"} if name == "bipartite_nosym" else {}
        spec = _plan(g, precision, "onepass", monkeypatch, **kw)
        monkeypatch.setenv("GFT_ONEPASS_GENERAL", "1")
        gen = _plan(g, precision, "onepass", monkeypatch, **kw)
        monkeypatch.delenv("GFT_ONEPASS_GENERAL")
        ts, tg = spec.tuning(), gen.tuning()
        assert tg["variant"] == 2 and tg["onepass_fwd"] == 2 and tg["onepass_inv"] == 2, (name, tg)
        assert (ts["onepass_fwd"], ts["onepass_inv"]) != (2, 2), (name, ts)
        x = torch.from_numpy(wl.gaussian(1001, g.n, wl.rng_for(5, g.n, 71))).to(dev)
        y = spec.forward(x)
        assert torch.equal(y, gen.forward(x)), name
        assert torch.equal(spec.inverse(y), gen.inverse(y)), name


def _bipartite_nosym(n=400):
    """A bipartite graph with no symmetry: under the normalized Laplacian its plan has no
    left stage, n/2 right Haar units and two blocks (Sec. III), so the forward runs the right
    stage on the result slab and the inverse stages sums and differences of coefficients."""
    rng = np.random.default_rng(5)
    a = n // 2
    E = {}
    for i in range(a):
        for j in rng.choice(n - a, 6, replace=False):
            E[(i, a + int(j))] = rng.uniform(0.5, 1.5)
    for i in range(a - 1):                       # connected
        E.setdefault((i, a + i), 1.0)
        E.setdefault((i + 1, a + i), 1.0)
    edges = list(E)
    return wl._graph(n, edges, np.array([E[e] for e in edges]), None, [], "bipartite_nosym")


@pytest.mark.parametrize("precision", ["fp32", "bf16", "split_bf16"])
def test_onepass_right_haar_units(precision, monkeypatch):
    dev = device()
    g = _bipartite_nosym()
    one = _plan(g, precision, "onepass", monkeypatch, laplacian="normalized")
    three = _plan(g, precision, "passes", monkeypatch, laplacian="normalized")
    st = one.info()
    assert st["num_stages"] == 0 and st["num_right_units"] == g.n // 2 and st["num_blocks"] == 2
    assert one.tuning()["variant"] == 2
    X = wl.gaussian(777, g.n, wl.rng_for(5, g.n, 67))
    x = torch.from_numpy(X).to(dev)
    y = one.forward(x)
    assert torch.equal(y, three.forward(x))
    xr = one.inverse(y)
    assert torch.equal(xr, three.inverse(y))
    _, Ua = aligned_oracle_basis(g, one.basis(), sv_tol=1e-8, laplacian="normalized")
    assert O.relative_error(to_np(y), O.forward(X.astype(np.float64), Ua)) <= TOL[precision]
    assert O.relative_error(to_np(xr), O.inverse(to_np(y).astype(np.float64), Ua)) <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "bf16", "split_bf16"])
def test_onepass_epilogue_form_and_ragged_counts(precision, monkeypatch):
    """Signal counts around the panel heights (one partial panel, exact panels, a panel
    plus one row) and an empty batch; the GEMM-epilogue form agrees too."""
    dev = device()
    g = wl.config5b_graph()
    one = _plan(g, precision, "onepass", monkeypatch)
    three = _plan(g, precision, "passes", monkeypatch)
    epi = _plan(g, precision, "epilogue", monkeypatch)
    assert epi.tuning()["variant"] == 1 or epi.tuning()["variant"] == 0
    for S in (1, 47, 48, 49, 64, 65, 193):
        x = torch.from_numpy(wl.gaussian(S, g.n, wl.rng_for(5, 4, S))).to(dev)
        y = one.forward(x)
        assert torch.equal(y, three.forward(x)), S
        assert torch.equal(y, epi.forward(x)), S
        assert torch.equal(one.inverse(y), three.inverse(y)), S
    assert one.forward(torch.zeros((0, g.n), device=dev)).shape == (0, g.n)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("din,dout", [("bf16", "bf16"), ("bf16", "fp32"), ("fp32", "bf16")])
def test_onepass_bf16_storage(din, dout, precision, monkeypatch):
    """BF16 signals and/or coefficients: bit-equal to the three-pass form with the same
    storage."""
    dev = device()
    g = wl.config5b_graph()
    one = _plan(g, precision, "onepass", monkeypatch, in_dtype=din, out_dtype=dout)
    three = _plan(g, precision, "passes", monkeypatch, in_dtype=din, out_dtype=dout)
    assert one.tuning()["variant"] == 2
    td = {"bf16": torch.bfloat16, "fp32": torch.float32}
    X = wl.gaussian(333, g.n, wl.rng_for(5, 5, 333))
    x = torch.from_numpy(X).to(dev).to(td[din])
    y = one.forward(x)
    assert y.dtype == td[dout]
    assert torch.equal(y, three.forward(x))
    assert torch.equal(one.inverse(y), three.inverse(y))


def test_onepass_needs_no_workspace(monkeypatch):
    """The allocation-free apply takes any number of signals on a one-pass plan: there is no
    workspace to fit in the static scratch (8192 signals is the three-pass limit here)."""
    dev = device()
    g = wl.config5b_graph()
    plan = _plan(g, "bf16", "onepass", monkeypatch)
    assert plan.tuning()["variant"] == 2
    S = 20000
    x = torch.from_numpy(wl.gaussian(S, g.n, wl.rng_for(5, 6))).to(dev)
    lib = G.load_library()
    for d, fn in ((0, G.gft_forward), (1, G.gft_inverse)):
        out = torch.full_like(x, float("nan"))
        st = lib.gft_apply_noalloc(plan.handle, d, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   S, G._stream_ptr(None))
        assert st == 0, lib.gft_last_error()
        assert torch.equal(out, fn(plan, x))


def test_onepass_captured_graph_replays_equal_eager(monkeypatch):
    """hipGraph capture of the large engine: one-pass plans with FP32 and BF16 blocks
    (forward and inverse) replay bit-equal to eager, with eager work between replays.  A
    plan forced to the three-pass form, whose workspace comes from the stream-ordered pool
    per call, is refused under capture (GFT_ERR_UNSUPPORTED) without disturbing the capture,
    and the allocation-free apply records it in the same graph instead."""
    dev = device()
    g = wl.config5b_graph()
    rng = wl.rng_for(5, 12)
    one32 = _plan(g, "fp32", "onepass", monkeypatch)
    one16 = _plan(g, "bf16", "onepass", monkeypatch)
    three = _plan(g, "fp32", "passes", monkeypatch)
    assert one32.tuning()["variant"] == 2 and one16.tuning()["variant"] == 2
    assert three.tuning()["variant"] == 0
    x = torch.from_numpy(wl.gaussian(3001, g.n, rng)).to(dev)
    x3 = torch.from_numpy(wl.gaussian(700, g.n, rng)).to(dev)
    y32, r32, y16, y3 = (torch.empty_like(x), torch.empty_like(x), torch.empty_like(x), torch.empty_like(x3))
    eager = [one32.forward(x).clone(), None, one16.forward(x).clone(), three.forward(x3).clone()]
    eager[1] = one32.inverse(eager[0]).clone()
    lib = G.load_library()

    def record(stream):
        one32.forward(x, out=y32, stream=stream)
        one32.inverse(y32, out=r32, stream=stream)
        one16.forward(x, out=y16, stream=stream)
        st = lib.gft_apply_noalloc(three.handle, 0, ctypes.c_void_p(x3.data_ptr()), ctypes.c_void_p(y3.data_ptr()),
                                   x3.shape[0], G._stream_ptr(stream))
        assert st == 0, lib.gft_last_error()

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        record(None)                                     # warm-up on the side stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        with pytest.raises(G.GFTError, match="stream capture"):
            three.forward(x3, out=y3)
        record(None)
    outs = (y32, r32, y16, y3)
    for _ in range(3):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o, e)
        one16.inverse(one16.forward(x))                  # eager work between replays
        three.forward(x3)
        torch.cuda.synchronize()
