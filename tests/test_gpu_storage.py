"""BF16 storage of signals and/or coefficients (options in_dtype / out_dtype).

Only the storage changes: BF16 inputs are widened exactly to FP32, the transform runs as
with FP32 storage, and outputs are rounded to the nearest BF16 (ties to even).  So
  * a BF16 output must equal, bit for bit, the FP32-storage output of the same engine
    rounded to BF16 by torch (round to nearest even), and a BF16 input must give exactly
    the FP32-storage result on the widened values;
  * against the FP64 oracle (fed the BF16-rounded inputs widened to FP64), a BF16 output
    adds at most 2^-9 relative rounding per coefficient: the bound used is 2.5e-3 with
    FP32 blocks; FP32 outputs keep the FP32 bound 1e-5.
"""
import numpy as np
import pytest

import paper_1907_07875_amd as G
import workloads as wl
from oracle import gft_oracle as O
from tests.gpu_helpers import aligned_oracle_basis, device, to_np, torch

pytestmark = pytest.mark.gpu

TOL_OUT = {"fp32": 1e-5, "bf16": 2.5e-3}
TD = {"fp32": torch.float32, "bf16": torch.bfloat16}
COMBOS = [("bf16", "bf16"), ("bf16", "fp32"), ("fp32", "bf16")]


def _signals(X, dtype, dev):
    return torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(TD[dtype]).to(dev)


@pytest.mark.parametrize("engine", ["butterfly", "generic"])
@pytest.mark.parametrize("din,dout", COMBOS)
@pytest.mark.parametrize("S", [1037, 16])
def test_grid8x8_storage(engine, din, dout, S):
    dev = device()
    g = wl.config2_graph()
    X = wl.ar1_field(S, 8, 8, 0.95, wl.rng_for(2, S, 7))
    plan = G.Plan.from_graph(g, engine=engine, in_dtype=din, out_dtype=dout)
    ref = G.Plan.from_graph(g, engine=engine)                      # FP32 storage
    assert plan.engine() == engine
    x = _signals(X, din, dev)
    y = plan.forward(x)
    assert y.dtype == TD[dout] and y.shape == x.shape
    # bit-exact against the FP32-storage kernel on the same (widened) values
    y32 = ref.forward(x.float())
    assert torch.equal(y, y32.to(TD[dout])), "BF16 storage changed more than the rounding"
    # oracle
    _, Ua = aligned_oracle_basis(g, plan.basis(), sv_tol=1e-9)
    Xd = to_np(x)
    err = O.relative_error(to_np(y), O.forward(Xd, Ua))
    assert err <= TOL_OUT[dout], f"forward {din}->{dout}: {err:.3e}"
    # inverse reads coefficients in out_dtype and writes signals in in_dtype
    xr = plan.inverse(y)
    assert xr.dtype == TD[din]
    assert torch.equal(xr, ref.inverse(y.float()).to(TD[din]))
    err_i = O.relative_error(to_np(xr), O.inverse(to_np(y), Ua))
    assert err_i <= TOL_OUT[din], f"inverse {dout}->{din}: {err_i:.3e}"


@pytest.mark.parametrize("g", [wl.path(7), wl.config3_graph(), wl.cycle(13)], ids=lambda g: f"{g.name}{g.n}")
def test_generic_odd_n_tails(g):
    """n not a multiple of 4: tiles end inside a 4-value vector (scalar tail path)."""
    dev = device()
    X = wl.gaussian(37, g.n, wl.rng_for(3, g.n, 9))
    plan = G.Plan.from_graph(g, engine="generic", in_dtype="bf16", out_dtype="bf16")
    ref = G.Plan.from_graph(g, engine="generic")
    x = _signals(X, "bf16", dev)
    y = plan.forward(x)
    assert torch.equal(y, ref.forward(x.float()).to(torch.bfloat16))
    _, Ua = aligned_oracle_basis(g, plan.basis(), sv_tol=1e-9)
    assert O.relative_error(to_np(y), O.forward(to_np(x), Ua)) <= TOL_OUT["bf16"]


def test_skeleton_bf16_blocks_bf16_storage():
    """Config 3 with BF16 blocks and BF16 storage (half the bytes of FP32 storage)."""
    dev = device()
    g = wl.config3_graph()
    X = wl.skeleton_walks(32, 3, 300, wl.rng_for(3, 11)).reshape(-1, 25)
    plan = G.Plan.from_graph(g, precision="bf16", in_dtype="bf16", out_dtype="bf16")
    x = _signals(X, "bf16", dev)
    y = plan.forward(x)
    _, Ua = aligned_oracle_basis(g, plan.basis(), sv_tol=1e-9)
    assert O.relative_error(to_np(y), O.forward(to_np(x), Ua)) <= 2e-2


def test_in_place_rules():
    dev = device()
    g = wl.config2_graph()
    X = wl.gaussian(500, 64, wl.rng_for(2, 500, 3))
    plan = G.Plan.from_graph(g, in_dtype="bf16", out_dtype="bf16")
    x = _signals(X, "bf16", dev)
    want = plan.forward(x)
    xi = x.clone()
    plan.forward(xi, out=xi)                      # in place, equal types
    assert torch.equal(xi, want)
    mixed = G.Plan.from_graph(g, in_dtype="bf16", out_dtype="fp32")
    lib = G.load_library()
    st = lib.gft_forward(mixed.handle, G.ctypes.c_void_p(x.data_ptr()), G.ctypes.c_void_p(x.data_ptr()),
                         x.shape[0], G._stream_ptr(None))
    assert G.STATUS.get(st) == "GFT_ERR_ALIGNMENT"


@pytest.mark.parametrize("din,dout", COMBOS)
@pytest.mark.parametrize("which", ["wpath1024", "grid64_large"])
def test_large_engine_storage(which, din, dout):
    """The large engine with BF16 storage: the stage pass widens BF16 rows exactly, and the
    GEMM epilogue (forward, output order written by the GEMM) or the last stage pass rounds
    to BF16; bit-equal to the FP32-storage plan rounded, and within the oracle bound."""
    dev = device()
    g = wl.config5b_graph() if which == "wpath1024" else wl.grid_recursive(16)
    plan = G.Plan.from_graph(g, engine="large", in_dtype=din, out_dtype=dout)
    ref = G.Plan.from_graph(g, engine="large")
    assert plan.engine() == "large"
    X = wl.gaussian(301, g.n, wl.rng_for(5, g.n, 41))
    x = _signals(X, din, dev)
    y = plan.forward(x)
    assert y.dtype == TD[dout]
    assert torch.equal(y, ref.forward(x.float()).to(TD[dout]))
    xr = plan.inverse(y)
    assert xr.dtype == TD[din]
    assert torch.equal(xr, ref.inverse(y.float()).to(TD[din]))
    _, Ua = aligned_oracle_basis(g, plan.basis(), sv_tol=1e-9)
    assert O.relative_error(to_np(y), O.forward(to_np(x), Ua)) <= TOL_OUT[dout]
    assert O.relative_error(to_np(xr), O.inverse(to_np(y), Ua)) <= TOL_OUT[din]


@pytest.mark.parametrize("pair", [(wl.path(8), wl.path(8)), (wl.path(6), wl.path(5)), (wl.path(40), wl.path(24)),
                                  (wl.path_recursive(64), wl.path_recursive(64))],
                         ids=lambda p: f"{p[0].name}{p[0].n}x{p[1].name}{p[1].n}")
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_product_engine_bf16_storage(pair, precision, monkeypatch):
    """Product plans with BF16 signals and coefficients (dense factors; n = 30 takes the
    scalar path): bit-equal to the FP32-storage plan of the same form rounded, within the
    oracle bound; mixed storage types are refused."""
    monkeypatch.setenv("GFT_PRODUCT_FORM", "dense")
    dev = device()
    ga, gb = pair
    plan = G.Plan.from_product(ga, gb, precision=precision, in_dtype="bf16", out_dtype="bf16")
    ref = G.Plan.from_product(ga, gb, precision=precision)
    g = wl.cartesian_product(ga, gb)
    X = wl.gaussian(333, g.n, wl.rng_for(5, g.n, 43))
    x = _signals(X, "bf16", dev)
    y = plan.forward(x)
    assert y.dtype == torch.bfloat16
    assert torch.equal(y, ref.forward(x.float()).to(torch.bfloat16))
    xr = plan.inverse(y)
    assert torch.equal(xr, ref.inverse(y.float()).to(torch.bfloat16))
    _, Ua = aligned_oracle_basis(g, plan.basis(), sv_tol=1e-8)
    tol = TOL_OUT["bf16"] if precision == "fp32" else 2e-2
    assert O.relative_error(to_np(y), O.forward(to_np(x), Ua)) <= tol
    with pytest.raises(G.GFTError) as e:
        G.Plan.from_product(ga, gb, in_dtype="bf16", out_dtype="fp32")
    assert e.value.status_name == "GFT_ERR_UNSUPPORTED"


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_batch_bf16_storage(precision):
    """A mixed batch with BF16 signals and coefficients (register phase and LDS programs):
    bit-equal to the FP32-storage batch rounded, every graph within the oracle bound."""
    dev = device()
    rng = wl.rng_for(4, 21)
    graphs = [wl.path(7), wl.grid(8, 8), wl.config3_graph(), wl.cycle(40), wl.symmetric_bipartite(120, wl.rng_for(4, 120)),
              wl.grid(12, 12), wl.path(64), wl.grid(5, 5), wl.path(90)]
    counts = np.array([300, 2000, 900, 1, 70, 500, 1200, 33, 250])
    xs = [wl.gaussian(int(c), g.n, rng) for g, c in zip(graphs, counts)]
    flat = np.concatenate([a.reshape(-1) for a in xs])
    offs = torch.from_numpy(np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)).to(dev)
    plan = G.gft_plan_batch(graphs, precision=precision, in_dtype="bf16", out_dtype="bf16")
    ref = G.gft_plan_batch(graphs, precision=precision)
    x = _signals(flat, "bf16", dev)
    y = G.gft_forward_batch(plan, x, offs)
    assert y.dtype == torch.bfloat16
    assert torch.equal(y, G.gft_forward_batch(ref, x.float(), offs).to(torch.bfloat16))
    xr = G.gft_inverse_batch(plan, y, offs)
    assert torch.equal(xr, G.gft_inverse_batch(ref, y.float(), offs).to(torch.bfloat16))
    yn, xn = to_np(y), to_np(x)
    pos = 0
    tol = TOL_OUT["bf16"] if precision == "fp32" else 2e-2
    for i, (g, c) in enumerate(zip(graphs, counts)):
        a, b = pos, pos + int(c) * g.n
        pos = b
        _, Ua = aligned_oracle_basis(g, plan.basis(i), sv_tol=1e-9)
        err = O.relative_error(yn[a:b].reshape(-1, g.n), O.forward(xn[a:b].reshape(-1, g.n), Ua))
        assert err <= tol, f"graph {i} ({g.name}{g.n}): {err:.3e}"
    with pytest.raises(TypeError):
        G.gft_forward_batch(plan, x.float(), offs)
