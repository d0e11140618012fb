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


def test_large_engine_rejects_bf16_storage():
    device()
    plan = G.Plan.from_graph(wl.path(64), engine="large", in_dtype="bf16")
    with pytest.raises(G.GFTError) as e:
        plan.prepare()
    assert e.value.status_name == "GFT_ERR_UNSUPPORTED"
