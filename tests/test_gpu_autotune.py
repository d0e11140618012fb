"""Plan-time tile autotuning of the generic engine (options.tile_override = 0).

The tuner only picks how many signals a workgroup stages per tile; every tile height runs
the same products in the same order, so the tuned plan must agree bit for bit with every
fixed tile height, and the chosen height must be one of the allowed ones.
"""
import numpy as np
import pytest

import paper_1907_07875_amd as G
import workloads as wl
from tests.gpu_helpers import device, torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("g,prec", [(wl.config3_graph(), "bf16"), (wl.grid(8, 8), "fp32"),
                                    (wl.cycle(13), "fp32"), (wl.grid(12, 12), "split_bf16")],
                         ids=lambda v: getattr(v, "name", v))
def test_tuned_tile_is_bit_identical_to_fixed_tiles(g, prec):
    dev = device()
    X = wl.gaussian(3001, g.n, wl.rng_for(9, g.n))
    x = torch.from_numpy(X).to(dev)
    tuned = G.Plan.from_graph(g, engine="generic", precision=prec)
    ft, it = tuned.tiles()
    assert ft in (16, 32, 64, 128) and it in (16, 32, 64, 128)
    y = tuned.forward(x)
    xr = tuned.inverse(y)
    checked = 0
    for tile in (16, 32, 64, 128):
        try:
            fixed = G.Plan.from_graph(g, engine="generic", precision=prec, tile=tile)
            assert fixed.tiles() == (tile, tile)
        except G.GFTError as e:          # tile does not fit in LDS for this graph
            assert e.status_name == "GFT_ERR_UNSUPPORTED"
            continue
        assert torch.equal(fixed.forward(x), y)
        assert torch.equal(fixed.inverse(y), xr)
        checked += 1
    assert checked >= 2


def test_tiles_of_other_engines():
    device()
    assert G.Plan.from_graph(wl.grid(8, 8)).tiles() == (16, 16)            # butterfly, per wave
    assert G.Plan.from_graph(wl.path(64), engine="large").tiles() == (0, 0)
