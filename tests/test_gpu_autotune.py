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


# ----------------------------------------------------- launch tuning of every engine, cache

ENGINE_CASES = [
    ("butterfly", wl.config2_graph, {}, 300_001),
    ("generic", lambda: wl.grid(11, 11), {"engine": "generic"}, 20_003),
    ("large", wl.config5b_graph, {}, 3_001),
    ("large", wl.config5b_graph, {"precision": "bf16"}, 3_001),
    ("large", wl.config5a_graph, {"engine": "large"}, 601),
    ("product", wl.config5a_graph, {}, 2_001),
]


@pytest.mark.parametrize("case", ENGINE_CASES, ids=lambda c: f"{c[0]}-{c[1]().name}-{c[2].get('precision', 'fp32')}")
def test_tuned_launch_choices_are_bit_identical_and_cached(case, tmp_path, monkeypatch):
    """options.autotune on (timed candidates, or the cache) against the built-in choices:
    the same coefficients and signals bit for bit; a second plan of the same graph takes
    its choices from the cache without timing."""
    monkeypatch.setenv("GFT_TUNE_CACHE", str(tmp_path / "tuning.txt"))
    engine, make, kw, S = case
    dev = device()
    g = make()
    tuned = G.Plan.from_graph(g, **kw)
    fixed = G.Plan.from_graph(g, autotune=False, **kw)
    t, f = tuned.tuning(), fixed.tuning()
    assert t["engine"] == f["engine"] == engine
    assert t["source"] in ("timed", "cached") and f["source"] == "builtin" and f["tune_ms"] == 0
    x = torch.from_numpy(wl.gaussian(S, g.n, wl.rng_for(9, g.n, 77))).to(dev)
    y = tuned.forward(x)
    assert torch.equal(y, fixed.forward(x))
    assert torch.equal(tuned.inverse(y), fixed.inverse(y))
    again = G.Plan.from_graph(g, **kw).tuning()
    assert again["source"] == "cached" and again["tune_ms"] == 0
    for k in ("fwd_tile", "inv_tile", "grid_fwd", "grid_inv", "variant", "large_tile_kb"):
        assert again[k] == t[k], k
    if engine == "large":
        assert t["large_tile_kb"] in (20, 40, 80)


def test_batch_tuning_bit_identical_and_reported(tmp_path, monkeypatch):
    monkeypatch.setenv("GFT_TUNE_CACHE", str(tmp_path / "tuning.txt"))
    dev = device()
    rng = wl.rng_for(4, 9)
    graphs = [wl.path(7), wl.grid(8, 8), wl.config3_graph(), wl.cycle(40), wl.symmetric_bipartite(120, wl.rng_for(4, 120)),
              wl.grid(12, 12), wl.path(64), wl.grid(16, 16)]
    counts = np.array([3000, 20000, 9000, 1, 700, 5000, 12000, 2500])
    xs = [wl.gaussian(int(c), g.n, rng) for g, c in zip(graphs, counts)]
    flat = torch.from_numpy(np.concatenate([a.reshape(-1) for a in xs])).to(dev)
    offs = torch.from_numpy(np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)).to(dev)
    tuned = G.gft_plan_batch(graphs)
    fixed = G.gft_plan_batch(graphs, autotune=False)
    t, f = tuned.tuning(), fixed.tuning()
    assert t["source"] in ("timed", "cached") and f["source"] == "builtin"
    assert 1 <= t["batch_rounds"] <= 4 and t["batch_cost16"] in (8, 11, 14)
    assert (f["batch_rounds"], f["batch_cost16"]) == (2, 11)
    y = G.gft_forward_batch(tuned, flat, offs)
    assert torch.equal(y, G.gft_forward_batch(fixed, flat, offs))
    assert torch.equal(G.gft_inverse_batch(tuned, y, offs), G.gft_inverse_batch(fixed, y, offs))


def test_tuning_cache_file_is_read_by_a_new_process(tmp_path, monkeypatch):
    """The tuning cache file carries a choice to another process: the same plan there is
    prepared without timing."""
    import os
    import subprocess
    import sys
    path = tmp_path / "tuning.txt"
    monkeypatch.setenv("GFT_TUNE_CACHE", str(path))
    device()
    g = wl.grid(9, 9)
    assert G.Plan.from_graph(g).tuning()["source"] in ("timed", "cached")
    assert path.exists() and len(path.read_text().splitlines()) >= 1
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r); import paper_1907_07875_amd as G, workloads as wl; "
            "print(G.Plan.from_graph(wl.grid(9, 9)).tuning()['source'])" % root)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240,
                         env=dict(os.environ, GFT_TUNE_CACHE=str(path)))
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == "cached"
