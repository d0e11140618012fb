"""Degenerate and signed graphs on the GPU against the FP64 oracle: a single node, two nodes with and
without an edge (paired and not), an isolated node beside an edge, an edgeless graph with a
pairing, and a batch mixing them with empty signal ranges.  The GFT of an edgeless graph is
any orthonormal basis of one eigenspace (eigenvalue 0), so parity is checked after the
usual per-cluster alignment."""
import numpy as np
import pytest

import paper_1907_07875_amd as G
import workloads as wl
from oracle import gft_oracle as O
from tests.gpu_helpers import aligned_oracle_basis, device, gpu_basis, to_np, torch

pytestmark = pytest.mark.gpu


def _graph(n, edges, weights=None, stages=(), name="tiny"):
    src = np.array([a for a, _ in edges], dtype=np.int32)
    dst = np.array([b for _, b in edges], dtype=np.int32)
    w = np.array(weights if weights is not None else [1.0] * len(edges), dtype=np.float64)
    return wl.Graph(n, src, dst, w, None, [np.asarray(s, dtype=np.int32) for s in stages], name)


CASES = [
    _graph(1, [], name="single"),
    _graph(2, [(0, 1)], name="edge"),
    _graph(2, [(0, 1)], [0.5], stages=[[1, 0]], name="edge_paired"),
    _graph(2, [], name="no_edges"),
    _graph(4, [], stages=[[1, 0, 3, 2]], name="edgeless_paired"),
    _graph(3, [(0, 1)], [2.0], name="isolated"),
    _graph(5, [(0, 1), (3, 4)], stages=[[4, 3, 2, 1, 0]], name="two_components_paired"),
]


@pytest.mark.parametrize("g", CASES, ids=lambda g: g.name)
@pytest.mark.parametrize("S", [0, 1, 37])
def test_degenerate_graph_parity(g, S):
    dev = device()
    plan = G.Plan.from_graph(g)
    Uplan = plan.basis()
    lam, Ua = aligned_oracle_basis(g, Uplan, sv_tol=1e-9)
    np.testing.assert_allclose(plan.eigenvalues(), lam, atol=1e-12)
    assert np.abs(gpu_basis(plan, dev) - Uplan).max() <= 2e-6
    X = wl.gaussian(S, g.n, wl.rng_for(11, g.n, S))
    x = torch.from_numpy(X).to(dev)
    y = plan.forward(x)
    assert tuple(y.shape) == (S, g.n)
    if S:
        assert O.relative_error(to_np(y), O.forward(X.astype(np.float64), Ua)) <= 1e-5
        assert O.relative_error(to_np(plan.inverse(y)), X.astype(np.float64)) <= 2e-5


def test_degenerate_graphs_in_one_batch():
    """The same graphs in one batch launch, some with no signals, against their single plans."""
    dev = device()
    counts = [5, 0, 17, 1, 0, 33, 8]
    bp = G.gft_plan_batch(CASES)
    X = [wl.gaussian(c, g.n, wl.rng_for(12, i, c)) for i, (g, c) in enumerate(zip(CASES, counts))]
    flat = np.concatenate([x.reshape(-1) for x in X]).astype(np.float32)
    off = torch.from_numpy(np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)).to(dev)
    y = G.gft_forward_batch(bp, torch.from_numpy(flat).to(dev), off)
    yh = to_np(y)
    pos = 0
    for g, x in zip(CASES, X):
        k = x.size
        if k:
            single = to_np(G.Plan.from_graph(g).forward(torch.from_numpy(x).to(dev)))
            assert np.abs(yh[pos:pos + k].reshape(x.shape) - single).max() <= 1e-6, g.name
        pos += k
    xr = to_np(G.gft_inverse_batch(bp, y, off))
    assert O.relative_error(xr, flat.astype(np.float64)) <= 2e-5


SIGNED = [
    wl.path(9, weights=[1.0, -0.5, 2.0, 0.3, 0.3, 2.0, -0.5, 1.0],
            loops=[0.2, -0.1, 0.0, 0.5, 1.0, 0.5, 0.0, -0.1, 0.2], name="signed_path"),
    wl.path(40, weights=list(np.r_[np.linspace(-1, 1, 19), [0.7], np.linspace(1, -1, 19)]),
            loops=list(np.r_[np.linspace(0.5, -0.5, 20), np.linspace(-0.5, 0.5, 20)]), name="signed_path"),
]


@pytest.mark.parametrize("g", SIGNED, ids=lambda g: f"{g.name}{g.n}")
def test_signed_weights_and_self_loops_parity(g):
    """Negative edge weights and self-loops (an indefinite Laplacian, which the
    decomposition accepts): every engine the plan can take matches the oracle."""
    dev = device()
    for engine in ("auto", "generic"):
        plan = G.Plan.from_graph(g, engine=engine)
        lam, Ua = aligned_oracle_basis(g, plan.basis(), sv_tol=1e-9)
        assert lam.min() < 0 or g.n > 9
        X = wl.gaussian(300, g.n, wl.rng_for(13, g.n))
        y = plan.forward(torch.from_numpy(X).to(dev))
        assert O.relative_error(to_np(y), O.forward(X.astype(np.float64), Ua)) <= 1e-5, engine
        assert O.relative_error(to_np(plan.inverse(y)), X.astype(np.float64)) <= 2e-5, engine
