"""GPU parity of the fast GFT kernels against the FP64 oracle (through the C ABI).

The oracle's eigenbasis is aligned to the basis the GPU applies inside each eigenvalue
cluster (sign and rotation within an eigenspace are free, Sec. III); the comparison then
covers every coefficient of every signal.  FP32 tolerance: relative error <= 1e-5.
"""
import numpy as np
import pytest

import paper_1907_07875_amd as G
import workloads as wl
from oracle import gft_oracle as O
from tests.gpu_helpers import aligned_oracle_basis, device, gpu_basis, to_np, torch

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5


def _check_graph(g, X, tol=TOL_FP32, engine="auto", precision="fp32", basis_tol=2e-6,
                 laplacian="combinatorial"):
    """Forward, inverse and round trip of plan(g) on X against the oracle.

    The oracle basis is rotated, inside each eigenvalue cluster, onto the plan's FP64 basis
    (the freedom Sec. III allows), after checking that the plan's basis spans the oracle's
    eigenspaces; the basis the GPU applies must equal the plan's to `basis_tol`.
    """
    dev = device()
    plan = G.Plan.from_graph(g, engine=engine, precision=precision, laplacian=laplacian)
    Uplan = plan.basis()
    lam, Ua = aligned_oracle_basis(g, Uplan, sv_tol=1e-9, laplacian=laplacian)
    Uhat = gpu_basis(plan, dev)
    assert np.abs(Uhat - Uplan).max() <= basis_tol, np.abs(Uhat - Uplan).max()
    Xd = X.astype(np.float64)
    x = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
    y = plan.forward(x)
    C_ref = O.forward(Xd, Ua)
    err = O.relative_error(to_np(y), C_ref)
    assert err <= tol, f"{g.name}: forward relative error {err:.3e}"
    # inverse of the oracle's coefficients (FP32-rounded) reproduces the oracle's signal
    C32 = C_ref.astype(np.float32)
    xr = plan.inverse(torch.from_numpy(C32).to(dev))
    err_i = O.relative_error(to_np(xr), O.inverse(C32.astype(np.float64), Ua))
    assert err_i <= tol, f"{g.name}: inverse relative error {err_i:.3e}"
    rt = O.relative_error(to_np(plan.inverse(y)), Xd)
    assert rt <= 2 * tol, f"{g.name}: round trip error {rt:.3e}"
    return plan, Uhat, lam, err


def test_config1_path8_dct2():
    """Path N=8 (one Haar stage, blocks 4+4): GPU basis is DCT-II up to sign."""
    g = wl.config1_graph()
    X = wl.gaussian(4096, 8, wl.rng_for(1), dtype=np.float64)
    plan, Uhat, lam, _ = _check_graph(g, X)
    np.testing.assert_allclose(np.abs(Uhat.T @ O.dct2_matrix(8)), np.eye(8), atol=2e-6)
    np.testing.assert_allclose(lam, O.path_eigenvalues(8), atol=1e-12)


@pytest.mark.parametrize("engine", ["generic", "butterfly"])
@pytest.mark.parametrize("S", [1, 15, 16, 17, 63, 64, 65, 1000, (1 << 14) + 37])
def test_config2_grid8x8_ragged(S, engine):
    g = wl.config2_graph()
    X = wl.ar1_field(S, 8, 8, 0.95, wl.rng_for(2, S))
    _check_graph(g, X, engine=engine)


@pytest.mark.parametrize("engine", ["auto", "generic"])
def test_config2_grid8x8_full_size(engine):
    """2^20 AR(1) signals: the shape and launch configuration the benchmark times."""
    g = wl.config2_graph()
    X = wl.ar1_field(1 << 20, 8, 8, 0.95, wl.rng_for(2))
    _check_graph(g, X, engine=engine)


@pytest.mark.parametrize("g", [wl.path(32), wl.path(64), wl.cycle(32), wl.cycle_two_stage(64),
                               wl.grid(4, 16), wl.grid3d(4, 4, 8)],
                         ids=lambda g: f"{g.name}{g.n}s{len(g.stages)}")
def test_butterfly_engine_shapes(g):
    """Uniform hypercube plans on the register-butterfly engine (S = 1, 2, 3 stages)."""
    X = wl.gaussian(2000, g.n, wl.rng_for(4, g.n, 3))
    _check_graph(g, X, engine="butterfly")


def test_auto_engine_choice():
    device()
    assert G.Plan.from_graph(wl.config2_graph()).engine() == "butterfly"
    assert G.Plan.from_graph(wl.config3_graph()).engine() == "butterfly"          # one stage, n odd
    assert G.Plan.from_graph(wl.config3_graph(), precision="bf16").engine() == "butterfly"
    assert G.Plan.from_graph(wl.config3_graph(), precision="fp16").engine() == "generic"
    assert G.Plan.from_graph(wl.config2_graph(), engine="generic").engine() == "generic"


def test_butterfly_engine_rejects_non_uniform_plan():
    dev = device()
    plan = G.Plan.from_graph(wl.grid(11, 11), engine="butterfly")     # two stages, 36-node leaf
    with pytest.raises(G.GFTError) as e:
        plan.forward(torch.zeros((16, 121), device=dev))
    assert e.value.status_name == "GFT_ERR_UNSUPPORTED"


def test_config3_skeleton_fp32():
    g = wl.config3_graph()
    X = wl.skeleton_walks(8, 3, 40, wl.rng_for(3, 1)).reshape(-1, 25)
    _check_graph(g, X)


@pytest.mark.parametrize("g", [wl.path(4), wl.path(7), wl.path(64), wl.cycle(8), wl.cycle(13),
                               wl.cycle(64), wl.grid(4, 4), wl.grid(5, 5), wl.grid(16, 16),
                               wl.symmetric_bipartite(40, wl.rng_for(4, 40)),
                               wl.symmetric_bipartite(128, wl.rng_for(4, 128))],
                         ids=lambda g: f"{g.name}{g.n}")
def test_config4_families_single(g):
    X = wl.gaussian(3000, g.n, wl.rng_for(4, g.n, 7))
    _check_graph(g, X)


def test_no_symmetry_is_dense_gft():
    """A plan with no stages is the dense GFT (one block)."""
    g = wl.symmetric_bipartite(24, wl.rng_for(4, 99))
    g.stages = []
    X = wl.gaussian(500, g.n, wl.rng_for(4, 98))
    _check_graph(g, X)


def test_empty_batch_is_noop():
    dev = device()
    plan = G.Plan.from_graph(wl.config2_graph())
    x = torch.zeros((0, 64), device=dev)
    y = plan.forward(x)
    assert y.shape == (0, 64)


def test_in_place_forward():
    dev = device()
    g = wl.config2_graph()
    plan = G.Plan.from_graph(g)
    X = wl.gaussian(777, 64, wl.rng_for(2, 5))
    x = torch.from_numpy(X).to(dev)
    ref = plan.forward(x.clone())
    plan.forward(x, out=x)
    torch.cuda.synchronize()
    assert torch.equal(x, ref)


def test_misaligned_and_overlapping_rejected():
    dev = device()
    plan = G.Plan.from_graph(wl.path(8))
    buf = torch.zeros(8 * 101, device=dev)
    with pytest.raises(G.GFTError) as e:
        G.load_library()
        import ctypes
        G._check(G.load_library().gft_forward(plan.handle, ctypes.c_void_p(buf.data_ptr() + 4),
                                              ctypes.c_void_p(buf.data_ptr() + 4096), 10, None))
    assert e.value.status_name == "GFT_ERR_ALIGNMENT"
    with pytest.raises(G.GFTError) as e:
        import ctypes
        G._check(G.load_library().gft_forward(plan.handle, ctypes.c_void_p(buf.data_ptr()),
                                              ctypes.c_void_p(buf.data_ptr() + 64), 10, None))
    assert e.value.status_name == "GFT_ERR_ALIGNMENT"


def test_adjoint_dot_product():
    """<U^T x, y> = <x, U y>: the inverse kernel is the adjoint of the forward kernel."""
    dev = device()
    g = wl.config3_graph()
    plan = G.Plan.from_graph(g)
    rng = wl.rng_for(3, 11)
    x = torch.from_numpy(wl.gaussian(2048, 25, rng)).to(dev)
    yv = torch.from_numpy(wl.gaussian(2048, 25, rng)).to(dev)
    lhs = (plan.forward(x).double() * yv.double()).sum().item()
    rhs = (x.double() * plan.inverse(yv).double()).sum().item()
    assert abs(lhs - rhs) <= 1e-5 * (abs(lhs) + (x.double().norm() * yv.double().norm()).item())


def test_gpu_basis_matches_plan_basis():
    dev = device()
    for g in (wl.config2_graph(), wl.config3_graph(), wl.cycle(12)):
        plan = G.Plan.from_graph(g)
        np.testing.assert_allclose(gpu_basis(plan, dev), plan.basis(), atol=2e-6)


AUTOGRAD_TOL = {"fp32": (2e-5, 1e-3), "bf16": (2e-2, 0.1)}   # (gradient rel. err, FD abs. err)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_autograd_backward_is_inverse_kernel(precision):
    """Backward of GFTFunction (the adjoint kernel) on the skeleton, FP32 and BF16 leaf
    blocks (the configured c3 case): against the oracle gradient U g, the dot-product test
    and central finite differences (h = 1 is exact for a linear map up to rounding; with
    BF16 blocks every forward rounds block inputs, so the FD bound is that rounding)."""
    dev = device()
    g = wl.config3_graph()
    plan = G.Plan.from_graph(g, precision=precision)
    assert plan.engine() == "butterfly"
    gtol, fdtol = AUTOGRAD_TOL[precision]
    X = wl.skeleton_walks(4, 3, 16, wl.rng_for(3, 12)).reshape(-1, 25)[:192]
    x = torch.from_numpy(X).to(dev).requires_grad_(True)
    w = torch.from_numpy(wl.gaussian(X.shape[0], 25, wl.rng_for(3, 13))).to(dev)
    y = G.gft(x, plan)
    (y * w).sum().backward()
    _, Ua = aligned_oracle_basis(g, plan.basis(), sv_tol=1e-9)
    # loss = sum(w * (x U)) -> grad_x = w U^T
    ref = to_np(w) @ Ua.T
    err = O.relative_error(to_np(x.grad), ref)
    assert err <= gtol, f"{precision}: gradient relative error {err:.3e}"
    if precision == "bf16":
        assert err > 1e-6, "BF16 gradient suspiciously exact: the adjoint may not run BF16 blocks"
    # the backward is the inverse kernel itself
    assert torch.equal(x.grad, plan.inverse(w))
    xd = x.detach()
    for (s_, i) in ((0, 0), (5, 13), (191, 24)):
        e = torch.zeros_like(xd)
        e[s_, i] = 1.0
        fp = (plan.forward(xd + e).double() * w.double()).sum().item()
        fm = (plan.forward(xd - e).double() * w.double()).sum().item()
        assert abs((fp - fm) / 2 - x.grad[s_, i].item()) <= fdtol, (s_, i, (fp - fm) / 2, x.grad[s_, i].item())


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_autograd_igft_backward_is_forward_kernel(precision):
    """Backward of IGFTFunction (x = U y, grad_y = U^T grad_x, the forward kernel) against
    the oracle gradient and finite differences; igft inverts gft."""
    dev = device()
    g = wl.config3_graph()
    plan = G.Plan.from_graph(g, precision=precision)
    gtol, fdtol = AUTOGRAD_TOL[precision]
    rng = wl.rng_for(3, 14)
    y = torch.from_numpy(wl.gaussian(160, 25, rng)).to(dev).requires_grad_(True)
    w = torch.from_numpy(wl.gaussian(160, 25, rng)).to(dev)
    x = G.igft(y, plan)
    (x * w).sum().backward()
    _, Ua = aligned_oracle_basis(g, plan.basis(), sv_tol=1e-9)
    # loss = sum(w * (y U^T)) -> grad_y = w U
    err = O.relative_error(to_np(y.grad), to_np(w) @ Ua)
    assert err <= gtol, f"{precision}: gradient relative error {err:.3e}"
    assert torch.equal(y.grad, plan.forward(w))
    yd = y.detach()
    for (s_, k) in ((0, 0), (77, 6), (159, 24)):
        e = torch.zeros_like(yd)
        e[s_, k] = 1.0
        fp = (plan.inverse(yd + e).double() * w.double()).sum().item()
        fm = (plan.inverse(yd - e).double() * w.double()).sum().item()
        assert abs((fp - fm) / 2 - y.grad[s_, k].item()) <= fdtol
    # gft after igft returns the coefficients (to the precision's tolerance)
    back = G.gft(G.igft(yd, plan), plan)
    assert O.relative_error(to_np(back), to_np(yd)) <= 2 * gtol


@pytest.mark.parametrize("engine", ["auto", "generic", "large"])
@pytest.mark.parametrize("g", [wl.config2_graph(), wl.config3_graph(), wl.cycle_two_stage(16),
                               wl.weighted_symmetric_path(64, wl.rng_for(9, 64))],
                         ids=lambda g: f"{g.name}{g.n}")
def test_normalized_laplacian_parity(g, engine):
    """GFT of the symmetric normalized Laplacian D^{-1/2} L D^{-1/2} on every engine."""
    X = wl.gaussian(1500, g.n, wl.rng_for(9, g.n, 3))
    _check_graph(g, X, engine=engine, laplacian="normalized")


def _c4_with_stage():
    g = wl.cycle(4)
    g.stages = [np.array([3, 2, 1, 0], dtype=np.int32)]
    return g


def _cycle_no_stage(n):
    g = wl.cycle(n)
    g.stages = []
    return g


def _k_regular_bipartite(m, weights):
    edges, w = [], []
    for r, wr in enumerate(weights):
        for i in range(m):
            edges.append((i, m + (i + r) % m))
            w.append(wr)
    return wl._graph(2 * m, edges, w, name=f"krbg{len(weights)}_")


@pytest.mark.parametrize("engine", ["auto", "generic", "large"])
@pytest.mark.parametrize("g", [_c4_with_stage(), _cycle_no_stage(12), _cycle_no_stage(30),
                               _k_regular_bipartite(16, [0.3, 1.7, 0.9])],
                         ids=lambda g: f"{g.name}{g.n}s{len(g.stages)}")
def test_right_haar_parity(g, engine):
    """Plans with right Haar units (forward: after the blocks; inverse: before them)."""
    plan = G.Plan.from_graph(g, engine=engine)
    assert plan.info()["num_right_leaves"] >= 1
    X = wl.gaussian(2500, g.n, wl.rng_for(9, g.n, 4))
    _check_graph(g, X, engine=engine)


def test_right_haar_large_k_regular_bipartite():
    """n = 600 3-regular weighted bipartite graph: blocks E, F of 300 on the large engine."""
    g = _k_regular_bipartite(300, [0.4, 1.1, 0.8])
    plan = G.Plan.from_graph(g)
    assert plan.engine() == "large" and plan.info()["max_block"] == 300
    X = wl.gaussian(700, g.n, wl.rng_for(9, 600))
    _check_graph(g, X)
    _check_graph(g, X, precision="split_bf16", tol=1e-5, basis_tol=5e-6)


@pytest.mark.parametrize("g", [wl.grid(8, 8), wl.path(16), wl.config3_graph()], ids=lambda g: f"{g.name}{g.n}")
def test_searched_pairings_parity(g):
    """Stages from gft_find_pairing (6 for the 8x8 grid) run on the GPU like given ones."""
    st = G.gft_find_pairing(g.n, g.src, g.dst, g.weight, g.self_loop, max_stages=8)
    h = wl._graph(g.n, np.stack([g.src, g.dst], 1), g.weight, loops=g.self_loop, stages=st, name=g.name)
    X = wl.gaussian(2000, g.n, wl.rng_for(9, g.n, 5))
    _check_graph(h, X)


# n odd and n = 2 mod 4 keep the signals' own LDS layout; n = 0 mod 8 and n = 4 mod 8 pad the
# rows (to n + 4 and n + 8; n = 60 and 92 reach the largest padded tiles of 32- and 48-slot
# sides)
ONE_STAGE_GRAPHS = [wl.config3_graph(), wl.path(17), wl.cycle(31), wl.path(63),
                    wl.weighted_symmetric_path(33, wl.rng_for(9, 33)), wl.path(8), wl.path(12),
                    wl.cycle(22), wl.path(40), wl.path(44), wl.cycle(48), wl.cycle(60),
                    wl.symmetric_bipartite(40, wl.rng_for(4, 40)),
                    wl.weighted_symmetric_path(36, wl.rng_for(9, 36)),
                    # 48-slot sides
                    wl.path(72), wl.cycle(84), wl.cycle(92), wl.symmetric_bipartite(72, wl.rng_for(4, 72)),
                    wl.weighted_symmetric_path(90, wl.rng_for(9, 90)),
                    # equal 48-node blocks: no uniform kernel of that shape, the padded layout
                    wl.path(96)]


@pytest.mark.parametrize("S", [1, 15, 17, 1003])
@pytest.mark.parametrize("g", ONE_STAGE_GRAPHS, ids=lambda g: f"{g.name}{g.n}")
def test_one_stage_butterfly_general(g, S):
    """One-stage plans that are not uniform hypercubes (V_Z nodes, unequal or split blocks,
    8 <= n <= 64) on the register butterfly engine: padded slots, the LDS row layouts and
    exact tile tails; FP32 blocks and BF16 blocks (16x16x16 MFMA on inputs rounded after the
    FP32 Haar stage)."""
    assert G.Plan.from_graph(g).engine() == "butterfly"
    X = wl.gaussian(S, g.n, wl.rng_for(9, g.n, S))
    _check_graph(g, X, engine="butterfly")
    assert G.Plan.from_graph(g, precision="bf16").engine() == "butterfly"
    _, _, _, err = _check_graph(g, X, engine="butterfly", precision="bf16", tol=2e-2, basis_tol=1e-2)
    assert err > 1e-5, "BF16 error suspiciously small: blocks may not run in BF16"


TWO_STAGE_GRAPHS = [wl.grid(5, 5), wl.grid(6, 6), wl.grid(7, 7), wl.grid(3, 3), wl.grid(5, 7),
                    wl.grid(8, 5), wl.grid(9, 9), wl.grid(10, 10), wl.cycle_two_stage(20),
                    wl.cycle_two_stage(44),
                    # equal 32-node blocks: no uniform kernel of that shape, the padded layout
                    wl.grid(16, 8)]


@pytest.mark.parametrize("S", [1, 17, 1003])
@pytest.mark.parametrize("g", TWO_STAGE_GRAPHS, ids=lambda g: f"{g.name}{g.n}")
def test_two_stage_butterfly_general(g, S):
    """Two-stage plans that are not uniform hypercubes (odd and unequal grids under LR then
    UD, fixed nodes at either stage, components) on the register butterfly's padded
    two-stage layout: 16- and 32-slot sides, sign flips on the difference side, ragged S."""
    assert G.Plan.from_graph(g).engine() == "butterfly"
    X = wl.gaussian(S, g.n, wl.rng_for(9, g.n, S, 5))
    _check_graph(g, X, engine="butterfly")


@pytest.mark.parametrize("io", [("bf16", "bf16"), ("fp32", "bf16"), ("bf16", "fp32")])
@pytest.mark.parametrize("g", [wl.config3_graph(), wl.path(12), wl.cycle(22), wl.path(44), wl.cycle(48),
                               wl.grid(5, 5), wl.grid(10, 10)],
                         ids=lambda g: f"{g.name}{g.n}")
def test_one_stage_butterfly_storage(io, g):
    """BF16 storage on the padded layouts, one and two stages (16-byte groups of 8 values
    split across padded rows when n = 4 mod 8) equals FP32 storage rounded."""
    dev = device()
    X = wl.gaussian(1003, g.n, wl.rng_for(9, g.n, 8))
    plan = G.Plan.from_graph(g, in_dtype=io[0], out_dtype=io[1])
    ref = G.Plan.from_graph(g, engine="butterfly")
    assert plan.engine() == "butterfly"
    x = torch.from_numpy(X).to(dev).to({"fp32": torch.float32, "bf16": torch.bfloat16}[io[0]])
    y = plan.forward(x)
    assert torch.equal(y, ref.forward(x.float()).to(y.dtype))
    assert torch.equal(plan.inverse(y), ref.inverse(y.float()).to(x.dtype))


def test_every_mixed_batch_graph_runs_single():
    """Each of the 146 graphs of the mixed batch, planned alone with the automatic engine
    choice, runs (every shape the choice can land on has a compiled kernel) and matches the
    oracle (its eigenbasis aligned per eigenvalue cluster), forward and inverse."""
    dev = device()
    for g in wl.config4_graphs(wl.rng_for(4)):
        plan = G.Plan.from_graph(g)
        X = wl.gaussian(19, g.n, wl.rng_for(4, 7, g.n))
        _, Ua = aligned_oracle_basis(g, plan.basis(), sv_tol=1e-9)
        y = plan.forward(torch.from_numpy(X).to(dev))
        ref = O.forward(X.astype(np.float64), Ua)
        err = O.relative_error(to_np(y), ref)
        assert err <= TOL_FP32, f"{g.name}{g.n} on {plan.engine()}: forward {err:.3e}"
        C32 = ref.astype(np.float32)
        xr = to_np(plan.inverse(torch.from_numpy(C32).to(dev)))
        err_i = O.relative_error(xr, O.inverse(C32.astype(np.float64), Ua))
        assert err_i <= TOL_FP32, f"{g.name}{g.n} on {plan.engine()}: inverse {err_i:.3e}"
