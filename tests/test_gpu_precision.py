"""Reduced-precision leaf blocks (BF16, FP16, split BF16 hi+lo) against the FP64 oracle.

Haar stages stay FP32; the block products take 16-bit operands with FP32 accumulation.
Tolerances (relative Frobenius error of aligned coefficients): BF16 <= 2e-2, FP16 <= 5e-3,
split BF16 <= 1e-5.
"""
import numpy as np
import pytest

import workloads as wl
from tests.test_gpu_parity import _check_graph

pytestmark = pytest.mark.gpu

TOL = {"bf16": 2e-2, "fp16": 5e-3, "split_bf16": 1e-5}
BASIS_TOL = {"bf16": 1e-2, "fp16": 2e-3, "split_bf16": 5e-6}

GRAPHS = [wl.config3_graph(), wl.config2_graph(), wl.cycle(13), wl.path(8),
          wl.symmetric_bipartite(40, wl.rng_for(4, 40)), wl.grid(16, 16)]


@pytest.mark.parametrize("precision", ["bf16", "fp16", "split_bf16"])
@pytest.mark.parametrize("g", GRAPHS, ids=lambda g: f"{g.name}{g.n}")
def test_reduced_precision_parity(g, precision):
    X = wl.gaussian(3000, g.n, wl.rng_for(3, g.n, 5))
    _, _, _, err = _check_graph(g, X, tol=TOL[precision], precision=precision,
                                basis_tol=BASIS_TOL[precision])
    if precision == "bf16":
        assert err > 1e-5, "BF16 error suspiciously small: blocks may not run in BF16"


def test_skeleton_bf16_config3_shape():
    """Config 3 shape: [sequences, 3 channels, frames, 25 joints] smooth walks, BF16 blocks."""
    g = wl.config3_graph()
    X = wl.skeleton_walks(64, 3, 300, wl.rng_for(3, 2)).reshape(-1, 25)
    _check_graph(g, X, tol=TOL["bf16"], precision="bf16", basis_tol=BASIS_TOL["bf16"])
