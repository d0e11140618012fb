"""Shared helpers of the GPU parity tests (no transform arithmetic of their own)."""
import hashlib

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import gft_oracle as O  # noqa: E402


def device():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return torch.device("cuda:0")


def gpu_basis(plan, dev):
    """The basis the GPU applies: forward of the n unit vectors (row i = U^T e_i)."""
    eye = torch.eye(plan.n, device=dev, dtype=torch.float32)
    return plan.forward(eye).double().cpu().numpy()


_EIG_CACHE = {}


def _graph_key(graph, laplacian):
    h = hashlib.sha1()
    for a in (graph.src, graph.dst, graph.weight, graph.self_loop):
        if a is not None:
            h.update(np.ascontiguousarray(a).tobytes())
    return (int(graph.n), laplacian, h.hexdigest())


def oracle_eig(graph, laplacian="combinatorial"):
    """The oracle's eigenvalues and eigenbasis of the graph's Laplacian (FP64 eigh), kept
    per graph for the session: the 4096-node grid is solved once for all tests."""
    key = _graph_key(graph, laplacian)
    if key not in _EIG_CACHE:
        L = O.laplacian_of(graph) if laplacian == "combinatorial" else O.normalized_laplacian_of(graph)
        _EIG_CACHE[key] = O.gft(L)
    return _EIG_CACHE[key]


def aligned_oracle_basis(graph, Uhat, sv_tol=1e-5, laplacian="combinatorial"):
    """Oracle eigenbasis rotated onto Uhat inside each eigenvalue cluster (sign / rotation
    are free in a GFT); asserts Uhat spans the oracle's eigenspaces."""
    lam, U = oracle_eig(graph, laplacian)
    Ua, min_sv = O.align(U, Uhat, lam)
    assert min_sv > 1 - sv_tol, f"GPU basis leaves the oracle eigenspaces: min singular value {min_sv}"
    return lam, Ua


def to_np(t):
    return t.double().cpu().numpy()
