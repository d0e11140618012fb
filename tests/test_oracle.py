"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Each test checks an oracle function against something other than itself: a closed form,
a value printed in the paper (``tests/golden``), an independent formula for the same
quantity, an invariant, or brute force on tiny inputs.
"""
import math
import os

import numpy as np
import pytest

import workloads as wl
from oracle import gft_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_graph(n, rng, p=0.5, loops=True):
    src, dst, w = [], [], []
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < p:
                src.append(i)
                dst.append(j)
                w.append(rng.uniform(0.1, 2.0))
    s = rng.uniform(0.0, 1.0, n) if loops else None
    return np.array(src), np.array(dst), np.array(w), s


def _sym_graph(phi, rng, p=0.6):
    """Random phi-symmetric weighted graph with self-loops (Definition 2)."""
    n = len(phi)
    W = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            if W[i, j] == 0 and rng.random() < p:
                w = rng.uniform(0.1, 2.0)
                for a, b in ((i, j), (phi[i], phi[j])):
                    if a != b:
                        W[a, b] = W[b, a] = w
    s = rng.uniform(0.0, 1.0, n)
    s = 0.5 * (s + s[phi])
    return W, s


# ------------------------------------------------------------------ Laplacian (Sec. II-B)

def test_laplacian_matches_quadratic_form():
    """eq. lqf: f^T L f equals the edge/self-loop sum, for random graphs and signals."""
    rng = np.random.default_rng(1)
    for n in (1, 2, 5, 9):
        src, dst, w, s = _rand_graph(n, rng)
        L = O.laplacian(n, src, dst, w, s)
        for _ in range(4):
            f = rng.standard_normal(n)
            assert f @ L @ f == pytest.approx(O.quadratic_form(f, n, src, dst, w, s), rel=1e-12, abs=1e-12)


def test_laplacian_round_trips_through_weights():
    """eqs. sw_from_l and l_from_sw invert each other; diagonal uses s_i + sum_{j!=i} w_ij."""
    rng = np.random.default_rng(2)
    src, dst, w, s = _rand_graph(7, rng)
    L = O.laplacian(7, src, dst, w, s)
    W, s2 = O.weights_from_laplacian(L)
    np.testing.assert_allclose(s2, s, atol=1e-13)
    for a, b, x in zip(src, dst, w):
        assert W[a, b] == pytest.approx(x) and W[b, a] == pytest.approx(x)
    np.testing.assert_allclose(O.laplacian_from_weights(W, s2), L, atol=1e-13)
    # row sums of L are the self-loops (eq. sw_from_l), so with no loops L 1 = 0
    L0 = O.laplacian(7, src, dst, w, None)
    np.testing.assert_allclose(L0 @ np.ones(7), 0.0, atol=1e-12)


# ------------------------------------------------------------------ GFT closed forms

def test_uniform_path_is_dct2():
    """Unit-weight path: GFT = DCT-II (Sec. I), eigenvalues 2 - 2cos(pi k/N)."""
    for N in (2, 3, 8, 13):
        g = wl.path(N)
        lam, U = O.gft(O.laplacian_of(g))
        np.testing.assert_allclose(lam, O.path_eigenvalues(N), atol=1e-12)
        D = O.dct2_matrix(N)
        # distinct eigenvalues: only the sign of each column is free
        np.testing.assert_allclose(np.abs(U.T @ D), np.eye(N), atol=1e-12)


def test_forward_matches_dct_formula_elementwise():
    """C[s,k] = a_k sum_i x_i cos(pi k (2i+1)/2N) up to one sign per k (pins X @ U vs X @ U^T)."""
    rng = np.random.default_rng(3)
    N = 8
    X = rng.standard_normal((5, N))
    lam, U = O.gft(O.laplacian_of(wl.path(N)))
    C = O.forward(X, U)
    for k in range(N):
        a = math.sqrt(1.0 / N) if k == 0 else math.sqrt(2.0 / N)
        ref = np.array([a * sum(X[s, i] * math.cos(math.pi * k * (2 * i + 1) / (2 * N)) for i in range(N))
                        for s in range(5)])
        sign = np.sign(U[0, k])   # DCT-II columns are positive at node 0
        np.testing.assert_allclose(C[:, k], sign * ref, atol=1e-12)
    np.testing.assert_allclose(O.inverse(C, U), X, atol=1e-12)


def test_forward_matches_brute_force_sum():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((3, 6))
    src, dst, w, s = _rand_graph(6, rng)
    lam, U = O.gft(O.laplacian(6, src, dst, w, s))
    np.testing.assert_allclose(O.forward(X, U), O.brute_force_gft_apply(X, U), atol=1e-12)


def test_path_with_loop_two_is_dst4():
    """Path with a self-loop of weight 2 on its first node: GFT = DST-IV (Sec. I)."""
    for N in (4, 8):
        loops = np.zeros(N)
        loops[0] = 2.0
        lam, U = O.gft(O.laplacian_of(wl.path(N, loops=loops)))
        np.testing.assert_allclose(np.abs(U.T @ O.dst4_matrix(N)), np.eye(N), atol=1e-12)


def test_cycle_eigenvalues():
    for n in (3, 4, 12, 80):
        lam, _ = O.gft(O.laplacian_of(wl.cycle(n)))
        np.testing.assert_allclose(lam, O.cycle_eigenvalues(n), atol=1e-11)


def test_grid_is_kronecker_dct():
    """Uniform grid: GFT = DCT-II (x) DCT-II (Sec. V-D), up to rotations in eigenspaces."""
    N = 8
    lam, U = O.gft(O.laplacian_of(wl.grid(N, N)))
    D = O.dct2_matrix(N)
    K = np.kron(D, D)     # node k*N + l  <->  row index of kron
    mu = O.path_eigenvalues(N)
    klam = (mu[:, None] + mu[None, :]).reshape(-1)
    order = np.argsort(klam, kind="stable")
    np.testing.assert_allclose(lam, klam[order], atol=1e-12)
    Ua, min_sv = O.align(U, K[:, order], lam)
    assert min_sv > 1 - 1e-10
    np.testing.assert_allclose(Ua, K[:, order], atol=1e-10)
    # multiplicity 7 at eigenvalue 4, 25 pairs, 33 distinct values
    sizes = sorted(len(c) for c in O.clusters(lam))
    assert len(sizes) == 33 and sizes.count(2) == 25 and sizes.count(7) == 1


def test_c4_worked_example():
    """The 4-cycle GFT printed in Sec. III is an eigenbasis of the cycle Laplacian."""
    rows, lam_ref = [], None
    scale = 1.0
    for line in open(os.path.join(GOLDEN, "c4_cycle.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        if line.startswith("scale"):
            scale = float(line.split()[1])
        elif line.startswith("eigenvalues"):
            lam_ref = np.array([float(v) for v in line.split()[1:]])
        else:
            rows.append([float(v) for v in line.split()])
    Uc4 = scale * np.array(rows)
    L = O.laplacian_of(wl.cycle(4))
    np.testing.assert_allclose(Uc4.T @ Uc4, np.eye(4), atol=1e-15)
    np.testing.assert_allclose(Uc4.T @ L @ Uc4, np.diag(lam_ref), atol=1e-14)
    lam, U = O.gft(L)
    np.testing.assert_allclose(lam, lam_ref, atol=1e-13)
    Ua, min_sv = O.align(U, Uc4, lam)
    assert min_sv > 1 - 1e-12
    np.testing.assert_allclose(Ua, Uc4, atol=1e-12)


# ------------------------------------------------------------------ alignment

def test_align_recovers_rotation_and_flags_wrong_space():
    rng = np.random.default_rng(5)
    lam = np.array([0.0, 1.0, 1.0, 1.0, 2.5, 3.0, 3.0])
    U, _ = np.linalg.qr(rng.standard_normal((7, 7)))
    Q = np.eye(7)
    for C in O.clusters(lam):
        Qc, _ = np.linalg.qr(rng.standard_normal((len(C), len(C))))
        Q[np.ix_(C, C)] = Qc
    Uhat = U @ Q
    Ua, min_sv = O.align(U, Uhat, lam)
    assert min_sv > 1 - 1e-12
    np.testing.assert_allclose(Ua, Uhat, atol=1e-12)
    # swapping two columns from different eigenspaces is detected
    bad = Uhat.copy()
    bad[:, [0, 4]] = bad[:, [4, 0]]
    _, sv_bad = O.align(U, bad, lam)
    assert sv_bad < 0.5


def test_paper_error_metrics():
    """RE vs its second form in eq. re; delta ignores signs; epsilon of an exact basis is 0."""
    rng = np.random.default_rng(6)
    U, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    V, _ = np.linalg.qr(U + 0.01 * rng.standard_normal((6, 6)))
    assert O.re_metric(V, U) == pytest.approx(np.linalg.norm(V.T @ U - np.eye(6)) / math.sqrt(6), rel=1e-12)
    S = np.diag([1, -1, 1, -1, -1, 1.0])
    assert O.delta_metric(U @ S, U) < 1e-14
    X = rng.standard_normal((10, 6))
    assert O.epsilon_metric(U @ S, U, X) < 1e-24


def test_paper_error_metrics_worked_examples():
    """delta, epsilon and RE of Sec. VI-B on small bases worked out by hand, with non-zero
    error, so that a wrong normalisation (1/n for 1/sqrt(n), a sum for the mean over signals)
    or a missing absolute value fails.

    2x2: U = I and U_hat the rotation by 60 degrees, columns (1/2, sqrt3/2), (-sqrt3/2, 1/2).
      |U_hat^T U| - I = [[-1/2, sqrt3/2], [sqrt3/2, -1/2]]: squared Frobenius norm 2, so
      delta = sqrt(2) / sqrt(2) = 1; RE = ||U - U_hat||_F / ||U||_F = sqrt(2) / sqrt(2) = 1.
      Signals x1 = (1, 0), x2 = (0, 2): true coefficients (1, 0) and (0, 2), the rotated
      basis gives (1/2, -sqrt3/2) and (sqrt3, 1); the squared differences of magnitudes sum
      to 1/4 + 3/4 = 1 and 3 + 1 = 4, so epsilon = (1 + 4) / 2 = 5/2.
    3x3: U_hat = [[0.6, -0.8, 0], [0.8, 0.6, 0], [0, 0, 1]]: |U_hat^T| - I has entries
      -0.4, -0.4, 0.8, 0.8 and zeros, squared norm 1.6, so delta = sqrt(1.6 / 3); a sign
      flip of any column of U_hat leaves delta unchanged (RE then changes).
    """
    c, s = 0.5, math.sqrt(3.0) / 2.0
    U = np.eye(2)
    Uh = np.array([[c, -s], [s, c]])
    assert O.delta_metric(Uh, U) == pytest.approx(1.0, abs=1e-15)
    assert O.re_metric(Uh, U) == pytest.approx(1.0, abs=1e-15)
    X = np.array([[1.0, 0.0], [0.0, 2.0]])
    assert O.epsilon_metric(Uh, U, X) == pytest.approx(2.5, abs=1e-14)
    U3 = np.eye(3)
    V3 = np.array([[0.6, -0.8, 0.0], [0.8, 0.6, 0.0], [0.0, 0.0, 1.0]])
    assert O.delta_metric(V3, U3) == pytest.approx(math.sqrt(1.6 / 3.0), abs=1e-15)
    V3f = V3 @ np.diag([1.0, -1.0, -1.0])
    assert O.delta_metric(V3f, U3) == pytest.approx(math.sqrt(1.6 / 3.0), abs=1e-15)
    assert O.re_metric(V3f, U3) > O.re_metric(V3, U3)
    # epsilon on the 3x3 pair: x = (1, 1, 1) has true coefficients (1, 1, 1) and rotated
    # ones (1.4, -0.2, 1): (1 - 1.4)^2 + (1 - 0.2)^2 = 0.16 + 0.64 = 0.8 (one signal)
    assert O.epsilon_metric(V3, U3, np.ones((1, 3))) == pytest.approx(0.8, abs=1e-14)


def test_max_row_relative_error_worked_example():
    """Per-signal relative error on rows worked out by hand: row 0 ||(0, 4)|| / ||(3, 0)|| =
    4/3, row 1 ||(0, -1)|| / ||(0, 2)|| = 1/2, so the maximum is 4/3 (the batch Frobenius form
    gives sqrt(17/13), the column-wise one sqrt(17)/2: both differ)."""
    A = np.array([[3.0, 4.0], [0.0, 1.0]])
    B = np.array([[3.0, 0.0], [0.0, 2.0]])
    assert O.max_row_relative_error(A, B) == pytest.approx(4.0 / 3.0, abs=1e-15)
    assert O.relative_error(A, B) == pytest.approx(math.sqrt(17.0 / 13.0), abs=1e-15)
    assert O.max_row_relative_error(B, B) == 0.0
    assert O.max_row_relative_error(np.zeros((0, 2)), np.zeros((0, 2))) == 0.0


# ------------------------------------------------------------------ Haar stages (Sec. III)

def test_haar_unit_is_scaled_sum_and_difference():
    """Fig. haar: a Haar unit maps (x1,x2) to ((x1+x2)/sqrt2, (x1-x2)/sqrt2)."""
    y = O.haar_unit(3.0, 1.0)
    np.testing.assert_allclose(y, [4 / math.sqrt(2), 2 / math.sqrt(2)], atol=1e-15)


def test_bnp_action_matches_elementwise_definition():
    """eq. Bnp and the element formula printed after it; B symmetric and orthogonal."""
    rng = np.random.default_rng(7)
    for n, p in ((8, 4), (8, 3), (7, 3), (5, 0), (6, 1)):
        B = O.bnp(n, p)
        x = rng.standard_normal(n)
        y = B @ x
        for i in range(1, n + 1):          # 1-based, as printed
            if i <= p:
                ref = (x[i - 1] + x[n - i]) / math.sqrt(2)
            elif i <= n - p:
                ref = x[i - 1]
            else:
                ref = (-x[i - 1] + x[n - i]) / math.sqrt(2)
            assert y[i - 1] == pytest.approx(ref, abs=1e-14)
        np.testing.assert_allclose(B, B.T, atol=0)
        np.testing.assert_allclose(B @ B, np.eye(n), atol=1e-15)


def test_bphi_is_permuted_bnp():
    """B_phi (eq. B_phi) for the reversal phi equals B_{n,p} of eq. Bnp."""
    for n in (4, 5, 8, 9):
        np.testing.assert_allclose(O.b_phi(wl.reversal(n)), O.bnp(n, n // 2), atol=0)
    rng = np.random.default_rng(8)
    for phi in O.involutions(6)[::7]:
        B = O.b_phi(phi)
        np.testing.assert_allclose(B.T @ B, np.eye(6), atol=1e-15)
        np.testing.assert_allclose(B @ B, np.eye(6), atol=1e-15)


def test_golden_involutions():
    for line in open(os.path.join(GOLDEN, "involutions.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tok = line.split()
        phi = np.array([int(v) - 1 for v in tok[1:5]])
        assert O.is_involution(phi)
        assert O.p_phi(phi) == int(tok[6])
        if tok[0] == "phi_b":
            X, Y, Z = O.partition(phi)
            assert list(X) == [0] and list(Y) == [3] and list(Z) == [1, 2]


def test_involution_enumeration_matches_count_formula():
    """Brute-force enumeration vs T(n) of Sec. V-F (T(8) = 764)."""
    for n in range(1, 9):
        invs = O.involutions(n)
        assert len(invs) == O.involution_count(n)
        assert len({tuple(p) for p in invs}) == len(invs)
        assert all(O.is_involution(p) for p in invs)
    assert O.involution_count(8) == 764
    assert not O.is_involution(np.array([1, 2, 0]))


# ------------------------------------------------------------------ decomposition (Sec. IV)

def test_decompose_closed_form_matches_block_product():
    """Thm. decompose (weights) equals the blocks of B_phi^T L B_phi (eqs. blkdiag_G, Lpm)."""
    rng = np.random.default_rng(9)
    cases = [wl.reversal(8), wl.reversal(9), np.array([3, 1, 2, 0]),
             np.array([0, 4, 2, 6, 1, 5, 3, 7, 8])]
    for phi in cases:
        for _ in range(3):
            W, s = _sym_graph(phi, rng)
            L = O.laplacian_from_weights(W, s)
            Lphi, Lp, Lm, plus, minus = O.decompose_matrix(L, phi)
            Wp, sp, plus2, Wm, sm, minus2 = O.decompose_weights(W, s, phi)
            assert list(plus) == list(plus2) and list(minus) == list(minus2)
            np.testing.assert_allclose(O.laplacian_from_weights(Wp, sp), Lp, atol=1e-13)
            np.testing.assert_allclose(O.laplacian_from_weights(Wm, sm), Lm, atol=1e-13)
            # Thm. blockdiag: zero coupling between V_X u V_Z and V_Y
            np.testing.assert_allclose(Lphi[np.ix_(plus, minus)], 0.0, atol=1e-13)


def test_decomposition_yields_eigenbasis():
    """Lemma graph_sym: B_phi diag(U+, U-) is a GFT of a phi-symmetric graph."""
    rng = np.random.default_rng(10)
    phi = np.array([5, 1, 4, 3, 2, 0, 6])
    W, s = _sym_graph(phi, rng)
    L = O.laplacian_from_weights(W, s)
    _, Lp, Lm, plus, minus = O.decompose_matrix(L, phi)
    n = len(phi)
    V = np.zeros((n, n))
    lp, Up = O.gft(Lp)
    lm, Um = O.gft(Lm)
    V[np.ix_(plus, np.arange(len(plus)))] = Up
    V[np.ix_(minus, len(plus) + np.arange(len(minus)))] = Um
    U = O.b_phi(phi) @ V
    lam = np.concatenate([lp, lm])
    np.testing.assert_allclose(U.T @ U, np.eye(n), atol=1e-13)
    np.testing.assert_allclose(L @ U, U * lam, atol=1e-12)
    np.testing.assert_allclose(np.sort(lam), O.gft(L)[0], atol=1e-12)


def test_removal_cases_of_sec4c():
    """The three edge-removal cases described after Thm. decompose."""
    # case 1: edge b between i in X and phi(i) in Y -> self-loop 2b in G-
    b = 0.7
    W = np.array([[0, b], [b, 0.0]])
    _, _, _, Wm, sm, _ = O.decompose_weights(W, np.zeros(2), np.array([1, 0]))
    assert sm[0] == pytest.approx(2 * b)
    # case 3: edges d from a Z node to i and phi(i): one edge sqrt2 d kept in G+,
    # self-loops -(sqrt2-1)d on the X node and (2-sqrt2)d on the Z node, self-loop d in G-
    d = 1.3
    W = np.zeros((3, 3))
    W[0, 1] = W[1, 0] = W[2, 1] = W[1, 2] = d
    Wp, sp, plus, Wm, sm, minus = O.decompose_weights(W, np.zeros(3), np.array([2, 1, 0]))
    assert list(plus) == [0, 1] and list(minus) == [2]
    assert Wp[0, 1] == pytest.approx(math.sqrt(2) * d)
    assert sp[0] == pytest.approx(-(math.sqrt(2) - 1) * d)
    assert sp[1] == pytest.approx((2 - math.sqrt(2)) * d)
    assert sm[0] == pytest.approx(d)


def test_symmetry_iff_block_diagonal_brute_force():
    """Lemma graph_sym / Thm. blockdiag by brute force over every involution of n <= 6.

    A graph symmetric under one involution phi0 is tested against all T(n) involutions:
    Definition 2 holds for phi exactly when B_phi^T L B_phi decouples V_X u V_Z from V_Y.
    """
    rng = np.random.default_rng(11)
    for n in (3, 4, 5, 6):
        invs = O.involutions(n)
        for trial in range(3):
            phi0 = invs[rng.integers(len(invs))]
            W, s = _sym_graph(phi0, rng, p=0.7)
            L = O.laplacian_from_weights(W, s)
            nsym = 0
            for phi in invs:
                sym = O.is_phi_symmetric(W, s, phi, tol=1e-12)
                Lphi, _, _, plus, minus = O.decompose_matrix(L, phi)
                decoupled = np.abs(Lphi[np.ix_(plus, minus)]).max(initial=0.0) < 1e-12
                assert sym == decoupled, (n, phi0, phi)
                nsym += sym
            trivial = bool(np.all(phi0 == np.arange(n)))
            assert nsym >= (1 if trivial else 2)    # identity and phi0


def test_two_sparse_eigenvector_lemma():
    """Lemma 2sparse: star / complete graphs have eigenvectors (e_i - e_j)/sqrt2."""
    n = 6
    star = wl._graph(n, [(0, j) for j in range(1, n)])
    comp = wl._graph(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
    for g, (i, j) in ((star, (2, 5)), (comp, (0, 3))):
        L = O.laplacian_of(g)
        u = np.zeros(n)
        u[i], u[j] = 1 / math.sqrt(2), -1 / math.sqrt(2)
        Lu = L @ u
        lam = u @ Lu
        np.testing.assert_allclose(Lu, lam * u, atol=1e-13)


def test_k_regular_bipartite_eigen_pairing():
    """Lemma k-rbg: (u1; u2) with lambda gives (u1; -u2) with 2k - lambda."""
    # 2-regular bipartite: the 8-cycle with parts {even}, {odd}, relabelled evens first
    n = 8
    order = list(range(0, n, 2)) + list(range(1, n, 2))
    pos = {v: i for i, v in enumerate(order)}
    edges = [(pos[i], pos[(i + 1) % n]) for i in range(n)]
    L = O.laplacian_of(wl._graph(n, edges))
    lam, U = O.gft(L)
    for k in range(n):
        u = U[:, k].copy()
        u[n // 2:] *= -1
        np.testing.assert_allclose(L @ u, (4 - lam[k]) * u, atol=1e-12)


def test_normalized_laplacian_closed_forms():
    """Symmetric normalized Laplacian (Sec. II-B) pinned without its own formula:
    k-regular graphs give L / k (cycle: 1 - cos(2 pi k / n)); the unweighted path has
    eigenvalues 1 - cos(pi k / (n - 1)); D^{1/2} 1 spans the null space; the spectrum equals
    that of the random-walk Laplacian D^{-1} L (a similar matrix, computed separately)."""
    n = 10
    lam = np.linalg.eigvalsh(O.normalized_laplacian_of(wl.cycle(n)))
    np.testing.assert_allclose(lam, np.sort(1 - np.cos(2 * np.pi * np.arange(n) / n)), atol=1e-13)
    for n in (2, 3, 7, 16):
        lam = np.linalg.eigvalsh(O.normalized_laplacian_of(wl.path(n)))
        np.testing.assert_allclose(lam, np.sort(1 - np.cos(np.pi * np.arange(n) / (n - 1))), atol=1e-13)
    g = wl._graph(12, [(i, i + 1) for i in range(11)] + [(0, 5), (3, 9)],
                  wl.rng_for(9, 1).uniform(0.1, 1.0, 13))
    d = O.degrees(g.n, g.src, g.dst, g.weight)
    Ln = O.normalized_laplacian_of(g)
    np.testing.assert_allclose(Ln @ np.sqrt(d), 0, atol=1e-13)
    rw = np.sort(np.linalg.eigvals(np.diag(1 / d) @ O.laplacian_of(g)).real)
    np.testing.assert_allclose(np.linalg.eigvalsh(Ln), rw, atol=1e-12)
    with pytest.raises(ValueError):
        O.normalized_laplacian(3, [0], [1], [1.0])        # node 2 has no edge


def test_normalized_bipartite_spectrum_is_symmetric_about_one():
    """Normalized-Laplacian analogue of Lemma k-rbg: for any bipartite graph, (u1; -u2) is an
    eigenvector with eigenvalue 2 - lambda (parts listed first / second)."""
    rng = wl.rng_for(9, 2)
    p, q = 5, 8
    edges, wts = [], []
    for i in range(p):
        for j in range(q):
            if rng.random() < 0.5 or j == i:
                edges.append((i, p + j))
                wts.append(rng.uniform(0.5, 1.5))
    g = wl._graph(p + q, edges, wts)
    Ln = O.normalized_laplacian_of(g)
    lam, U = O.gft(Ln)
    for k in range(p + q):
        u = U[:, k].copy()
        u[p:] *= -1
        np.testing.assert_allclose(Ln @ u, (2 - lam[k]) * u, atol=1e-12)


def test_connected_components():
    g = wl._graph(7, [(0, 1), (1, 2), (3, 4), (5, 6)])
    comps = O.connected_components(O.laplacian_of(g))
    assert comps == [[0, 1, 2], [3, 4], [5, 6]]


def test_matrix_gft_op_counts_match_table3():
    for line in open(os.path.join(GOLDEN, "table3_opcounts.txt")):
        line = line.split("#")[0].strip()
        if not line:
            continue
        t = line.split()
        assert O.matrix_gft_ops(int(t[1])) == (int(t[2]), int(t[3]))
