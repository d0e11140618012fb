"""CPU FP64 oracle for the graph Fourier transform and its symmetry decomposition.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The library never calls it
and shares no code with it.

Every function is a plain, slow statement of a definition from Lu & Ortega, "Fast Graph
Fourier Transforms Based on Graph Symmetry and Bipartition":

* the Laplacian L = D - W + S and its conversions (Sec. II-B, eqs. def_laplacian,
  sw_from_l, l_from_sw) and the quadratic form (eq. lqf);
* the GFT: L = U diag(lambda) U^T, basis ordered by increasing eigenvalue, coefficient k
  of signal x equal to u_k^T x (Sec. II-B);
* the Haar butterfly stage B_{n,p} (eq. Bnp) and its permuted form B_phi (eq. B_phi);
* involutions and phi-symmetry (Sec. IV-A, Definitions 1-2, eq. p_phi);
* the block diagonalisation B_phi^T L B_phi (Thm. blockdiag) and the sub-graph weights
  of G+ and G- (Thm. decompose);
* the paper's error metrics RE, delta and epsilon (Sec. VI-B).

The fast transform is exact (it factors the same U), so the oracle for its output is the
dense definition itself: ``forward(X, U) = X @ U`` with ``U`` from ``numpy.linalg.eigh``.
Where eigenvalues repeat, any orthonormal basis of each eigenspace is a valid GFT
(Sec. III, the C4 example); ``align`` resolves that freedom before comparing.

Conventions: node labels are 0-based; signals are rows of X ([S, n], signal-major).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

SQRT2 = math.sqrt(2.0)


# --------------------------------------------------------------------------- Sec. II-B

def laplacian(n, src, dst, weight, self_loop=None):
    """Dense Laplacian L = D - W + S (eqs. def_laplacian and l_from_sw).

    l_ii = s_i + sum_{j != i} w_ij and l_ij = -w_ij for i != j.  Each undirected edge
    (src[e], dst[e]) is listed once; repeated listings add up.
    """
    L = np.zeros((n, n), dtype=np.float64)
    for i, j, w in zip(np.asarray(src), np.asarray(dst), np.asarray(weight, dtype=np.float64)):
        i, j = int(i), int(j)
        if i == j:
            raise ValueError("self-loops go in self_loop, not in the edge list")
        L[i, j] -= w
        L[j, i] -= w
        L[i, i] += w
        L[j, j] += w
    if self_loop is not None:
        L[np.arange(n), np.arange(n)] += np.asarray(self_loop, dtype=np.float64)
    return L


def laplacian_of(graph):
    """Laplacian of a ``workloads.Graph``."""
    return laplacian(graph.n, graph.src, graph.dst, graph.weight, graph.self_loop)


def degrees(n, src, dst, weight):
    """d_i = sum_{j != i} w_ij (the degree of eq. l_from_sw: self-loops excluded)."""
    d = np.zeros(n, dtype=np.float64)
    for i, j, w in zip(np.asarray(src), np.asarray(dst), np.asarray(weight, dtype=np.float64)):
        d[int(i)] += w
        d[int(j)] += w
    return d


def normalized_laplacian(n, src, dst, weight, self_loop=None):
    """Symmetric normalized Laplacian D^{-1/2} L D^{-1/2} (Sec. II-B), written entry by entry:
    l_ij / sqrt(d_i d_j) with L = D - W + S and d the degrees.  Every node needs d_i > 0."""
    L = laplacian(n, src, dst, weight, self_loop)
    d = degrees(n, src, dst, weight)
    if np.any(d <= 0):
        raise ValueError("the normalized Laplacian needs every node to have a positive degree")
    Ln = np.empty_like(L)
    for i in range(n):
        for j in range(n):
            Ln[i, j] = L[i, j] / np.sqrt(d[i] * d[j])
    return Ln


def normalized_laplacian_of(graph):
    return normalized_laplacian(graph.n, graph.src, graph.dst, graph.weight, graph.self_loop)


def weights_from_laplacian(L):
    """Inverse map of eq. sw_from_l: s_i = sum_j l_ij and w_ij = -l_ij (i != j)."""
    L = np.asarray(L, dtype=np.float64)
    s = L.sum(axis=1)
    W = -L.copy()
    np.fill_diagonal(W, 0.0)
    return W, s


def quadratic_form(f, n, src, dst, weight, self_loop=None):
    """f^T L f written as the sum of eq. lqf: sum_edges w (f_i - f_j)^2 + sum_k s_k f_k^2."""
    f = np.asarray(f, dtype=np.float64)
    q = 0.0
    for i, j, w in zip(src, dst, weight):
        q += float(w) * (f[int(i)] - f[int(j)]) ** 2
    if self_loop is not None:
        q += float(np.sum(np.asarray(self_loop) * f * f))
    return q


def gft(L):
    """GFT basis: eigenvectors of L as columns, ascending eigenvalue (Sec. II-B)."""
    lam, U = np.linalg.eigh(np.asarray(L, dtype=np.float64))
    return lam, U


def forward(X, U):
    """GFT coefficients of each signal row: C[s, k] = u_k^T x_s."""
    return np.asarray(X, dtype=np.float64) @ U


def inverse(C, U):
    """Inverse GFT by orthogonality of U: X[s] = U c_s."""
    return np.asarray(C, dtype=np.float64) @ U.T


# --------------------------------------------------------------------------- Sec. III

def bnp(n, p):
    """The butterfly stage B_{n,p} of eq. Bnp (p Haar units on i <-> n+1-i, 1-based)."""
    if not 0 <= 2 * p <= n:
        raise ValueError("need 0 <= p <= n/2")
    B = np.zeros((n, n))
    r = 1.0 / SQRT2
    for i in range(p):
        B[i, i] = r
        B[i, n - 1 - i] = r
        B[n - 1 - i, i] = r
        B[n - 1 - i, n - 1 - i] = -r
    for i in range(p, n - p):
        B[i, i] = 1.0
    return B


def haar_unit(x1, x2):
    """The Haar unit: diag(1,-1) Theta^T(1,2,pi/4) applied to (x1, x2) (Fig. haar)."""
    c = s = 1.0 / SQRT2
    # Theta(1,2,theta): Theta_11 = Theta_22 = cos, Theta_21 = sin, Theta_12 = -sin (eq. givens)
    theta_T = np.array([[c, s], [-s, c]])
    flip = np.array([[1.0, 0.0], [0.0, -1.0]])
    return flip @ theta_T @ np.array([x1, x2], dtype=np.float64)


# --------------------------------------------------------------------------- Sec. IV

def is_involution(phi):
    """Definition 1: phi(phi(i)) = i for every node."""
    phi = np.asarray(phi)
    n = len(phi)
    if np.any(phi < 0) or np.any(phi >= n):
        return False
    return bool(np.all(phi[phi] == np.arange(n)))


def p_phi(phi):
    """Number of Haar units of phi (eq. p_phi): half the number of non-fixed nodes."""
    phi = np.asarray(phi)
    return int(np.sum(phi != np.arange(len(phi)))) // 2


def partition(phi):
    """Node sets of Sec. IV-B: Z = fixed points, X = smaller label of each pair, Y = partners.

    Which side of the axis is X is a free choice; the smaller label is taken here.
    """
    phi = np.asarray(phi)
    idx = np.arange(len(phi))
    Z = idx[phi == idx]
    X = idx[phi > idx]
    Y = phi[X]
    return X, Y, Z


def is_phi_symmetric(W, s, phi, tol=0.0):
    """Definition 2: w_ij = w_phi(i)phi(j) for all i, j, including self-loops s_i = s_phi(i)."""
    phi = np.asarray(phi)
    W = np.asarray(W, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    ok_w = np.abs(W - W[np.ix_(phi, phi)]).max(initial=0.0) <= tol
    ok_s = np.abs(s - s[phi]).max(initial=0.0) <= tol
    return bool(ok_w and ok_s)


def b_phi(phi):
    """Orthogonal matrix B_phi of eq. B_phi (a permuted B_{n,p_phi})."""
    phi = np.asarray(phi)
    n = len(phi)
    X, Y, Z = partition(phi)
    B = np.zeros((n, n))
    r = 1.0 / SQRT2
    for i in X:
        B[i, i] = r
        B[i, phi[i]] = r
    for i in Y:
        B[i, i] = -r
        B[i, phi[i]] = r
    for i in Z:
        B[i, i] = 1.0
    return B


def decompose_matrix(L, phi):
    """L_phi = B_phi^T L B_phi and its two diagonal blocks (Thm. blockdiag, eq. Lpm).

    Returns (L_phi, L_plus, L_minus, plus_nodes, minus_nodes): L_plus is L_phi restricted
    to V+ = X u Z and L_minus to V- = Y, both in ascending node-label order.
    """
    B = b_phi(phi)
    Lphi = B.T @ np.asarray(L, dtype=np.float64) @ B
    X, Y, Z = partition(phi)
    plus = np.sort(np.concatenate([X, Z]))
    minus = np.sort(Y)
    return Lphi, Lphi[np.ix_(plus, plus)], Lphi[np.ix_(minus, minus)], plus, minus


def decompose_weights(W, s, phi):
    """Weights and self-loops of G+ and G- by the closed forms of Thm. decompose.

    Returns (W_plus, s_plus, plus_nodes, W_minus, s_minus, minus_nodes), with nodes in
    ascending label order.
    """
    phi = np.asarray(phi)
    W = np.asarray(W, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    X, Y, Z = partition(phi)
    Xs, Zs = set(X.tolist()), set(Z.tolist())
    plus = np.sort(np.concatenate([X, Z]))
    minus = np.sort(Y)

    Wp = np.zeros((len(plus), len(plus)))
    sp = np.zeros(len(plus))
    for a, i in enumerate(plus):
        for b, j in enumerate(plus):
            if i == j:
                continue
            if i in Xs and j in Xs:
                Wp[a, b] = W[i, j] + W[i, phi[j]]
            elif i in Zs and j in Zs:
                Wp[a, b] = W[i, j]
            else:
                Wp[a, b] = SQRT2 * W[i, j]
        if i in Xs:
            sp[a] = s[i] - (SQRT2 - 1.0) * sum(W[i, j] for j in Z)
        else:
            sp[a] = s[i] + (2.0 - SQRT2) * sum(W[i, j] for j in X)

    Wm = np.zeros((len(minus), len(minus)))
    sm = np.zeros(len(minus))
    for a, i in enumerate(minus):
        for b, j in enumerate(minus):
            if i != j:
                Wm[a, b] = W[i, j] - W[i, phi[j]]
        sm[a] = s[i] + 2.0 * sum(W[i, j] for j in X) + sum(W[i, j] for j in Z)
    return Wp, sp, plus, Wm, sm, minus


def laplacian_from_weights(W, s):
    """Dense Laplacian from a weight matrix (zero diagonal) and self-loops (eq. l_from_sw)."""
    W = np.asarray(W, dtype=np.float64)
    L = -W.copy()
    np.fill_diagonal(L, 0.0)
    L[np.diag_indices_from(L)] = np.asarray(s) + W.sum(axis=1) - np.diag(W)
    return L


def involutions(n):
    """All involutions of {0..n-1} by brute force (each one is a set of disjoint pairs)."""
    out = []

    def rec(phi, i):
        while i < n and phi[i] != -1:
            i += 1
        if i == n:
            out.append(np.array(phi, dtype=np.int32))
            return
        phi[i] = i
        rec(phi, i + 1)
        for j in range(i + 1, n):
            if phi[j] == -1:
                phi[i], phi[j] = j, i
                rec(phi, i + 1)
                phi[i], phi[j] = -1, -1
        phi[i] = -1

    rec([-1] * n, 0)
    return out


def involution_count(n):
    """Number of involutions T(n) = sum_k n! / (2^k (n-2k)! k!) (Sec. V-F)."""
    return sum(math.factorial(n) // (2 ** k * math.factorial(n - 2 * k) * math.factorial(k))
               for k in range(n // 2 + 1))


def connected_components(L, tol=0.0):
    """Connected components of the graph whose Laplacian is L (nonzero off-diagonals)."""
    n = L.shape[0]
    seen = np.zeros(n, dtype=bool)
    comps = []
    for r in range(n):
        if seen[r]:
            continue
        stack, comp = [r], []
        seen[r] = True
        while stack:
            v = stack.pop()
            comp.append(v)
            for u in np.nonzero(np.abs(L[v]) > tol)[0]:
                if u != v and not seen[u]:
                    seen[u] = True
                    stack.append(u)
        comps.append(sorted(comp))
    return comps


# --------------------------------------------------------------------------- comparison

def clusters(lam, tol=None):
    """Group ascending eigenvalues into clusters of (numerically) repeated values.

    Consecutive eigenvalues closer than ``tol`` (default 1e-9 * max(1, |lambda|_max)) join
    one cluster.  Returns a list of index arrays.
    """
    lam = np.asarray(lam, dtype=np.float64)
    if tol is None:
        tol = 1e-9 * max(1.0, float(np.abs(lam).max(initial=0.0)))
    groups, cur = [], [0]
    for k in range(1, len(lam)):
        if lam[k] - lam[k - 1] <= tol:
            cur.append(k)
        else:
            groups.append(np.array(cur))
            cur = [k]
    if len(lam):
        groups.append(np.array(cur))
    return groups


def polar(M):
    """Orthogonal polar factor of a square matrix (nearest orthogonal matrix)."""
    A, _, Bt = np.linalg.svd(M)
    return A @ Bt


def align(U_ref, U_hat, lam, tol=None):
    """Rotate the reference basis onto U_hat inside each eigenvalue cluster.

    For a cluster C with M = U_ref[:, C]^T U_hat[:, C], Q_C = polar(M) is the orthogonal
    map (a sign when |C| = 1) that best carries U_ref[:, C] to U_hat[:, C].  Returns
    (U_aligned = U_ref @ blockdiag(Q_C), min_sv) where min_sv is the smallest singular
    value of any M: close to 1 iff U_hat spans the same eigenspaces as U_ref.
    """
    U_ref = np.asarray(U_ref, dtype=np.float64)
    U_hat = np.asarray(U_hat, dtype=np.float64)
    out = np.empty_like(U_ref)
    min_sv = np.inf
    for C in clusters(lam, tol):
        M = U_ref[:, C].T @ U_hat[:, C]
        sv = np.linalg.svd(M, compute_uv=False)
        min_sv = min(min_sv, float(sv.min()))
        out[:, C] = U_ref[:, C] @ polar(M)
    return out, min_sv


def relative_error(A, B):
    """||A - B||_F / ||B||_F."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    den = np.linalg.norm(B)
    return float(np.linalg.norm(A - B) / (den if den > 0 else 1.0))


def max_row_relative_error(A, B):
    """Largest per-signal relative error max_s ||a_s - b_s|| / ||b_s|| over the rows (signals)
    of A and B: the signal-by-signal form of ``relative_error`` (a row of B that is zero counts
    with a denominator of 1e-300)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    num = np.linalg.norm(A - B, axis=1)
    den = np.maximum(np.linalg.norm(B, axis=1), 1e-300)
    return float((num / den).max(initial=0.0))


def re_metric(U_hat, U):
    """Relative error RE(U_hat, U) = ||U - U_hat||_F / ||U||_F (eq. re)."""
    return float(np.linalg.norm(U - U_hat) / np.linalg.norm(U))


def delta_metric(U_hat, U):
    """Sign-normalised error delta = || |U_hat^T U| - I ||_F / sqrt(n) (Sec. VI-B)."""
    n = U.shape[0]
    return float(np.linalg.norm(np.abs(U_hat.T @ U) - np.eye(n)) / math.sqrt(n))


def epsilon_metric(U_hat, U, X):
    """Empirical error (1/M) sum_i sum_j (|u_j^T x_i| - |uhat_j^T x_i|)^2 (Sec. VI-B)."""
    X = np.asarray(X, dtype=np.float64)
    return float(np.mean(np.sum((np.abs(X @ U) - np.abs(X @ U_hat)) ** 2, axis=1)))


# --------------------------------------------------------------------------- closed forms

def dct2_matrix(N):
    """Orthonormal DCT-II basis as columns: u_k(i) = a_k cos(pi k (2i+1) / (2N))."""
    i = np.arange(N)[:, None]
    k = np.arange(N)[None, :]
    U = np.cos(np.pi * k * (2 * i + 1) / (2 * N)) * math.sqrt(2.0 / N)
    U[:, 0] /= SQRT2
    return U


def dst4_matrix(N):
    """Orthonormal DST-IV basis as columns: u_k(i) = sqrt(2/N) sin(pi (2i+1)(2k+1) / (4N))."""
    i = np.arange(N)[:, None]
    k = np.arange(N)[None, :]
    return math.sqrt(2.0 / N) * np.sin(np.pi * (2 * i + 1) * (2 * k + 1) / (4 * N))


def path_eigenvalues(N):
    """Eigenvalues 2 - 2 cos(pi k / N) of the unit-weight N-node path, ascending."""
    return 2.0 - 2.0 * np.cos(np.pi * np.arange(N) / N)


def cycle_eigenvalues(n):
    """Eigenvalues 2 - 2 cos(2 pi k / n) of the unit-weight n-cycle, ascending."""
    return np.sort(2.0 - 2.0 * np.cos(2.0 * np.pi * np.arange(n) / n))


# --------------------------------------------------------------------------- op counts

def matrix_gft_ops(n):
    """Adds and multiplies of a dense n x n matrix-vector GFT (Table tab:runtime)."""
    return n * (n - 1), n * n


def brute_force_gft_apply(X, U):
    """Coefficient-by-coefficient C[s, k] = sum_i U[i, k] X[s, i] (for tiny inputs)."""
    X = np.asarray(X, dtype=np.float64)
    S, n = X.shape
    C = np.zeros((S, U.shape[1]))
    for s, k, i in itertools.product(range(S), range(U.shape[1]), range(n)):
        C[s, k] += U[i, k] * X[s, i]
    return C
