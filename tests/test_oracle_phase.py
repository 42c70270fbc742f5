"""Pins of the oracle's phase recovery (Section 2), CPU only."""
import os

import numpy as np
import pytest

import workloads as W
from oracle.metrics import eps_K
from oracle.phase import (mround, partition2, randomized_svd, recovery_path_general,
                          recovery_path_lattice, recovery_vector2, recovery_vector2_prefix,
                          low_rank_factorization, wrapped_phase)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load_fig5():
    path, subs, cut = [], {}, None
    for line in open(os.path.join(GOLD, "partition_fig5.txt")):
        p = line.split()
        if not p or p[0].startswith("#"):
            continue
        if p[0] == "path":
            path.append((int(p[1]), int(p[2])))
        elif p[0] == "cut":
            cut = int(p[1])
        elif p[0] == "sub":
            subs.setdefault(int(p[1]), []).append((int(p[2]), int(p[3])))
    return np.array(path), cut, subs


def test_partition2_worked_example():
    P, cut, subs = _load_fig5()
    parts = partition2(P, 1, [1, cut])
    assert [r for r, _ in parts] == [1, 4]
    for r, sub in parts:
        assert [tuple(x) for x in sub.tolist()] == subs[r]


def _check_def23(P, N, root, adjacency):
    # Definition 2.3: P(:,2) a permutation of all nodes but the root, non-decreasing
    # depth, P(i,1) the predecessor of P(i,2)
    assert sorted(P[:, 1].tolist()) == sorted(set(range(N)) - {root})
    depth = {root: 0}
    for bg, ed in P:
        assert bg in depth, "predecessor must precede its child"
        depth[ed] = depth[bg] + 1
        assert adjacency(bg, ed)
    ds = [depth[e] for e in P[:, 1]]
    assert ds == sorted(ds)


@pytest.mark.parametrize("d,n", [(2, 8), (3, 5)])
def test_lattice_comb_tree_is_a_valid_path(d, n):
    q = (n // 2,) * d
    P = recovery_path_lattice(d, n, q)
    root = int(np.ravel_multi_index(q, (n,) * d))
    coords = np.array(np.unravel_index(np.arange(n ** d), (n,) * d)).T
    _check_def23(P, n ** d, root, lambda a, b: np.abs(coords[a] - coords[b]).sum() == 1)
    # depth equals the Manhattan distance: every edge is a unit axis edge (minimum spanning weight)
    assert len(P) == n ** d - 1


def test_general_path_is_mst_bfs():
    rng = W.rng(21, 0)
    X = rng.random((60, 2))
    P = recovery_path_general(X, root=0)
    _check_def23(P, 60, 0, lambda a, b: True)
    # weight equals the MST of the complete graph (the DT contains an MST); brute-force Prim
    w = np.linalg.norm(X[P[:, 0]] - X[P[:, 1]], axis=1).sum()
    D = np.linalg.norm(X[:, None] - X[None], axis=2)
    inT = np.zeros(60, bool)
    inT[0] = True
    best = D[0].copy()
    tot = 0.0
    for _ in range(59):
        best[inT] = np.inf
        j = int(np.argmin(best))
        tot += best[j]
        inT[j] = True
        best = np.minimum(best, D[j])
    assert abs(w - tot) < 1e-12


def test_round_half_away_from_zero():
    assert mround(np.array([0.5, -0.5, 1.5, -1.49, 2.5]) ).tolist() == [1.0, -1.0, 2.0, -1.0, 3.0]


def test_recovery_vector2_unwraps_smooth_phase_exactly():
    n = 16
    P = recovery_path_lattice(2, n, (0, 0))
    a = np.array(np.unravel_index(np.arange(n * n), (n, n))).T / n
    phi = 3.1 * a[:, 0] - 2.3 * a[:, 1] + 1.7 * a[:, 0] * a[:, 1] + 5.2
    u = wrapped_phase(np.exp(2j * np.pi * phi))
    v, D = recovery_vector2(u, 0.25, P, 0)
    shift = v - phi
    assert np.allclose(shift, np.round(shift[0]), atol=1e-12)   # v = phi + integer constant
    assert D == [0]


def test_recovery_vector2_flags_jump():
    n = 16
    P = recovery_path_lattice(2, n, (0, 0))
    a = np.array(np.unravel_index(np.arange(n * n), (n, n))).T / n
    phi = 0.5 * a[:, 0] + np.where(a[:, 1] >= 0.5, 0.35, 0.0)
    u = wrapped_phase(np.exp(2j * np.pi * phi))
    _, D = recovery_vector2(u, 0.25, P, 0)
    flagged = np.array(D[1:])
    assert len(flagged) == n and (a[flagged, 1] == 0.5).all()


def test_loop_equals_prefix_sum():
    rng = W.rng(22, 0)
    X = rng.random((80, 3))
    P = recovery_path_general(X, root=5)
    u = rng.random(80) - 0.5
    v, _ = recovery_vector2(u, 1.0, P, 5)
    assert np.allclose(recovery_vector2_prefix(u, P, 5, u[5]), v, atol=1e-12)


def test_randomized_svd_exact_on_low_rank():
    rng = W.rng(23, 0)
    A = rng.standard_normal((200, 5)) @ rng.standard_normal((5, 150))
    R = rng.choice(200, 10, replace=False)
    C = rng.choice(150, 10, replace=False)
    U, s, V = randomized_svd(lambda i: A[i], lambda j: A[:, j], 200, 150, R, C, 5, rng)
    assert np.linalg.norm(U @ np.diag(s) @ V.T - A) / np.linalg.norm(A) < 1e-10


@pytest.mark.parametrize("r", [5, 6])
def test_low_rank_factorization_lemma22_regime(r):
    # Phi = x^T xi on [0,1)^3 x [0,1)^3 (Example 2's phase on lattices): increments
    # along the paths stay below 1/4, so Lemma 2.2 applies and the recovery is exact
    n, d = 8, 3
    pts = np.array(np.unravel_index(np.arange(n ** d), (n,) * d)).T / n
    X1, X2 = pts, pts * 0.9
    Phi = lambda I, J: X1[I] @ X2[J].T
    kr = lambda i: np.exp(2j * np.pi * Phi([i], np.arange(n ** d))[0])
    kc = lambda j: np.exp(2j * np.pi * Phi(np.arange(n ** d), [j])[:, 0])
    q = (0,) * d
    P1 = recovery_path_lattice(d, n, q)
    P2 = recovery_path_lattice(d, n, q)
    U, V, H = low_rank_factorization(kr, kc, n ** d, P1, P2, r, 2, W.rng(23, r))
    assert len(H.Dr) == 1 and len(H.Dc) == 1
    S = W.index_sample(n ** d, 128, 23, 2)
    Kt = np.exp(2j * np.pi * Phi(S, S))
    assert eps_K(Kt, U, V, S) < 1e-12
    # recovered rows and columns agree at every intersection (Lemma 2.2)
    i, j = 17, 301
    assert abs(H.row(i)[j] - H.col(j)[i]) < 1e-12
    # e^{2 pi i Psi} = K on recovered entries
    assert np.allclose(np.exp(2j * np.pi * H.row(i)), kr(i), atol=1e-12)


# ---- branch reconciliation (the extension for integer frequency lattices) ----

from oracle.kernel import Kernel, x_points, xi_points  # noqa: E402
from oracle.phase import (max_block_increment, reconciled_low_rank_factorization,  # noqa: E402
                          sample_order, splitmix64)


def test_splitmix64_published_outputs():
    # the first two outputs of splitmix64 from state 0 (Steele, Lea, Flood 2014; Vigna's reference code)
    z = splitmix64(np.array([0, 0x9E3779B97F4A7C15], dtype=np.uint64))
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4]


def test_sample_order_is_a_seeded_permutation():
    a = sample_order(1000, 7, 0)
    assert sorted(a.tolist()) == list(range(1000))
    assert np.array_equal(a, sample_order(1000, 7, 0))
    assert not np.array_equal(a, sample_order(1000, 7, 1))
    assert not np.array_equal(a, sample_order(1000, 8, 0))


def _iso3d_handles(n):
    K = Kernel(3, n, "iso3d")
    N = K.N
    return K, (lambda i: K.entries([i], np.arange(N))[0]), (lambda j: K.entries(np.arange(N), [j])[:, 0])


def _true_iso3d_phase(n, I, J):
    x, xi = x_points(3, n)[I], xi_points(3, n)[J]
    c = (3 + np.prod(np.sin(2 * np.pi * x), axis=1)) / 100
    return x @ xi.T + c[:, None] * np.linalg.norm(xi, axis=1)[None, :]


def test_literal_recovery_fails_on_integer_lattice():
    """Outside Lemma 2.2 (steps of x.xi up to ~1 along rows) the literal Alg. 7 mixes branches."""
    n = 16
    K, kr, kc = _iso3d_handles(n)
    N = K.N
    P1 = recovery_path_lattice(3, n, (0, 0, 0))
    P2 = recovery_path_lattice(3, n, (n // 2,) * 3)
    U, V, H = low_rank_factorization(kr, kc, N, P1, P2, 8, 2, W.rng(24, 0))
    i, j = int(np.ravel_multi_index((12, 1, 2), (n,) * 3)), 300
    assert abs(H.row(i)[j] - H.col(j)[i]) > 0.5          # intersections disagree by an integer
    S = W.index_sample(N, 128, 24, 1)
    assert eps_K(K.entries(S, S), U, V, S) > 0.1


def test_reconciled_recovery_returns_the_true_phase():
    """Closed form: with both anchors at Phi = 0 (x = 0, xi = 0) and rank(Phi) = 4 <= r, the
    reconciled recovery reproduces Phi = x.xi + c(x)|xi| itself."""
    n = 16
    K, kr, kc = _iso3d_handles(n)
    N = K.N
    P1 = recovery_path_lattice(3, n, (0, 0, 0))
    P2 = recovery_path_lattice(3, n, (n // 2,) * 3)
    U, V, H, info = reconciled_low_rank_factorization(kr, kc, N, P1, P2, xi_points(3, n), 8, 2, 99)
    S = W.index_sample(N, 200, 24, 2)
    T = W.index_sample(N, 200, 24, 3)
    assert np.abs(U[S] @ V[T].T - _true_iso3d_phase(n, S, T)).max() < 1e-9
    assert eps_K(K.entries(S, S), U, V, S) < 1e-12
    # the integer shift of every accepted row undoes the aliasing x_d -> x_d - 1 of x_d > 1/2
    x = x_points(3, n)[info["R"]]
    assert np.array_equal(info["m"], (x > 0.5).astype(np.int64))
    assert (info["a"] == 0).all()
    # accepted rows and columns keep clear of the unwrap limit
    assert not ((x > 0.4) & (x < 0.6)).any()
    xi = xi_points(3, n)[info["C"]]
    assert (np.abs(xi) <= 0.45 * n).all()
    assert len(info["R"]) == len(info["C"]) == 17


def test_reconciled_equals_literal_in_lemma22_regime():
    """Inside Lemma 2.2 no vector is rejected, every shift is zero and both give Psi = Phi."""
    n, d = 8, 3
    pts = np.array(np.unravel_index(np.arange(n ** d), (n,) * d)).T / n
    X1, X2 = pts, pts * 0.9
    Phi = lambda I, J: X1[I] @ X2[J].T
    kr = lambda i: np.exp(2j * np.pi * Phi([i], np.arange(n ** d))[0])
    kc = lambda j: np.exp(2j * np.pi * Phi(np.arange(n ** d), [j])[:, 0])
    P = recovery_path_lattice(d, n, (0,) * d)
    U, V, H, info = reconciled_low_rank_factorization(kr, kc, n ** d, P, P, X2, 5, 2, 3)
    assert (info["m"] == 0).all() and (info["a"] == 0).all()
    order_r = [int(i) for i in sample_order(n ** d, 3, 0)]
    assert info["R"].tolist() == [0] + [i for i in order_r if i != 0][:10]   # D_r = [root], then rq rows
    S = W.index_sample(n ** d, 128, 25, 0)
    assert np.abs(U[S] @ V[S].T - Phi(S, S)).max() < 1e-10


def test_max_block_increment_ignores_cut_edges():
    P = np.array([[0, 1], [1, 2], [2, 3]])
    v = np.array([0.0, 0.1, 0.9, 1.0])
    assert abs(max_block_increment(v, P, np.array([0, 0, 0, 0])) - 0.8) < 1e-15
    assert abs(max_block_increment(v, P, np.array([0, 0, 1, 1])) - 0.1) < 1e-15


# ---- the tau schedule and Partition2 anchoring, pinned by closed forms ------------------------
#
# Phi(x, xi) = x . xi + 0.35 [x1 >= 1/2] + 0.31 [xi2 >= 0.2] on x = a/n and xi = 0.9 (b - n/2)/n
# (n = 32).  Inside each block every path step of Phi is below 0.03, so Lemma 2.2 holds there;
# the two jumps are what the schedule (Sec. 2.3.4) and Partition2 (Alg. 6) must handle:
#   * root column (xi = 0): Phi = 0.35 [x1 >= 1/2].  The comb tree rooted at x = 0 crosses
#     x1 = 1/2 on one edge only (along the a2 = 0 line), so exactly one row node is flagged for
#     every tau <= 0.35: node (n/2, 0), which roots the second row block.
#   * root row (x = 0): Phi = 0.31 [xi2 >= 0.2].  The comb tree rooted at xi = 0 crosses that
#     line once per xi1 column: n = 32 > 16 flags for every tau <= 0.31, none above.  The
#     schedule 1/4 + j/40 therefore stops at j = 3, tau = 0.325.
#   * every block root (s, t) sits where Phi(root_s, root_t) lies in (-1/2, 1/2], so the raw
#     anchors carry no integer offset and every recovered row and column equals Phi itself.

def _two_jump_phase(n):
    N = n * n
    a = np.array(np.unravel_index(np.arange(N), (n, n))).T
    x = a / n
    xi = (a - n // 2) / n * 0.9

    def Phi(I, J):
        I, J = np.atleast_1d(I), np.atleast_1d(J)
        return x[I] @ xi[J].T + 0.35 * (x[I, 0] >= 0.5)[:, None] + 0.31 * (xi[J, 1] >= 0.2)[None, :]
    return Phi, x, xi


def test_tau_schedule_and_block_anchors_closed_form():
    from oracle.phase import recovery_matrix2
    n = 32
    N = n * n
    Phi, x, xi = _two_jump_phase(n)
    kr = lambda i: np.exp(2j * np.pi * Phi([i], np.arange(N))[0])
    kc = lambda j: np.exp(2j * np.pi * Phi(np.arange(N), [j])[:, 0])
    P1 = recovery_path_lattice(2, n, (0, 0))
    P2 = recovery_path_lattice(2, n, (n // 2, n // 2))
    H = recovery_matrix2(kr, kc, N, P1, P2)
    assert abs(H.tau - 0.325) < 1e-12
    assert H.Dr[1:] == [(n // 2) * n] and H.Dc[1:] == []
    assert [r for r, _ in H.blocks_r] == [0, (n // 2) * n] and len(H.blocks_c) == 1
    assert np.array_equal(H.owner_r, (x[:, 0] >= 0.5).astype(np.int64))
    # every recovered row / column is Phi itself (block anchors without offsets)
    for i in W.index_sample(N, 12, 26, 0):
        assert np.abs(H.row(int(i)) - Phi([i], np.arange(N))[0]).max() < 1e-12
    for j in W.index_sample(N, 12, 26, 1):
        assert np.abs(H.col(int(j)) - Phi(np.arange(N), [j])[:, 0]).max() < 1e-12
    # Alg. 7 on top: rank(Phi) = 4 (x . xi, two indicator terms) <= r, so U V^T = Phi
    U, V, _ = low_rank_factorization(kr, kc, N, P1, P2, 8, 2, W.rng(26, 2))
    S = W.index_sample(N, 150, 26, 3)
    assert np.abs(U[S] @ V[S].T - Phi(S, S)).max() < 1e-9
    assert eps_K(np.exp(2j * np.pi * Phi(S, S)), U, V, S) < 1e-12


def test_tau_schedule_runs_out_at_one_half():
    """A phase with no smoothness (iid uniform entries): wrapped path increments are uniform on
    (-1/2, 1/2], so about (N - 1)(1 - 2 tau) of them reach tau -- about 51 > 16 at the last grid
    value below 1/2 (tau = 0.475, N = 32^2) -- and the schedule stops at 1/4 + 10/40 = 1/2."""
    from oracle.phase import recovery_matrix2
    n = 32
    N = n * n
    g = W.rng(27, 0)
    Phi = g.random((N, N))
    kr = lambda i: np.exp(2j * np.pi * Phi[i])
    kc = lambda j: np.exp(2j * np.pi * Phi[:, j])
    P = recovery_path_lattice(2, n, (0, 0))
    H = recovery_matrix2(kr, kc, N, P, P)
    assert abs(H.tau - 0.5) < 1e-12
    # one grid step earlier the root row and column each carry more than 16 increments >= 0.475:
    # by the prefix-sum identity of Alg. 4 the increments are wrap(u(ed) - u(bg)) of the raw phases
    for vec in (Phi[:, 0], Phi[0, :]):
        u = wrapped_phase(np.exp(2j * np.pi * vec))
        w = u[P[:, 1]] - u[P[:, 0]]
        w = w - mround(w)
        assert (np.abs(w) >= 0.475).sum() > 16
    assert len(H.Dr) - 1 <= 16 and len(H.Dc) - 1 <= 16
