"""Recovery paths and phase recovery on scattered point sets (Alg. 5, Algs. 6-7; needs an MI355X).

The library computes the Euclidean minimum spanning tree directly (Prim on the device) and orders it
breadth-first on the host; the oracle builds it as the paper does, from the Delaunay triangulation.
The trees are the same, so the paths must be equal as integer arrays.  Phase recovery then follows the
lattice recovery's steps on these paths; with Example 2 in the paper's own reading (x, xi random in
[0, 1)^3, Phi = x . xi) the phase is smooth along the paths, nothing is rejected or shifted, and the
recovered U V^T must match the oracle's and reproduce K.
"""
import numpy as np
import pytest

import workloads as W
from oracle.kernel import Kernel, direct_sum
from oracle.metrics import eps_K, rel_l2
from oracle.phase import reconciled_low_rank_factorization, recovery_path_general

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _mod():
    import paper_1908_09376_amd as M
    return M


@pytest.mark.parametrize("d,N", [(2, 2000), (3, 4096)])
def test_recovery_path_equals_delaunay_mst_bfs(d, N):
    M = _mod()
    pts = W.rng(54, d).random((N, d))
    print(f"[rec-points] path d={d} N={N}", flush=True)
    P = M.recovery_path(pts, root=0)
    Po = recovery_path_general(pts, root=0)
    assert P.shape == Po.shape == (N - 1, 2)
    assert np.array_equal(P, Po)


def _example2_unit(n, key):
    """Example 2 as printed: N = n^3 points x and xi, both uniform in [0, 1)^3."""
    g = W.rng(*key)
    N = n ** 3
    return g.random((N, 3)), g.random((N, 3))


@pytest.mark.parametrize("n", [8, 16])
def test_phase_recover_points_example2(n):
    M = _mod()
    x, xi = _example2_unit(n, (55, n))
    N = len(x)
    K = Kernel(3, n, "linear", points=(x, xi))
    sample = lambda is_row, i: (K.entries([i], np.arange(N))[0] if is_row else K.entries(np.arange(N), [i])[:, 0])
    print(f"[rec-points] Example 2 recovery N = {n}^3", flush=True)
    U, V, info = M.phase_recover(3, n, sample, r=4, q=2, seed=560 + n, points=(x, xi))
    kr = lambda i: K.entries([i], np.arange(N))[0]
    kc = lambda j: K.entries(np.arange(N), [j])[:, 0]
    P1, P2 = recovery_path_general(x, 0), recovery_path_general(xi, 0)
    Uo, Vo, H, oinfo = reconciled_low_rank_factorization(kr, kc, N, P1, P2, xi, 4, 2, 560 + n)
    assert info["tau"] == H.tau
    assert np.array_equal(info["R"], oinfo["R"]) and np.array_equal(info["C"], oinfo["C"])
    assert not info["m"].any() and not info["a"].any()
    assert info["rejected_rows"] == 0 and info["rejected_cols"] == 0
    U, V = U.cpu().numpy(), V.cpu().numpy()
    S = W.index_sample(N, 256, 5, 561)
    T = W.index_sample(N, 256, 5, 562)
    assert np.abs(U[S] @ V[T].T - Uo[S] @ Vo[T].T).max() < 1e-9
    # Psi = Phi + an integer constant (the anchors' branch): exp(2 pi i U V^T) reproduces K
    assert eps_K(K.entries(S, S), U, V, S) < 1e-12


def test_example2_recovered_phase_through_midbf():
    """Example 2 end to end in Scenario 2: rows and columns of K only -> recovered U V^T -> MIDBF on
    the scattered points with the low-rank phase -> the apply against the direct sum of the true K."""
    M = _mod()
    n = 16
    x, xi = _example2_unit(n, (57, n))
    N = len(x)
    K = Kernel(3, n, "linear", points=(x, xi))
    sample = lambda is_row, i: (K.entries([i], np.arange(N))[0] if is_row else K.entries(np.arange(N), [i])[:, 0])
    U, V, _ = M.phase_recover(3, n, sample, r=4, q=2, seed=570, points=(x, xi))
    # the tree boxes take xi mapped from [-n/2, n/2)^3; these xi lie in [0, 1)^3 inside that box
    pts = (torch.from_numpy(x).to(DEV), torch.from_numpy(xi).to(DEV))
    F = M.MIDBF(3, n, "lowrank", leaf_box=4, U=U, V=V, points=pts, precisions=1)
    f = W.complex_gaussian(N, 1, 58)
    rows = W.sample_rows(N, 8, 256)
    g = F.apply(torch.from_numpy(np.ascontiguousarray(f.T)).to(DEV)[0]).cpu().numpy()
    err = rel_l2(g[rows], direct_sum(K, f, rows=rows)[:, 0])
    st = F.stats()
    print(f"[rec-points] Example 2 recovered -> MIDBF N = 16^3: ranks {st['k_min']}..{st['k_max']}, {err:.2e}",
          flush=True)
    assert err < 1e-5
    F.close()


@pytest.mark.parametrize("n", [8, 16])
def test_table4_flag_counts_against_oracle(n):
    """Table 4's quantity: nodes flagged as discontinuities along the root column (N_Dr) and root row
    (N_Dc) of Example 2 at a fixed threshold tau, for tau = 1/4, 1/6, 1/8, 1/10; equal to the oracle's
    counts on the same paths.  At tau = 1/4 nothing is flagged (the paper's choice for this example)."""
    from oracle.phase import RecoveredPhase
    M = _mod()
    x, xi = _example2_unit(n, (59, n))
    N = len(x)
    K = Kernel(3, n, "linear", points=(x, xi))
    sample = lambda is_row, i: (K.entries([i], np.arange(N))[0] if is_row else K.entries(np.arange(N), [i])[:, 0])
    kr = lambda i: K.entries([i], np.arange(N))[0]
    kc = lambda j: K.entries(np.arange(N), [j])[:, 0]
    P1, P2 = recovery_path_general(x, 0), recovery_path_general(xi, 0)
    counts = []
    for tau in (1 / 4, 1 / 6, 1 / 8, 1 / 10):
        _, _, info = M.phase_recover(3, n, sample, r=2, q=2, seed=590, tau=tau, points=(x, xi))
        H = RecoveredPhase(kr, kc, N, P1, 0, P2, 0, tau)
        got = (info["disc_rows_initial"], info["disc_cols_initial"])
        assert got == (len(H.Dr) - 1, len(H.Dc) - 1), (tau, got)
        counts.append(got)
    print(f"[rec-points] Table 4, n = {n}: (N_Dr, N_Dc) at tau = 1/4, 1/6, 1/8, 1/10: {counts}", flush=True)
    assert counts[0] == (0, 0)
