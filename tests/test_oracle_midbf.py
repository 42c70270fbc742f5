"""Pins of the plain CPU MIDBF (CPU only).

The factorization approximates K; its pins are the definition (dense K at
tiny N), the FFT closed form for Phi = x . xi, the adjoint identity, and the
CPQR residual bound of every interpolative decomposition.
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle.kernel import Kernel, direct_sum, fft_linear
from oracle.metrics import rel_l2
from oracle.midbf import MIDBF, Tree, column_id, mock_chebyshev_points

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_morton_numbering_matches_fig4():
    grid = np.loadtxt(os.path.join(GOLD, "morton_fig4.txt"), dtype=int)
    tr = Tree(2, 4, 1)        # 4 x 4 boxes of one point: level 2 of a unit-leaf tree
    for i in range(16):
        origin, side = tr.box(2, i)
        assert side == 1
        assert grid[origin[0], origin[1]] == i


@pytest.mark.parametrize("d,n,leaf", [(2, 32, 8), (3, 16, 4)])
def test_children_partition_parent(d, n, leaf):
    tr = Tree(d, n, leaf)
    for level in range(tr.L):
        for i in range(min(tr.count(level), 9)):
            pts = np.sort(tr.points(level, i))
            kids = np.sort(np.concatenate([tr.points(level + 1, tr.child(i, t)) for t in range(tr.P)]))
            assert np.array_equal(pts, kids)
    assert sorted(np.concatenate([tr.points(tr.L, i) for i in range(tr.count(tr.L))])) == list(range(n ** d))


def test_mock_chebyshev_samples():
    tr = Tree(2, 64, 8)
    s = mock_chebyshev_points(tr, 1, 3, 100)       # 32 x 32 box, 10 nodes per side
    box = set(tr.points(1, 3).tolist())
    assert set(s.tolist()) <= box and len(s) == 100
    origin, side = tr.box(1, 3)
    coords = np.array(np.unravel_index(s, (64, 64))).T
    assert coords.min(axis=0).tolist() == origin.tolist()           # Lobatto nodes reach both ends
    assert (coords.max(axis=0) == origin + side - 1).all()
    assert len(mock_chebyshev_points(tr, 3, 0, 600)) == 64           # small box taken whole


def test_column_id_exact_on_low_rank():
    rng = W.rng(11, 1)
    A = (rng.standard_normal((60, 7)) + 1j * rng.standard_normal((60, 7))) @ \
        (rng.standard_normal((7, 40)) + 1j * rng.standard_normal((7, 40)))
    k, piv, T, diag = column_id(A, 1e-10)
    assert k == 7
    rec = np.zeros_like(A)
    rec[:, piv] = A[:, piv[:k]] @ np.hstack([np.eye(k), T])
    assert rel_l2(rec, A) < 1e-12


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9])
def test_column_id_cpqr_bound(tol):
    K = Kernel(2, 64, "fio_ellipse")
    tr = Tree(2, 64, 8)
    cand = np.concatenate([tr.points(3, 4 * 5 + t) for t in range(4)])
    smp = mock_chebyshev_points(tr, 2, 6, 300)
    X = K.entries(smp, cand)
    k, piv, T, diag = column_id(X, tol)
    rec = np.zeros_like(X)
    rec[:, piv] = X[:, piv[:k]] @ np.hstack([np.eye(k), T])
    err = np.linalg.norm(rec - X)
    n = X.shape[1]
    # ||X - X_skel [I T] Pi^T||_F = ||R22||_F <= sqrt(n-k) |R_{k+1,k+1}| <= sqrt(n-k) tol |R_11|
    assert err <= np.sqrt(n - k) * tol * diag[0] * (1 + 1e-8)
    assert diag[k] <= tol * diag[0] < diag[k - 1]


@pytest.mark.parametrize("phase", ["linear", "fio_ellipse", "fio_piecewise"])
def test_dense_brute_force_tiny(phase):
    # N = 16^2 (L = 1) and 32^2 (L = 2): densified factor product vs K
    for n, bound in ((16, 10 * 1e-6), (32, 10 * 1e-6)):
        K = Kernel(2, n, phase)
        F = MIDBF(K, tol=1e-6)
        assert rel_l2(F.dense(), K.dense()) < bound


def test_full_rank_blocks_are_exact():
    # at N = 32^2 every ID is full rank (k = n0) and the factorization is exact
    K = Kernel(2, 32, "fio_ellipse")
    F = MIDBF(K, tol=1e-6)
    assert all(k == 64 for side in F.rank_table().values() for lev in side for k in lev)
    assert rel_l2(F.dense(), K.dense()) < 1e-13


def test_fft_closed_form_through_factorization():
    K = Kernel(2, 64, "linear")
    F = MIDBF(K, tol=1e-6)
    f = W.complex_gaussian(K.N, 2, 12)
    assert rel_l2(F.apply(f), fft_linear(2, 64, f)) < 1e-5


def test_adjoint_identity_and_fio_accuracy():
    K = Kernel(2, 64, "fio_ellipse")
    F = MIDBF(K, tol=1e-6)
    f = W.complex_gaussian(K.N, 2, 13)
    h = W.complex_gaussian(K.N, 2, 14)
    lhs = np.vdot(h, F.apply(f))
    rhs = np.vdot(F.apply_adjoint(h), f)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13
    rows = W.sample_rows(K.N, 0, 256)
    assert rel_l2(F.apply(f)[rows], direct_sum(K, f, rows=rows)) < 1e-5
    ga = F.apply_adjoint(h)
    from oracle.kernel import direct_sum_adjoint
    assert rel_l2(ga[rows], direct_sum_adjoint(K, h, rows=rows)) < 1e-5


def test_odd_and_even_depth_structure():
    # L = 3 (n = 64): b = 2 steps, h* = 2, k x k middle blocks
    # L = 2 (n = 32): b = 1 step,  h* = 2, (P k) x (P k) middle blocks
    F3 = MIDBF(Kernel(2, 64, "linear"), tol=1e-6)
    assert (F3.L, F3.b, F3.hstar) == (3, 2, 2) and len(F3.mid) == 16 * 16
    F2 = MIDBF(Kernel(2, 32, "linear"), tol=1e-6)
    assert (F2.L, F2.b, F2.hstar) == (2, 1, 2) and len(F2.mid) == 4 * 4
    assert all(S.shape == (256, 256) for S in F2.mid.values())


def test_three_dimensional_lattice():
    K = Kernel(3, 16, "iso3d")
    F = MIDBF(K, tol=1e-6, leaf_box=4)     # n0 = 64, L = 2
    f = W.complex_gaussian(K.N, 1, 15)
    rows = W.sample_rows(K.N, 3, 128)
    assert rel_l2(F.apply(f)[rows], direct_sum(K, f, rows=rows)) < 1e-5


# ---- the fixed-rank variant (Sec. 3.5, closing paragraph) ---------------------

def test_fixed_rank_keeps_the_given_rank_everywhere():
    # every ID keeps min(rank, samples, candidates) columns: n0 = 64 leaf candidates, then 4 * rank
    K = Kernel(2, 64, "fio_ellipse")
    F = MIDBF(K, rank=20)
    for side in F.rank_table().values():
        for lev in side:
            assert set(lev) == {20}
    # the stored T blocks follow from the ranks alone: 4 * 20 candidates, 20 kept, at every ID of step 1;
    # 64 candidates at step 0
    nid = 4 ** (F.L + 1)
    t_entries = 2 * nid * (20 * (64 - 20) + 20 * (80 - 20))
    assert F.entry_count() - sum(S.size for S in F.mid.values()) == t_entries


def test_fixed_rank_full_rank_is_exact():
    # at 32^2 a rank of 64 keeps every leaf point: the factorization reproduces K
    K = Kernel(2, 32, "fio_ellipse")
    F = MIDBF(K, rank=64)
    assert rel_l2(F.dense(), K.dense()) < 1e-13


def test_fixed_rank_error_falls_with_the_rank():
    # 32^2 (one MSCS step, 64 leaf candidates): the error against the direct sum falls with the rank
    K = Kernel(2, 32, "fio_ellipse")
    f = W.complex_gaussian(K.N, 1, 16)
    gd = direct_sum(K, f)
    errs = [rel_l2(MIDBF(K, rank=r).apply(f), gd) for r in (24, 40, 56)]
    assert errs[0] > errs[1] > errs[2] > 0.0
    assert errs[2] < 1e-2


# ---- scattered points (Sec. 3.5, closing paragraph; Example 2 of Sec. 4) -------------------

def test_point_tree_on_the_lattice_is_the_lattice_tree():
    from oracle.kernel import x_points
    from oracle.midbf import PointTree
    lat = Tree(2, 32, 8)
    pt = PointTree(x_points(2, 32), lat.L)
    for level in range(lat.L + 1):
        for i in range(lat.count(level)):
            a, b = np.sort(lat.points(level, i)), np.sort(pt.points(level, i))
            assert np.array_equal(a, b), (level, i)
    for i in range(lat.count(lat.L)):        # leaves list their points by increasing number
        assert np.array_equal(lat.points(lat.L, i), pt.points(lat.L, i))


def test_point_samples_are_node_points():
    from oracle.midbf import PointTree
    x, _ = W.random_points(2, 32, 40)
    pt = PointTree(x, 2)
    for level in (1, 2):
        for i in range(pt.count(level)):
            pts = pt.points(level, i)
            for want in (9, 40, 400):
                s = pt.samples(level, i, want)
                q = int(np.ceil(want ** 0.5 - 1e-9))
                assert len(np.unique(s)) == len(s) and set(s) <= set(pts)
                if len(pts) <= q * q:
                    assert np.array_equal(s, pts)
                else:
                    assert len(s) <= q * q


@pytest.mark.parametrize("half", [False, True])
def test_scattered_points_dense_brute_force(half):
    # 2-D, N = 16^2 random points (half: x only in x_1 < 1/2, so half the nodes are empty); the
    # factor product against K itself
    x, xi = W.random_points(2, 16, 41, half=half)
    K = Kernel(2, 16, "linear", points=(x, xi))
    F = MIDBF(K, tol=1e-6, leaf_box=4)
    assert F.L == 2
    assert rel_l2(F.dense(), K.dense()) < 1e-5


def test_scattered_points_3d_nuft_and_adjoint():
    # Example 2 at N = 16^3: random x in [0,1)^3 and xi in [-8, 8)^3, Phi = x . xi
    x, xi = W.random_points(3, 16, 42)
    K = Kernel(3, 16, "linear", points=(x, xi))
    F = MIDBF(K, tol=1e-6, leaf_box=4)
    f = W.complex_gaussian(K.N, 2, 43)
    rows = W.sample_rows(K.N, 5, 128)
    assert rel_l2(F.apply(f)[rows], direct_sum(K, f, rows=rows)) < 1e-5
    h = W.complex_gaussian(K.N, 2, 44)
    lhs = np.vdot(h, F.apply(f))
    rhs = np.vdot(F.apply_adjoint(h), f)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13


def test_helmholtz_sphere_halves_dense():
    # Example 3 at refinement 3: 321 nodes on each half of the icosphere, Phi = h |x - xi| with
    # h = sqrt(N) / 10; the octree leaves are mostly empty (the points lie on a surface)
    X, O = W.icosphere_halves(3)
    N = len(X)
    K = Kernel(3, 16, ("helmholtz", np.sqrt(N) / 10), points=(X, O))
    F = MIDBF(K, tol=1e-6, leaf_box=4)
    assert F.L == 2
    assert rel_l2(F.dense(), K.dense()) < 1e-5
