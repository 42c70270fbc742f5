"""Plain CPU MIDBF (oracle; test infrastructure).

Follows Section 3 of the paper:
  * Sec. 3.1 -- trees T_X, T_Omega: 2^d-ary, nodes A^l_i numbered along the
    Z-order curve; node i has children P*i + t (Fig. 4: coordinate 1 is the
    more significant bit of each digit).  N = P^L n0.
  * Sec. 3.2 -- linear-scaling interpolative decomposition: sample t*k rows
    on a Mock-Chebyshev grid, pivoted QR K(s,:) Lambda = Q R, rank rule of
    Sec. 3.5, T = R11^{-1} R12, V = [I T] Lambda^*, and the row version U.
  * Sec. 3.3-3.5 -- LRCS, MSCS and recursive MSCS.  The recursion is unrolled
    by levels: at step s (s = 0, 1, ...), every row node A at level L-s is
    paired with every column node B at level s+1 (the blocks of the
    (s+1)-th split), and the row candidates of (A, B) are the skeletons that
    the children of A received against the parent of B at step s-1 (the
    rows of S^{L-s+1} restricted to the block).  The column side is
    symmetric.  The middle factor S is K restricted to the last skeletons.

Readings of the paper taken here: b = ceil(L/2) steps (odd L allowed); the
sample pool of an ID is the paired box's lattice points; rank k = number of
pivots with |R_jj| > tol |R_11|; if the samples limit the rank, the sample
count is doubled and the ID redone.

Pins: tests/test_oracle_midbf.py -- dense brute force at N = 16^2, 32^2
(exact when all IDs are full rank), the FFT closed form for Phi = x . xi
through the factorization, the adjoint identity, and the per-ID CPQR bound.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from .kernel import Kernel


# ---- trees (Sec. 3.1, Fig. 4) ---------------------------------------------

class Tree:
    """Z-ordered 2^d-ary tree over the index lattice {0..n-1}^d."""

    def __init__(self, d: int, n: int, leaf_box: int):
        if n % leaf_box:
            raise ValueError("n must be a multiple of the leaf box")
        L2 = int(round(math.log2(n // leaf_box)))
        if (leaf_box << L2) != n:
            raise ValueError("n / leaf_box must be a power of two")
        self.d, self.n, self.leaf_box, self.L = d, n, leaf_box, L2
        self.P = 1 << d

    def count(self, level: int) -> int:
        return self.P ** level

    def box(self, level: int, idx: int) -> tuple[np.ndarray, int]:
        """(origin (d,), side) of node idx at `level` in lattice index units."""
        side = self.n >> level
        origin = np.zeros(self.d, dtype=np.int64)
        for j in range(level):                     # digit j from the root down
            t = (idx >> (self.d * (level - 1 - j))) & (self.P - 1)
            for q in range(self.d):                # coordinate q: bit d-1-q of the digit
                bit = (t >> (self.d - 1 - q)) & 1
                origin[q] += bit * (self.n >> (j + 1))
        return origin, side

    def points(self, level: int, idx: int) -> np.ndarray:
        """Lattice point numbers (C order) of the box, in local C order."""
        origin, side = self.box(level, idx)
        loc = np.meshgrid(*([np.arange(side)] * self.d), indexing="ij")
        coords = [origin[q] + loc[q].ravel() for q in range(self.d)]
        return np.ravel_multi_index(coords, (self.n,) * self.d)

    def child(self, idx: int, t: int) -> int:
        return self.P * idx + t

    def parent(self, idx: int) -> int:
        return idx // self.P

    def size(self, level: int, idx: int) -> int:
        return (self.n >> level) ** self.d

    def samples(self, level: int, idx: int, count: int) -> np.ndarray:
        return mock_chebyshev_points(self, level, idx, count)


def unit_cube(pts: np.ndarray) -> np.ndarray:
    """A point set moved and scaled uniformly into [0, 1]^d: (p - min) / (largest extent)."""
    p = np.asarray(pts, dtype=np.float64)
    lo = p.min(axis=0)
    s = float((p.max(axis=0) - lo).max())
    return (p - lo) / (s if s > 0 else 1.0)


class PointTree:
    """Z-ordered 2^d-ary tree over a point set in [0, 1)^d (Sec. 3.5, closing paragraph).

    Node i at level l is the box of its Z-order digits, as in the lattice tree (Fig. 4): digit j
    (root first) holds bit l-1-j of every box coordinate, coordinate 1 the most significant bit.
    A node holds the points inside its box, listed leaf by leaf in Z order and by increasing point
    number inside a leaf; an empty node keeps its number and holds no point (its decompositions
    have nothing to compress).
    """

    def __init__(self, pts: np.ndarray, L: int):
        self.pts = np.asarray(pts, dtype=np.float64)
        self.d = self.pts.shape[1]
        self.L, self.P = L, 1 << self.d
        side = 1 << L
        cells = np.clip(np.floor(self.pts * side).astype(np.int64), 0, side - 1)
        leaf = np.zeros(len(self.pts), dtype=np.int64)
        for j in range(L):
            bit = L - 1 - j
            digit = np.zeros(len(self.pts), dtype=np.int64)
            for q in range(self.d):
                digit |= ((cells[:, q] >> bit) & 1) << (self.d - 1 - q)
            leaf = leaf * self.P + digit
        self.leaf_of = leaf
        self.order = np.lexsort((np.arange(len(self.pts)), leaf))
        counts = np.bincount(leaf, minlength=self.P ** L)
        self.start = np.concatenate([[0], np.cumsum(counts)])

    def count(self, level: int) -> int:
        return self.P ** level

    def points(self, level: int, idx: int) -> np.ndarray:
        w = self.P ** (self.L - level)
        return self.order[self.start[idx * w]:self.start[(idx + 1) * w]]

    def size(self, level: int, idx: int) -> int:
        return len(self.points(level, idx))

    def child(self, idx: int, t: int) -> int:
        return self.P * idx + t

    def parent(self, idx: int) -> int:
        return idx // self.P

    def samples(self, level: int, idx: int, count: int) -> np.ndarray:
        """Mock-Chebyshev samples of a node (Sec. 3.2) for scattered points.

        q = ceil(count^(1/d)) Chebyshev-Lobatto nodes per dimension over the bounding box of the
        node's points; for every node of the tensor grid (C order) the nearest point of the node
        (Euclidean; ties go to the larger point number), duplicates removed in first-seen order.
        A node with no more than q^d points is taken whole.
        """
        pts = self.points(level, idx)
        q = 1
        while q ** self.d < count:
            q += 1
        if len(pts) <= q ** self.d:
            return pts
        xyz = self.pts[pts]
        lo, hi = xyz.min(axis=0), xyz.max(axis=0)
        if q == 1:
            nodes = [0.5 * (lo[qd] + hi[qd]) * np.ones(1) for qd in range(self.d)]
        else:
            c = 0.5 * (1.0 - np.cos(np.pi * np.arange(q) / (q - 1)))
            nodes = [lo[qd] + (hi[qd] - lo[qd]) * c for qd in range(self.d)]
        grids = np.meshgrid(*nodes, indexing="ij")
        g = np.stack([gr.ravel() for gr in grids], axis=1)
        d2 = ((g[:, None, :] - xyz[None, :, :]) ** 2).sum(axis=2)         # grid nodes x points
        best = d2.min(axis=1, keepdims=True)
        pick = np.where(d2 == best, pts[None, :], -1).max(axis=1)          # ties: larger point number
        _, first = np.unique(pick, return_index=True)
        return pick[np.sort(first)]


def mock_chebyshev_points(tree: Tree, level: int, idx: int, count: int) -> np.ndarray:
    """About `count` lattice points of a box nearest to a tensor Chebyshev grid.

    Per dimension q = ceil(count^(1/d)) Chebyshev-Lobatto nodes over the box's
    index range, each rounded to the nearest lattice index, duplicates removed
    (Mock-Chebyshev sampling, Sec. 3.2).  A box with no more than q points per
    side is taken whole.
    """
    origin, side = tree.box(level, idx)
    q = 1
    while q ** tree.d < count:
        q += 1
    if q >= side:
        return tree.points(level, idx)
    j = np.arange(q)
    nodes = 0.5 * (side - 1) * (1.0 - np.cos(np.pi * j / (q - 1)))
    loc = np.unique(np.floor(nodes + 0.5).astype(np.int64))
    grids = np.meshgrid(*([loc] * tree.d), indexing="ij")
    coords = [origin[qd] + grids[qd].ravel() for qd in range(tree.d)]
    return np.ravel_multi_index(coords, (tree.n,) * tree.d)


# ---- linear-scaling ID (Sec. 3.2, rank rule of Sec. 3.5) -------------------

class ID:
    """Column ID of a sampled matrix X (m x n): X ~ X[:, skel] [I T] Pi^T."""

    __slots__ = ("k", "piv", "T", "cand", "diag", "m")

    def __init__(self, k, piv, T, cand, diag, m):
        self.k, self.piv, self.T, self.cand, self.diag, self.m = k, piv, T, cand, diag, m

    @property
    def skel(self) -> np.ndarray:
        return self.cand[self.piv[:self.k]]


def column_id(X: np.ndarray, tol: float, kcap: int | None = None, rank: int | None = None):
    """CPQR X[:, piv] = Q R; k = #{j : |R_jj| > tol |R_11|}; T = R11^{-1} R12.

    rank: the fixed-rank form the paper starts from (Sec. 3.5, closing paragraph):
    k = min(rank, m, n) whatever tol says.
    Returns (k, piv, T, |diag R|).  Pinned by the CPQR residual bound
    ||X - X[:,skel][I T]Pi^T||_F = ||R22||_F <= sqrt(n-k) |R_{k+1,k+1}| and
    by the dense brute-force tests.
    """
    m, n = X.shape
    if m == 0 or n == 0:       # an empty node on either side: nothing to compress
        return 0, np.arange(n), np.zeros((0, n), complex), np.zeros(0)
    R, piv = sla.qr(X, mode="r", pivoting=True)
    diag = np.abs(np.diag(R))
    if rank is not None:
        k = min(rank, m, n)
    elif diag.size == 0 or diag[0] == 0.0:
        k = 0
    else:
        small = np.nonzero(diag <= tol * diag[0])[0]
        k = int(small[0]) if small.size else diag.size
    if kcap is not None:
        k = min(k, kcap)
    T = sla.solve_triangular(R[:k, :k], R[:k, k:n]) if k > 0 else np.zeros((0, n), complex)
    return k, piv, T, diag


class MIDBF:
    """Factor K ~ U^L ... U^h S V^h ... V^L and apply it (Sec. 3).

    Storage: rows[s][(A, B)] is the row ID of block (A at level L-s, B at
    level s+1) and cols[s][(B, A)] the column ID of (B at level L-s of
    T_Omega, A at level s+1 of T_X).  mid[...] holds the middle blocks.
    """

    def __init__(self, K: Kernel, tol: float = 1e-6, leaf_box: int = 8, t: int = 5,
                 kcap: int | None = None, rank: int | None = None):
        self.K, self.tol, self.t, self.kcap, self.rank = K, tol, t, kcap, rank
        self.tree = Tree(K.d, K.n, leaf_box)
        if getattr(K, "points", False):
            # scattered points: the lattice tree's box hierarchy over each set's bounding cube
            L = self.tree.L
            self.tree_x = PointTree(unit_cube(K.x), L)
            self.tree_xi = PointTree(unit_cube(K.xi), L)
        else:
            self.tree_x = self.tree_xi = self.tree
        tr = self.tree
        self.L, self.P = tr.L, tr.P
        if self.L < 1:
            raise ValueError("need at least two tree levels (n >= 2 * leaf_box)")
        self.b = (self.L + 1) // 2          # number of MSCS steps
        self.hstar = self.L - self.b + 1    # level of the last row/column IDs
        self.rows: list[dict] = []
        self.cols: list[dict] = []
        self.samples_used: list[int] = []
        khat_r = khat_c = leaf_box ** K.d
        for s in range(self.b):
            r, kr = self._step(s, "row", khat_r)
            c, kc = self._step(s, "col", khat_c)
            self.rows.append(r)
            self.cols.append(c)
            khat_r, khat_c = kr, kc
        self._middle()

    # one unrolled MSCS step for one side
    def _step(self, s: int, side: str, khat: int):
        tr, K = self.tree, self.K
        la, lb = self.L - s, s + 1
        prev = None if s == 0 else (self.rows[s - 1] if side == "row" else self.cols[s - 1])
        # row side: candidates are x points, samples xi points; column side the reverse
        ctree, stree = (self.tree_x, self.tree_xi) if side == "row" else (self.tree_xi, self.tree_x)
        out = {}
        kmax = 0
        for a in range(tr.count(la)):
            if s == 0:
                cand_base = ctree.points(la, a)
            for bb in range(tr.count(lb)):
                if s == 0:
                    cand = cand_base
                else:
                    pb = tr.parent(bb)
                    cand = np.concatenate([prev[(tr.child(a, t), pb)].skel for t in range(self.P)])
                want = self.t * khat
                while True:
                    smp = stree.samples(lb, bb, want)
                    if side == "row":          # rows of K(cand, :) -> CPQR of K(cand, smp)^T
                        X = K.entries(cand, smp).T
                    else:                      # columns of K(:, cand) -> CPQR of K(smp, cand)
                        X = K.entries(smp, cand)
                    k, piv, T, diag = column_id(X, self.tol, self.kcap, self.rank)
                    box_pts = stree.size(lb, bb)
                    if k >= X.shape[0] and X.shape[0] < min(box_pts, len(cand)):
                        want *= 2              # rank limited by the samples: enlarge (Sec. 3.2)
                        continue
                    break
                out[(a, bb)] = ID(k, piv, T, cand, diag, X.shape[0])
                kmax = max(kmax, k)
        return out, kmax

    def _middle(self):
        tr, K = self.tree, self.K
        R, C = self.rows[-1], self.cols[-1]
        self.mid = {}
        nb = tr.count(self.b)
        for a in range(nb):
            for bb in range(nb):
                if self.L % 2 == 1:            # h* = b: k x k blocks
                    rows = R[(a, bb)].skel
                    cols = C[(bb, a)].skel
                else:                          # h* = b+1: (P k) x (P k) blocks
                    rows = np.concatenate([R[(tr.child(a, t), bb)].skel for t in range(self.P)])
                    cols = np.concatenate([C[(tr.child(bb, t), a)].skel for t in range(self.P)])
                self.mid[(a, bb)] = K.entries(rows, cols)

    # ---- apply (product of the factors, right to left) ---------------------
    def apply(self, f: np.ndarray) -> np.ndarray:
        """g ~ K f via V-side levels, the middle, then U-side levels."""
        return self._walk(f, adjoint=False)

    def apply_adjoint(self, g: np.ndarray) -> np.ndarray:
        """f ~ K^H g: conjugate-transposed factors in reverse order."""
        return self._walk(g, adjoint=True)

    def _walk(self, v: np.ndarray, adjoint: bool) -> np.ndarray:
        tr, P = self.tree, self.P
        v2 = v.reshape(self.K.N, -1).astype(np.complex128)
        up = self.rows if adjoint else self.cols      # factors used going up
        down = self.cols if adjoint else self.rows    # factors used going down
        tree_up = self.tree_x if adjoint else self.tree_xi      # candidates of the up side's leaves
        tree_down = self.tree_xi if adjoint else self.tree_x
        # going up: y[(node at L-s, partner at s+1)] = (interp)^op y_cand
        y = None
        for s in range(self.b):
            la, lb = self.L - s, s + 1
            ynew = {}
            for a in range(tr.count(la)):
                for bb in range(tr.count(lb)):
                    idd = up[s][(a, bb)]
                    if s == 0:
                        yc = v2[tree_up.points(la, a)]
                    else:
                        pb = tr.parent(bb)
                        yc = np.concatenate([y[(tr.child(a, t), pb)] for t in range(P)])
                    k, piv, T = idd.k, idd.piv, idd.T
                    # V = [I T]Pi^T (column side); U^H = [I conj(T)]Pi^T (row side, adjoint)
                    Top = np.conj(T) if adjoint else T
                    ynew[(a, bb)] = yc[piv[:k]] + Top @ yc[piv[k:]]
            y = ynew
        # middle: z[(node at h*, partner at b)]
        z = {}
        nb = tr.count(self.b)
        for a in range(nb):
            for bb in range(nb):
                S = self.mid[(a, bb)]
                if self.L % 2 == 1:
                    if adjoint:
                        z[(bb, a)] = np.conj(S).T @ y[(a, bb)]
                    else:
                        z[(a, bb)] = S @ y[(bb, a)]
                else:
                    if adjoint:   # input blocks y[(child(a), bb)], output z[(child(bb), a)]
                        yin = np.concatenate([y[(tr.child(a, t), bb)] for t in range(P)])
                        out = np.conj(S).T @ yin
                        sizes = [self.cols[-1][(tr.child(bb, t), a)].k for t in range(P)]
                        parts = np.split(out, np.cumsum(sizes)[:-1])
                        for t in range(P):
                            z[(tr.child(bb, t), a)] = parts[t]
                    else:
                        yin = np.concatenate([y[(tr.child(bb, t), a)] for t in range(P)])
                        out = S @ yin
                        sizes = [self.rows[-1][(tr.child(a, t), bb)].k for t in range(P)]
                        parts = np.split(out, np.cumsum(sizes)[:-1])
                        for t in range(P):
                            z[(tr.child(a, t), bb)] = parts[t]
        # going down: w = (interp)^op z over the candidates, summed over siblings
        out = np.zeros_like(v2)
        for s in reversed(range(self.b)):
            la, lb = self.L - s, s + 1
            znew = {}
            for a in range(tr.count(la)):
                for bb in range(tr.count(lb)):
                    idd = down[s][(a, bb)]
                    k, piv, T = idd.k, idd.piv, idd.T
                    zz = z[(a, bb)]
                    w = np.zeros((len(idd.cand), zz.shape[1]), dtype=np.complex128)
                    # U = Pi [I; T^T] (row side); V^H = Pi [I; T^H] (column side, adjoint)
                    Top = np.conj(T).T if adjoint else T.T
                    w[piv[:k]] = zz
                    w[piv[k:]] = Top @ zz
                    if s == 0:
                        out[tree_down.points(la, a)] += w
                    else:
                        pb = tr.parent(bb)
                        sizes = [down[s - 1][(tr.child(a, t), pb)].k for t in range(P)]
                        parts = np.split(w, np.cumsum(sizes)[:-1])
                        for t in range(P):
                            key = (tr.child(a, t), pb)
                            znew[key] = znew.get(key, 0) + parts[t]
            z = znew
        return out.reshape(v.shape)

    def dense(self) -> np.ndarray:
        """The N x N matrix of the factor product (apply to identity columns)."""
        return self.apply(np.eye(self.K.N, dtype=np.complex128))

    # ---- diagnostics ------------------------------------------------------
    def rank_table(self):
        return {"rows": [[v.k for v in d.values()] for d in self.rows],
                "cols": [[v.k for v in d.values()] for d in self.cols]}

    def entry_count(self) -> int:
        c = 0
        for side in (self.rows, self.cols):
            for d in side:
                for v in d.values():
                    c += v.T.size
        for S in self.mid.values():
            c += S.size
        return c
