"""Phase recovery and low-rank phase factorization (oracle; test infrastructure).

Section 2 of the paper, in its order:
  * Alg. 1   randomized SVD from O(1) rows and columns (Sec. 2.1);
  * Alg. 4   RecoveryVector2: unwrap a vector along a recovery path and flag
             discontinuities (Sec. 2.3.2);
  * Alg. 5   RecoveryPath: Delaunay triangulation -> minimum spanning tree ->
             breadth-first order (Sec. 2.3.3, Def. 2.3);
  * Partition2 (Sec. 2.3.4, Fig. 5) and Alg. 6 RecoveryMatrix2;
  * Alg. 7   LowRankFactorization (Sec. 2.3.5).

Readings of the paper taken here: the phase representative is
u = angle(K)/(2 pi) in (-1/2, 1/2]; round is half-away-from-zero; D starts
with the path root; on lattices the recovery path is the dimension-ordered
comb tree (an MST of axis edges, BFS order = Manhattan distance from the
root); rows and columns recovered in Alg. 6 are anchored at the recovered
root column / root row of their block (in-place updates).

An extension for phases on integer frequency lattices, where row steps of
Phi exceed the unwrap limit of Alg. 4, follows at the end of the module:
branch reconciliation of recovered rows against screened columns, with the
samples drawn in splitmix64-seeded orders.

Pins: tests/test_oracle_phase.py -- the Fig. 5 partition example, the
Definition 2.3 properties of the paths, exact unwrapping of smooth vectors,
the loop == prefix-sum identity of Alg. 4, Lemma 2.2's consistency in its
regime, exact recovery of low-rank matrices by Alg. 1, splitmix64's
published outputs, the failure of the literal recovery on the integer
lattice and the reconciled recovery of the closed-form phase there.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def mround(z):
    """round() with halves away from zero (the paper's MATLAB notation)."""
    return np.sign(z) * np.floor(np.abs(z) + 0.5)


def wrapped_phase(Kvals: np.ndarray) -> np.ndarray:
    """u = Im(log K)/(2 pi) = mod(Phi, 1) represented in (-1/2, 1/2]."""
    return np.angle(Kvals) / (2.0 * np.pi)


# ---- Alg. 4 -----------------------------------------------------------------

def recovery_vector2(u: np.ndarray, tau: float, P: np.ndarray, root: int,
                     v0: np.ndarray | None = None):
    """Unwrap u along the recovery path P ((N-1) x 2 rows (pred, node)).

    v(ed) = u(ed) - round(u(ed) - v(bg)); ed is flagged as a discontinuity
    when |v(ed) - v(bg)| >= tau.  ``v0`` supplies already-recovered values
    (Alg. 6 updates in place); by default v starts as u.
    Returns (v, D) with D = [root, flagged nodes...].
    """
    v = np.array(u if v0 is None else v0, dtype=np.float64, copy=True)
    D = [root]
    for bg, ed in P:
        v[ed] = u[ed] - mround(u[ed] - v[bg])
        if abs(v[ed] - v[bg]) >= tau:
            D.append(int(ed))
    return v, D


def recovery_vector2_prefix(u: np.ndarray, P: np.ndarray, root: int, anchor: float) -> np.ndarray:
    """The same recovery written as a rooted-tree prefix sum.

    Because v(bg) = u(bg) (mod 1), the update of Alg. 4 equals
    v(ed) = v(bg) + w(ed) with w(ed) = wrap(u(ed) - u(bg)), wrap(z) = z - round(z):
    every node is its root value plus the sum of wrapped increments on its path.
    """
    w = np.zeros_like(u)
    bg, ed = P[:, 0], P[:, 1]
    w[ed] = (u[ed] - u[bg]) - mround(u[ed] - u[bg])
    v = np.empty_like(u)
    v[root] = anchor
    for b_, e_ in P:                  # depth order: the parent is final before the child
        v[e_] = v[b_] + w[e_]
    return v


# ---- Alg. 5 and the lattice recovery path ------------------------------------

def recovery_path_general(X: np.ndarray, root: int = 0) -> np.ndarray:
    """P = bfsearch(minspantree(delaunayTriangulation(X))) (Alg. 5).

    Edges of the Delaunay triangulation weighted by Euclidean length, a
    minimum spanning tree of that graph, then breadth-first order from root.
    """
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import breadth_first_order, minimum_spanning_tree
    from scipy.spatial import Delaunay

    tri = Delaunay(X)
    edges = set()
    for simplex in tri.simplices:
        for i in range(len(simplex)):
            for j in range(i + 1, len(simplex)):
                a, b = sorted((int(simplex[i]), int(simplex[j])))
                edges.add((a, b))
    e = np.array(sorted(edges))
    w = np.linalg.norm(X[e[:, 0]] - X[e[:, 1]], axis=1)
    G = coo_matrix((w, (e[:, 0], e[:, 1])), shape=(len(X), len(X))).tocsr()
    T = minimum_spanning_tree(G)
    T = T + T.T
    order, pred = breadth_first_order(T, root, directed=False, return_predecessors=True)
    return np.array([[pred[v], v] for v in order[1:]], dtype=np.int64)


def recovery_path_lattice(d: int, n: int, root_coords) -> np.ndarray:
    """Recovery path of a lattice: the dimension-ordered comb tree.

    parent(p) = p - sign(p_j - q_j) e_j with j the last coordinate where p
    differs from the root q; all edges are unit axis edges, so the tree is a
    minimum spanning tree of the (degenerate) Delaunay graph.  Rows are sorted
    by depth (= Manhattan distance to q), ties by node number.
    """
    N = n ** d
    grids = np.meshgrid(*([np.arange(n)] * d), indexing="ij")
    coords = np.stack([g.ravel() for g in grids], axis=1)
    q = np.asarray(root_coords)
    diff = coords - q[None, :]
    depth = np.abs(diff).sum(axis=1)
    nz = diff != 0
    # last differing coordinate
    jlast = np.where(nz.any(axis=1), d - 1 - np.argmax(nz[:, ::-1], axis=1), -1)
    nodes = np.nonzero(jlast >= 0)[0]
    par = coords[nodes].copy()
    jj = jlast[nodes]
    par[np.arange(len(nodes)), jj] -= np.sign(diff[nodes, jj])
    pred = np.ravel_multi_index(tuple(par.T), (n,) * d)
    order = np.lexsort((nodes, depth[nodes]))
    return np.stack([pred[order], nodes[order]], axis=1).astype(np.int64)


def path_root(P: np.ndarray, N: int) -> int:
    missing = np.setdiff1d(np.arange(N), P[:, 1])
    return int(missing[0])


# ---- Partition2 ---------------------------------------------------------------

def partition2(P: np.ndarray, root: int, D) -> list[tuple[int, np.ndarray]]:
    """Cut the tree at the edge into each node of D (other than the root).

    Returns [(subtree root, sub-P), ...] with subtree roots in the order of D;
    each sub-P keeps the row order of P (Fig. 5: P = [1,3;1,4;1,7;3,6;4,2;4,5]
    cut at 4 gives [1,3;1,7;3,6] and [4,2;4,5]).
    """
    cut = set(int(x) for x in D) - {root}
    owner = {root: root}
    for bg, ed in P:                          # depth order: owner(bg) is known
        owner[int(ed)] = int(ed) if int(ed) in cut else owner[int(bg)]
    roots = [root] + [int(x) for x in D if int(x) != root and int(x) in cut]
    seen, ordered = set(), []
    for r in roots:
        if r not in seen:
            seen.add(r)
            ordered.append(r)
    out = []
    for r in ordered:
        rows = [(int(bg), int(ed)) for bg, ed in P if owner[int(ed)] == r and int(ed) != r]
        out.append((r, np.array(rows, dtype=np.int64).reshape(-1, 2)))
    return out


# ---- Alg. 6 -------------------------------------------------------------------

class RecoveredPhase:
    """Function handle for the recovered Psi (Alg. 6 output).

    ``row(i)`` and ``col(j)`` return full recovered rows / columns of Psi,
    each anchored at the recovered root column / root row of its block.
    ``kfun_row(i)`` / ``kfun_col(j)`` give rows / columns of K (Scenario 2).
    """

    def __init__(self, kfun_row, kfun_col, N, P1, r1, P2, r2, tau):
        self.kfun_row, self.kfun_col, self.N = kfun_row, kfun_col, N
        self.P1, self.P2, self.r1, self.r2 = P1, P2, r1, r2
        u_col = wrapped_phase(kfun_col(r2))          # column at the X2 root, along P1
        u_row = wrapped_phase(kfun_row(r1))          # row at the X1 root, along P2
        _, self.Dr = recovery_vector2(u_col, tau, P1, r1)
        _, self.Dc = recovery_vector2(u_row, tau, P2, r2)
        self.blocks_r = partition2(P1, r1, self.Dr)
        self.blocks_c = partition2(P2, r2, self.Dc)
        self.owner_r = self._owner(self.blocks_r, N)
        self.owner_c = self._owner(self.blocks_c, N)
        # recovered root rows / columns of every block (s, t)
        self.root_row = {}      # (s, t) -> row Psi(root_s, :) restricted to block t
        self.root_col = {}      # (s, t) -> column Psi(:, root_t) restricted to block s
        for s, (rs, Ps) in enumerate(self.blocks_r):
            urow = wrapped_phase(kfun_row(rs))
            for t, (rt, Pt) in enumerate(self.blocks_c):
                v, _ = recovery_vector2(urow, 1.0, Pt, rt)     # anchor u(rs, rt)
                self.root_row[(s, t)] = v
        for t, (rt, Pt) in enumerate(self.blocks_c):
            ucol = wrapped_phase(kfun_col(rt))
            for s, (rs, Ps) in enumerate(self.blocks_r):
                v, _ = recovery_vector2(ucol, 1.0, Ps, rs)     # anchor u(rs, rt)
                self.root_col[(s, t)] = v

    @staticmethod
    def _owner(blocks, N):
        own = np.full(N, -1, dtype=np.int64)
        for s, (r, Ps) in enumerate(blocks):
            own[r] = s
            if len(Ps):
                own[Ps[:, 1]] = s
        return own

    def row(self, i: int) -> np.ndarray:
        """Psi(i, :): per column block t, unwrap along P2.B_t from Psi(i, root_t)."""
        s = self.owner_r[i]
        u = wrapped_phase(self.kfun_row(i))
        out = np.empty(self.N)
        for t, (rt, Pt) in enumerate(self.blocks_c):
            v0 = u.copy()
            v0[rt] = self.root_col[(s, t)][i]
            v, _ = recovery_vector2(u, 1.0, Pt, rt, v0=v0)
            members = self.owner_c == t
            out[members] = v[members]
        return out

    def col(self, j: int) -> np.ndarray:
        """Psi(:, j): per row block s, unwrap along P1.B_s from Psi(root_s, j)."""
        t = self.owner_c[j]
        u = wrapped_phase(self.kfun_col(j))
        out = np.empty(self.N)
        for s, (rs, Ps) in enumerate(self.blocks_r):
            v0 = u.copy()
            v0[rs] = self.root_row[(s, t)][j]
            v, _ = recovery_vector2(u, 1.0, Ps, rs, v0=v0)
            members = self.owner_r == s
            out[members] = v[members]
        return out


def recovery_matrix2(kfun_row, kfun_col, N, P1, P2, tau=0.25, dmax=16):
    """Alg. 6 with the tau schedule of Sec. 2.3.4.

    tau starts at 1/4 and grows by 1/40 while more than ``dmax`` discontinuities
    are flagged on the root row or column (no flags are possible at tau = 1/2).
    """
    r1, r2 = path_root(P1, N), path_root(P2, N)
    while True:
        H = RecoveredPhase(kfun_row, kfun_col, N, P1, r1, P2, r2, tau)
        if (len(H.Dr) - 1 <= dmax and len(H.Dc) - 1 <= dmax) or tau >= 0.5:
            H.tau = tau
            return H
        tau += 1.0 / 40.0


# ---- Alg. 1 -------------------------------------------------------------------

def randomized_svd(row, col, m, n, R, C, r, rng):
    """Rank-r A ~ U S V^T from O(1) rows (row(i)) and columns (col(j)) of A.

    Pivoted QR of A(R,:) gives Pi_col, of A(:,C)^T gives Pi_row; Q_col and
    Q_row are orthonormal bases of A(:,Pi_col) and A(Pi_row,:)^T; with
    I = [Pi_row, S_row], J = [Pi_col, S_col] (S random, drawn outside the
    pivots), M = Q_col(I,:)^+ A(I,J) (Q_row^T(:,J))^+ and svd(M) gives the
    factors.  Returns (U, sigma, V) with A ~ U diag(sigma) V^T.
    """
    AR = np.array([row(i) for i in R])                 # |R| x n
    AC = np.array([col(j) for j in C]).T               # m x |C|
    _, _, pc = sla.qr(AR, mode="economic", pivoting=True)
    pi_col = pc[:r]
    _, _, pr = sla.qr(AC.T, mode="economic", pivoting=True)
    pi_row = pr[:r]
    Acols = np.array([col(j) for j in pi_col]).T       # m x r
    Arows = np.array([row(i) for i in pi_row])         # r x n
    Qc, _ = np.linalg.qr(Acols)
    Qr, _ = np.linalg.qr(Arows.T)
    s_row = rng.choice(np.setdiff1d(np.arange(m), pi_row), r, replace=False)
    s_col = rng.choice(np.setdiff1d(np.arange(n), pi_col), r, replace=False)
    I = np.concatenate([pi_row, s_row])
    J = np.concatenate([pi_col, s_col])
    AIJ = np.array([row(i)[J] for i in I])
    M = np.linalg.pinv(Qc[I, :]) @ AIJ @ np.linalg.pinv(Qr.T[:, J])
    UM, sM, VMh = np.linalg.svd(M)
    return Qc @ UM[:, :r], sM[:r], Qr @ VMh.conj().T[:, :r]


# ---- Alg. 7 -------------------------------------------------------------------

def low_rank_factorization(kfun_row, kfun_col, N, P1, P2, r, q, rng, tau=0.25):
    """[U, V] with e^{2 pi i U V^T} ~ K from O(1) rows and columns of K.

    R, C = randperm(N, r q); Psi = RecoveryMatrix2; rSVD(Psi, R, C, r);
    V <- V Sigma.  Returns (U, V, H) with H the recovered-phase handle.
    """
    R = rng.choice(N, r * q, replace=False)
    C = rng.choice(N, r * q, replace=False)
    H = recovery_matrix2(kfun_row, kfun_col, N, P1, P2, tau=tau)
    Rext = np.unique(np.concatenate([R, np.asarray(H.Dr, dtype=np.int64)]))
    Cext = np.unique(np.concatenate([C, np.asarray(H.Dc, dtype=np.int64)]))
    U, sig, V = randomized_svd(H.row, H.col, N, N, Rext, Cext, r, rng)
    return U, V * sig[None, :], H


# ---- Extension: branch reconciliation (outside Lemma 2.2) ---------------------
#
# On an integer frequency lattice a row of K samples exp(2 pi i Phi(x, .)) at
# integer steps, so a step of Phi larger than 1/2 along the row is unwrapped to
# Phi - m.xi (m integer) or, near the half-integer boundary, to a mix of
# branches; columns (steps of size xi/n) stay inside the unwrap limit except
# next to the Nyquist frequency.  Rows and columns recovered by Alg. 6 then
# disagree at their intersections by integers and Alg. 1 mixes two matrices.
# The extension keeps Alg. 7's order of steps and changes three things:
#   1. a recovered vector is used only when every path increment inside its
#      block is below tau_amb in magnitude (no step near the unwrap limit);
#   2. each accepted row is fitted, over the accepted sampled columns, by
#      Psi_col(i, j) - Psi_row(i, j) = m . xi_j + a with integer m and a, and
#      accepted only when the fit is exact; the row is then shifted by m . xi + a;
#   3. Alg. 1's pivots and extra rows / columns are taken inside the accepted
#      samples (every vector it uses has passed 1 and 2).
# In the Lemma 2.2 regime nothing is rejected and every m, a is zero.

def splitmix64(z: np.ndarray) -> np.ndarray:
    """The splitmix64 output function (Steele, Lea, Flood 2014) on uint64 counters."""
    z = (z + np.uint64(0x9E3779B97F4A7C15)).astype(np.uint64)
    z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)).astype(np.uint64)
    z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)).astype(np.uint64)
    return z ^ (z >> np.uint64(31))


def sample_order(N: int, seed: int, stream: int) -> np.ndarray:
    """A seeded random order of 0..N-1: indices sorted by splitmix64(seed + 2 i + stream)
    (ties, which need a 64-bit collision, by index).  stream 0: rows, 1: columns."""
    with np.errstate(over="ignore"):
        ctr = (np.uint64(seed) + np.uint64(2) * np.arange(N, dtype=np.uint64) + np.uint64(stream))
        h = splitmix64(ctr)
    return np.lexsort((np.arange(N), h)).astype(np.int64)


def max_block_increment(v: np.ndarray, P: np.ndarray, owner: np.ndarray) -> float:
    """max |v(ed) - v(bg)| over the path edges whose ends lie in one block."""
    bg, ed = P[:, 0], P[:, 1]
    same = owner[bg] == owner[ed]
    if not same.any():
        return 0.0
    return float(np.abs(v[ed[same]] - v[bg[same]]).max())


def reconciled_low_rank_factorization(kfun_row, kfun_col, N, P1, P2, xi, r, q, seed, tau=0.25,
                                      tau_amb=0.4, fit_tol=1e-6):
    """Alg. 7 with branch reconciliation (the extension above).

    xi: (N, d) coordinates of the column points.  Samples are drawn in the
    seeded orders of sample_order (discontinuity nodes first).  Returns
    (U, V, H, info) with info holding the accepted rows R, columns C and the
    integer shifts m (|R| x d) and a (|R|).
    """
    H = recovery_matrix2(kfun_row, kfun_col, N, P1, P2, tau=tau)
    want = r * q
    # columns: accepted when no path step comes near the unwrap limit
    cand_c = list(H.Dc) + [int(j) for j in sample_order(N, seed, 1) if int(j) not in set(H.Dc)]
    C, cols = [], []
    for j in cand_c:
        v = H.col(j)
        if max_block_increment(v, P1, H.owner_r) < tau_amb:
            C.append(j)
            cols.append(v)
            if len(C) == want + len(H.Dc):
                break
    C = np.array(C, dtype=np.int64)
    AC = np.array(cols).T                                   # N x |C|
    Xc = np.c_[xi[C], np.ones(len(C))]
    Xall = np.c_[xi, np.ones(N)]
    cand_r = list(H.Dr) + [int(i) for i in sample_order(N, seed, 0) if int(i) not in set(H.Dr)]
    R, rows, shifts = [], [], []
    for i in cand_r:
        v = H.row(i)
        if max_block_increment(v, P2, H.owner_c) >= tau_amb:
            continue
        D = AC[i, :] - v[C]                                 # integers up to rounding
        coef = mround(np.linalg.lstsq(Xc, D, rcond=None)[0])
        if np.abs(D - Xc @ coef).max() > fit_tol:
            continue
        R.append(i)
        rows.append(v + Xall @ coef)
        shifts.append(coef)
        if len(R) == want + len(H.Dr):
            break
    R = np.array(R, dtype=np.int64)
    AR = np.array(rows)                                     # |R| x N
    # Alg. 1 with pivots inside the accepted samples
    A_RC = AR[:, C]
    _, _, pc = sla.qr(A_RC, mode="economic", pivoting=True)
    _, _, pr = sla.qr(A_RC.T, mode="economic", pivoting=True)
    kc, kr_ = pc[:r], pr[:r]
    Qc, _ = np.linalg.qr(AC[:, kc])
    Qr, _ = np.linalg.qr(AR[kr_, :].T)
    rest_r = [t for t in range(len(R)) if t not in set(kr_.tolist())][:r]
    rest_c = [t for t in range(len(C)) if t not in set(kc.tolist())][:r]
    It = np.concatenate([kr_, rest_r]).astype(np.int64)     # positions in R
    Jt = np.concatenate([kc, rest_c]).astype(np.int64)      # positions in C
    I, J = R[It], C[Jt]
    AIJ = AR[It][:, J]
    M = np.linalg.pinv(Qc[I, :]) @ AIJ @ np.linalg.pinv(Qr.T[:, J])
    UM, sM, VMh = np.linalg.svd(M)
    U = Qc @ UM[:, :r]
    V = (Qr @ VMh.conj().T[:, :r]) * sM[None, :r]
    shifts = np.array(shifts)
    info = {"R": R, "C": C, "m": shifts[:, :-1].astype(np.int64), "a": shifts[:, -1].astype(np.int64)}
    return U, V, H, info
