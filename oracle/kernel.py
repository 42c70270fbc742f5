"""Lattices, phases, kernel entries and the direct sum (oracle; test infrastructure).

The transform is g(x) = sum_{xi in Omega} exp(2 pi i Phi(x, xi)) f(xi), x in X
(Section 1, eq. 1), with unit weights.  X is the lattice {0..n-1}^d / n and
Omega the integer lattice {0..n-1}^d - n/2; points are numbered in C order
(last coordinate fastest).
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


def lattice_indices(d: int, n: int) -> np.ndarray:
    """(N, d) integer coordinates of the lattice points in C order."""
    grids = np.meshgrid(*([np.arange(n)] * d), indexing="ij")
    return np.stack([g.ravel() for g in grids], axis=1).astype(np.int64)


def x_points(d: int, n: int) -> np.ndarray:
    """Spatial points x = a / n in [0, 1)^d."""
    return lattice_indices(d, n).astype(np.float64) / n


def xi_points(d: int, n: int) -> np.ndarray:
    """Frequency points xi = b - n/2 (integers)."""
    return (lattice_indices(d, n) - n // 2).astype(np.float64)


# ---- phase functions -------------------------------------------------------
# Example 1 of Section 4 gives the ellipse phase; the other kinds are the
# workloads' piecewise 2-D phase and the 3-D phase.  Each takes x (m, d) and
# xi (p, d) and returns the (m, p) phase matrix in FP64.

def phase_linear(x: np.ndarray, xi: np.ndarray) -> np.ndarray:
    return x @ xi.T


def phase_fio_ellipse(x: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """Phi = x . xi + sqrt(c1(x)^2 xi1^2 + c2(x)^2 xi2^2) (Section 4, Example 1)."""
    s1, s2 = np.sin(TWO_PI * x[:, 0]), np.sin(TWO_PI * x[:, 1])
    k1, k2 = np.cos(TWO_PI * x[:, 0]), np.cos(TWO_PI * x[:, 1])
    c1 = (2.0 + s1 * s2) / 16.0
    c2 = (2.0 + k1 * k2) / 16.0
    rad = (c1[:, None] ** 2) * (xi[None, :, 0] ** 2) + (c2[:, None] ** 2) * (xi[None, :, 1] ** 2)
    return x @ xi.T + np.sqrt(rad)


def phase_fio_piecewise(x: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """Phi = x . xi + c(x)|xi|; c = (2+sin 2pi x1)/16 for x1 < 1/2, else (3+cos 2pi x2)/16."""
    c = np.where(x[:, 0] < 0.5,
                 (2.0 + np.sin(TWO_PI * x[:, 0])) / 16.0,
                 (3.0 + np.cos(TWO_PI * x[:, 1])) / 16.0)
    return x @ xi.T + c[:, None] * np.linalg.norm(xi, axis=1)[None, :]


def phase_iso3d(x: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """Phi = x . xi + c(x)|xi|, c = (3 + sin 2pi x1 sin 2pi x2 sin 2pi x3)/100."""
    c = (3.0 + np.sin(TWO_PI * x[:, 0]) * np.sin(TWO_PI * x[:, 1]) * np.sin(TWO_PI * x[:, 2])) / 100.0
    return x @ xi.T + c[:, None] * np.linalg.norm(xi, axis=1)[None, :]


PHASES = {
    "linear": phase_linear,
    "fio_ellipse": phase_fio_ellipse,
    "fio_piecewise": phase_fio_piecewise,
    "iso3d": phase_iso3d,
}


class Kernel:
    """Entry access K(I, J) = exp(2 pi i Phi(x_I, xi_J)) (Scenario 1, Table 1).

    ``phase`` is a kind name from PHASES, ("lowrank", U, V) for a phase
    given as Phi = U V^T (the output of Alg. 7), or ("helmholtz", h) for
    Phi = h |x - xi| on point sets.  ``points`` = (x, xi) replaces
    the lattices by given point sets (N x d each; Sec. 3.5, closing paragraph:
    non-uniform points), x in [0, 1)^d and xi in [-n/2, n/2)^d.
    """

    def __init__(self, d: int, n: int, phase, points=None):
        self.d, self.n = d, n
        if points is None:
            self.x = x_points(d, n)
            self.xi = xi_points(d, n)
        else:
            self.x = np.asarray(points[0], dtype=np.float64)
            self.xi = np.asarray(points[1], dtype=np.float64)
            if self.x.shape != self.xi.shape or self.x.shape[1] != d:
                raise ValueError("points: two N x d arrays")
        self.points = points is not None
        self.N = len(self.x)
        if isinstance(phase, tuple) and phase[0] == "lowrank":
            U, V = phase[1], phase[2]
            self._phi = lambda I, J: U[I] @ V[J].T
        elif isinstance(phase, tuple) and phase[0] == "helmholtz":
            # Phi = h |x - xi|_2 (Sec. 4, Example 3)
            h = float(phase[1])
            self._phi = lambda I, J: h * np.sqrt(((self.x[I][:, None, :] - self.xi[J][None, :, :]) ** 2).sum(axis=2))
        else:
            f = PHASES[phase]
            self._phi = lambda I, J: f(self.x[I], self.xi[J])

    def phi(self, I, J) -> np.ndarray:
        return self._phi(np.asarray(I), np.asarray(J))

    def entries(self, I, J) -> np.ndarray:
        return np.exp(1j * TWO_PI * self.phi(I, J))

    def dense(self) -> np.ndarray:
        idx = np.arange(self.N)
        return self.entries(idx, idx)


def direct_sum(K: Kernel, f: np.ndarray, rows=None, block: int = 256) -> np.ndarray:
    """g(rows) = sum_xi K(x, xi) f(xi) in FP64 by row blocks (eq. 1).

    Pinned by the FFT closed form for Phi = x . xi and by a brute-force dense
    product at small N.
    """
    f2 = f.reshape(K.N, -1)
    rows = np.arange(K.N) if rows is None else np.asarray(rows)
    cols = np.arange(K.N)
    out = np.empty((len(rows), f2.shape[1]), dtype=np.complex128)
    for s in range(0, len(rows), block):
        r = rows[s:s + block]
        out[s:s + block] = K.entries(r, cols) @ f2
    return out.reshape((len(rows),) + f.shape[1:])


def direct_sum_adjoint(K: Kernel, g: np.ndarray, rows=None, block: int = 256) -> np.ndarray:
    """f(rows) = sum_x conj(K(x, xi)) g(x): the adjoint K^H applied to g."""
    g2 = g.reshape(K.N, -1)
    rows = np.arange(K.N) if rows is None else np.asarray(rows)
    xs = np.arange(K.N)
    out = np.empty((len(rows), g2.shape[1]), dtype=np.complex128)
    for s in range(0, len(rows), block):
        r = rows[s:s + block]
        out[s:s + block] = np.conj(K.entries(xs, r)).T @ g2
    return out.reshape((len(rows),) + g.shape[1:])


def fft_linear(d: int, n: int, f: np.ndarray) -> np.ndarray:
    """Closed form of the transform for Phi = x . xi on the lattices (Section 1).

    g(a) = sum_b exp(2 pi i a.(b - n/2)/n) f(b) = (-1)^{sum a} n^d ifftn(F)(a),
    where F is f reshaped to the lattice.  Computed with numpy.fft.
    """
    f2 = f.reshape((n,) * d + (-1,))
    axes = tuple(range(d))
    G = np.fft.ifftn(f2, axes=axes) * (n ** d)
    a = lattice_indices(d, n).sum(axis=1)
    sign = np.where(a % 2 == 0, 1.0, -1.0) if n % 2 == 0 else np.exp(-1j * np.pi * a)
    return (G.reshape(n ** d, -1) * sign[:, None]).reshape(f.shape)
