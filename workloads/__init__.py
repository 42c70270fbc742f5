"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the method: it only names the workloads
(lattice sizes, phase kinds, tolerances) and draws seeded random inputs.
Both the CPU oracle and the HIP path receive exactly these arrays.

Workloads follow the shapes of the paper's Example 1 (Section 4, the 2-D
generalized Radon transform) on integer frequency grids, plus a 3-D lattice
and a piecewise-smooth 2-D phase.  Inputs are complex Gaussian with real parts drawn
before imaginary parts from numpy's default_rng seeded by [9376, workload, j].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# phase kinds (the formulas live separately in the oracle and in the HIP library)
LINEAR = "linear"                  # Phi = x . xi
FIO_ELLIPSE = "fio_ellipse"        # Example 1 phase
FIO_PIECEWISE = "fio_piecewise"    # piecewise-smooth c(x)|xi|
ISO3D = "iso3d"                    # 3-D phase x . xi + c(x)|xi|


@dataclass(frozen=True)
class Workload:
    name: str
    d: int
    n: int
    phase: str
    tol: float = 1e-6
    leaf_box: int = 8
    nrhs: int = 1
    cfg: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.n ** self.d


# The five workloads: 64^2 single RHS, 256^2 single RHS, 512^2 with 64 RHS,
# 32^3 through phase recovery with 16 RHS, 256^2 piecewise phase with 16 RHS.
WORKLOADS = {
    "fio64": Workload("fio64", 2, 64, FIO_ELLIPSE, cfg=0, nrhs=1),
    "fio256": Workload("fio256", 2, 256, FIO_ELLIPSE, cfg=1, nrhs=1),
    "fio512x64": Workload("fio512x64", 2, 512, FIO_ELLIPSE, cfg=2, nrhs=64),
    "iso3d32": Workload("iso3d32", 3, 32, ISO3D, cfg=3, nrhs=16),
    "pw256x16": Workload("pw256x16", 2, 256, FIO_PIECEWISE, cfg=4, nrhs=16),
    # Example 2 of Section 4: the 3-D non-uniform Fourier transform on N = 32^3 random points
    # (random_points(3, 32, 5)), Phi = x . xi, 16 right-hand sides
    "nuft3d32": Workload("nuft3d32", 3, 32, LINEAR, leaf_box=4, cfg=5, nrhs=16, extra={"points": True}),
}


def workload_points(w: Workload):
    """The point sets of a scattered-point workload (None for the lattices)."""
    return random_points(w.d, w.n, w.cfg) if w.extra.get("points") else None


def rng(*key: int) -> np.random.Generator:
    """Seeded generator; keys are (9376, workload index, stream index)."""
    return np.random.default_rng([9376, *key])


def complex_gaussian(N: int, nrhs: int, *key: int) -> np.ndarray:
    """N x nrhs complex128, iid N(0,1) real and imaginary parts, real drawn first.

    Column j is drawn from its own stream key (*key, j) so that any subset of
    columns can be regenerated alone.  Returned in Fortran order (column-major),
    which is the layout the C interface takes.
    """
    out = np.empty((N, nrhs), dtype=np.complex128, order="F")
    for j in range(nrhs):
        g = rng(*key, j)
        re = g.standard_normal(N)
        im = g.standard_normal(N)
        out[:, j] = re + 1j * im
    return out


def rhs_for(w: Workload, nrhs: int | None = None) -> np.ndarray:
    return complex_gaussian(w.N, w.nrhs if nrhs is None else nrhs, w.cfg)


def sample_rows(N: int, cfg: int, count: int = 256) -> np.ndarray:
    """The seeded row subset used for the sampled relative error (Section 4)."""
    count = min(count, N)
    return np.sort(rng(cfg, 999).choice(N, count, replace=False))


def batch_sizes(count: int = 32) -> np.ndarray:
    """Lattice sizes n for the uneven batch: N drawn uniformly from {64^2,128^2,256^2}."""
    return rng(2, 1000).choice(np.array([64, 128, 256]), count)


def batch_rhs(j: int, n: int) -> np.ndarray:
    return complex_gaussian(n * n, 1, 2, 1000 + j)


def adjoint_target(N: int, nrhs: int) -> np.ndarray:
    """The y of the least-squares loss ||K f - y||^2 (piecewise workload)."""
    out = np.empty((N, nrhs), dtype=np.complex128, order="F")
    for j in range(nrhs):
        g = rng(4, 100 + j)
        out[:, j] = g.standard_normal(N) + 1j * g.standard_normal(N)
    return out


def random_lowrank_factors(N: int, r: int, *key: int) -> tuple[np.ndarray, np.ndarray]:
    """Real N x r factors with moderate entries (tests of the low-rank phase path)."""
    g = rng(*key)
    return g.standard_normal((N, r)) * 0.5, g.standard_normal((N, r)) * 0.5


def index_sample(N: int, count: int, *key: int) -> np.ndarray:
    """Random distinct indices (without replacement) in [0, N)."""
    return rng(*key).choice(N, min(count, N), replace=False)


def random_points(d: int, n: int, *key: int, half: bool = False) -> tuple[np.ndarray, np.ndarray]:
    """Scattered point sets of Example 2 (Section 4): N = n^d points x uniform in [0, 1)^d and N
    frequencies xi = n (u - 1/2) with u uniform in [0, 1)^d (so xi spans the lattice's frequency box
    [-n/2, n/2)^d).  half: x confined to x_1 < 1/2, leaving half of every level's nodes empty."""
    g = rng(*key)
    N = n ** d
    x = g.random((N, d))
    if half:
        x[:, 0] *= 0.5
    xi = n * (g.random((N, d)) - 0.5)
    return x, xi


def icosphere_halves(refine: int) -> tuple[np.ndarray, np.ndarray]:
    """The point sets of Example 3 (Section 4): the nodes of a triangular mesh of the unit sphere made
    by refining an icosahedron `refine` times (every edge's midpoint becomes a node, projected onto
    the sphere), split into two halves by the sign of a fixed generic direction.  The mesh is
    centrally symmetric, so each half holds (10 * 4^refine + 2) / 2 nodes.  Returns (X, Omega)."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
             (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
             (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(refine):
        mid = {}

        def midpoint(a, b):
            key = (min(a, b), max(a, b))
            if key not in mid:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                mid[key] = len(verts) - 1
            return mid[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    P = np.array(verts)
    side = P @ np.array([0.2113248654, 0.5773502692, 0.7886751346])
    if np.any(side == 0.0):
        raise ValueError("a node lies on the splitting plane")
    return P[side > 0], P[side < 0]
