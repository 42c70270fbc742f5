"""Error measures of Section 4 (oracle; test infrastructure)."""
from __future__ import annotations

import numpy as np


def rel_l2(approx: np.ndarray, exact: np.ndarray) -> float:
    """||approx - exact||_2 / ||exact||_2 over all entries (Frobenius for blocks)."""
    return float(np.linalg.norm((approx - exact).ravel()) / np.linalg.norm(exact.ravel()))


def eps_b(gb: np.ndarray, gd: np.ndarray) -> float:
    """epsilon^b: relative error of the fast result on the sampled rows (Sec. 4)."""
    return rel_l2(gb, gd)


def eps_K(K_true: np.ndarray, U: np.ndarray, V: np.ndarray, S) -> float:
    """epsilon^K = ||e^{2 pi i Phi(S,S)} - e^{2 pi i U(S,:) V(S,:)^T}||_2 / ||e^{2 pi i Phi(S,S)}||_2."""
    approx = np.exp(2j * np.pi * (U[S] @ V[S].T))
    return float(np.linalg.norm(K_true - approx, 2) / np.linalg.norm(K_true, 2))
