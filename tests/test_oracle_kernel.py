"""Pins of the oracle's kernel entries and direct sum (CPU only)."""
import numpy as np
import pytest

import workloads as W
from oracle.kernel import (Kernel, direct_sum, direct_sum_adjoint, fft_linear,
                           phase_fio_ellipse, phase_fio_piecewise, phase_iso3d,
                           x_points, xi_points)
from oracle.metrics import rel_l2


def test_lattice_conventions():
    # C order, last coordinate fastest; x = a/n, xi = b - n/2
    x = x_points(2, 4)
    xi = xi_points(2, 4)
    assert x.shape == (16, 2)
    assert np.allclose(x[1], [0.0, 0.25]) and np.allclose(x[4], [0.25, 0.0])
    assert np.allclose(xi[0], [-2, -2]) and np.allclose(xi[15], [1, 1])


def test_fio_ellipse_hand_values():
    # Example 1 of Section 4, values worked by hand:
    # x=0: c1 = 1/8, c2 = 3/16; x=(1/4,1/4): c1 = 3/16, c2 = 1/8; x=(1/2,0): c1 = 1/8, c2 = 1/16
    x = np.array([[0.0, 0.0], [0.25, 0.25], [0.5, 0.0]])
    xi = np.array([[8.0, 0.0], [0.0, 16.0], [8.0, 16.0], [16.0, 8.0], [-8.0, 16.0]])
    P = phase_fio_ellipse(x, xi)
    assert P[0, 0] == pytest.approx(1.0, abs=1e-14)
    assert P[0, 1] == pytest.approx(3.0, abs=1e-14)
    assert P[0, 2] == pytest.approx(np.sqrt(10.0), abs=1e-14)
    assert P[1, 3] == pytest.approx(6.0 + np.sqrt(10.0), abs=1e-13)
    assert P[2, 4] == pytest.approx(-4.0 + np.sqrt(2.0), abs=1e-13)


def test_piecewise_and_3d_hand_values():
    x = np.array([[0.25, 0.3], [0.75, 0.5]])
    xi = np.array([[3.0, 4.0]])
    P = phase_fio_piecewise(x, xi)
    assert P[0, 0] == pytest.approx(0.75 + 1.2 + 15.0 / 16.0, abs=1e-13)
    assert P[1, 0] == pytest.approx(2.25 + 2.0 + 10.0 / 16.0, abs=1e-13)
    P3 = phase_iso3d(np.array([[0.25, 0.25, 0.25]]), np.array([[2.0, 3.0, 6.0]]))
    assert P3[0, 0] == pytest.approx(2.75 + 0.28, abs=1e-13)


@pytest.mark.parametrize("d,n", [(2, 16), (2, 32), (3, 8)])
def test_direct_sum_matches_fft_closed_form(d, n):
    # Phi = x . xi on the lattices is a discrete Fourier transform (Section 1)
    K = Kernel(d, n, "linear")
    f = W.complex_gaussian(K.N, 3, 77, d, n)
    g = direct_sum(K, f)
    assert rel_l2(g, fft_linear(d, n, f)) < 1e-12


def test_direct_sum_rows_and_blocks():
    K = Kernel(2, 16, "fio_ellipse")
    f = W.complex_gaussian(K.N, 2, 78)
    full = direct_sum(K, f, block=7)
    rows = W.sample_rows(K.N, 0, 40)
    assert np.allclose(direct_sum(K, f, rows=rows), full[rows], rtol=0, atol=1e-12)
    # a single entry of K times a unit vector picks one column
    e = np.zeros((K.N, 1), complex)
    e[5] = 1.0
    col = direct_sum(K, e)
    assert abs(col[3, 0] - np.exp(2j * np.pi * K.phi([3], [5])[0, 0])) < 1e-14


@pytest.mark.parametrize("phase", ["fio_ellipse", "fio_piecewise"])
def test_direct_adjoint_identity(phase):
    K = Kernel(2, 16, phase)
    f = W.complex_gaussian(K.N, 2, 79)
    h = W.complex_gaussian(K.N, 2, 80)
    lhs = np.vdot(h, direct_sum(K, f))
    rhs = np.vdot(direct_sum_adjoint(K, h), f)
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


def test_lowrank_branch_orientation():
    """Kernel(("lowrank", U, V)) evaluates Phi = U(I,:) V(J,:)^T: with U = [x, c(x)] and
    V = [xi, |xi|] it is the 3-D phase x . xi + c(x)|xi| (pinned by hand values above), and
    with U = x, V = xi the linear phase whose direct sum is the FFT."""
    n = 8
    x, xi = x_points(3, n), xi_points(3, n)
    c = (3.0 + np.prod(np.sin(2 * np.pi * x), axis=1)) / 100.0
    U = np.c_[x, c]
    V = np.c_[xi, np.linalg.norm(xi, axis=1)]
    I = W.index_sample(n ** 3, 50, 81, 0)
    J = W.index_sample(n ** 3, 60, 81, 1)
    low = Kernel(3, n, ("lowrank", U, V))
    assert np.abs(low.phi(I, J) - Kernel(3, n, "iso3d").phi(I, J)).max() < 1e-13
    assert low.phi(I, J).shape == (50, 60)
    lin = Kernel(2, 16, ("lowrank", x_points(2, 16), xi_points(2, 16)))
    f = W.complex_gaussian(256, 2, 81, 2)
    assert rel_l2(direct_sum(lin, f), fft_linear(2, 16, f)) < 1e-12
