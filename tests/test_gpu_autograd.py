"""Differentiation through the MIDBF apply (needs an MI355X).

loss = ||K f - y||^2 with forward = midbf_apply and backward =
midbf_apply_adjoint; checked against central finite differences (h = 1e-6,
FP64) and the dense K^H gradient 2 K^H (K f - y) at N = 32^2, and at the
256^2 piecewise-phase workload with 16 right-hand sides.
"""
import numpy as np
import pytest

import workloads as W
from oracle.kernel import Kernel, direct_sum, direct_sum_adjoint
from oracle.metrics import rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(DEV)


def test_gradient_matches_dense_and_finite_differences_32():
    import paper_1908_09376_amd as M
    n, nrhs = 32, 3
    F = M.MIDBF(2, n, "fio_piecewise")
    K = Kernel(2, n, "fio_piecewise")
    f0 = W.complex_gaussian(n * n, nrhs, 4, 7)
    y = W.adjoint_target(n * n, nrhs)
    f = _dev(f0).requires_grad_(True)
    yd = _dev(y)
    loss = (M.midbf_matvec(f, F) - yd).abs().pow(2).sum()
    loss.backward()
    grad = f.grad.cpu().numpy().T
    Kd = K.dense()
    dense = 2.0 * np.conj(Kd).T @ (Kd @ f0 - y)
    assert rel_l2(grad, dense) < 1e-5             # the dense K^H gradient, within the apply error

    def L(fv):
        with torch.no_grad():
            return float((M.midbf_matvec(_dev(fv), F) - yd).abs().pow(2).sum())
    h = 1e-6
    for (p, r) in [(5, 0), (700, 1), (1023, 2)]:
        for unit, part in ((1.0, "re"), (1j, "im")):
            e = np.zeros_like(f0)
            e[p, r] = unit * h
            fd = (L(f0 + e) - L(f0 - e)) / (2 * h)
            an = grad[p, r].real if part == "re" else grad[p, r].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (p, r, part, fd, an)


def test_gradient_piecewise_256_16rhs():
    import paper_1908_09376_amd as M
    w = W.WORKLOADS["pw256x16"]
    F = M.MIDBF(2, w.n, w.phase, tol=w.tol)
    f0 = W.rhs_for(w)
    y = W.adjoint_target(w.N, w.nrhs)
    f = _dev(f0).requires_grad_(True)
    yd = _dev(y)
    g = M.midbf_matvec(f, F)
    loss = (g - yd).abs().pow(2).sum()
    loss.backward()
    grad = f.grad.cpu().numpy().T
    # the same quantity assembled from explicit applies
    r = (g.detach() - yd)
    ref = 2.0 * F.apply_adjoint(r.contiguous()).cpu().numpy().T
    assert rel_l2(grad, ref) < 1e-13
    # against the definition on sampled rows: 2 K^H (K f - y) with the direct sums
    K = Kernel(2, w.n, w.phase)
    rows = W.sample_rows(w.N, w.cfg, 64)
    Kf = g.detach().cpu().numpy().T                     # the MIDBF residual enters both sides
    exact = 2.0 * direct_sum_adjoint(K, Kf - y, rows=rows)
    assert rel_l2(grad[rows], exact) < 1e-5
    # the forward itself vs the direct sum
    assert rel_l2(Kf[rows[:32]], direct_sum(K, f0, rows=rows[:32])) < 1e-5


def test_gradient_through_a_factorization_of_the_adjoint():
    """The backward through a factorization of K^H (adjoint=True) in split FP16, 256^2 x 64 piecewise
    phase: the gradient 2 K^H (K f - y) against the direct adjoint sum of the same residual on seeded
    rows, and against the FP64 backward of the forward factors."""
    import paper_1908_09376_amd as M
    w = W.WORKLOADS["pw256x16"]
    F = M.MIDBF(2, w.n, w.phase, tol=w.tol, precisions=1 | 8)
    FH = M.MIDBF(2, w.n, w.phase, tol=w.tol, precisions=8, adjoint=True)
    F.tune(64, "fp16x3")
    FH.tune(64, "fp16x3")
    f0 = W.complex_gaussian(w.N, 64, 81)
    y = W.complex_gaussian(w.N, 64, 82)
    f = _dev(f0).to(torch.complex64).requires_grad_(True)
    yd = _dev(y).to(torch.complex64)
    g = M.midbf_matvec(f, F, "fp16x3", adjoint_factor=FH)
    (g - yd).abs().pow(2).sum().backward()
    grad = f.grad.to(torch.complex128).cpu().numpy().T
    r = g.detach().to(torch.complex128).cpu().numpy().T - y
    rows = W.sample_rows(w.N, w.cfg, 64)
    exact = 2.0 * direct_sum_adjoint(Kernel(2, w.n, w.phase), r, rows=rows)
    assert rel_l2(grad[rows], exact) < 1e-5
    ref = 2.0 * F.apply_adjoint(_dev(r)).cpu().numpy().T
    assert rel_l2(grad, ref) < 1e-5
    with pytest.raises(ValueError):
        M.midbf_matvec(f, F, "fp16x3", adjoint_factor=F)
    FH.close()
    F.close()
