"""The adjoint apply f = K^H g on the matrix cores, FP32 and FP64 (needs an MI355X).

With 16 or more right-hand sides the adjoint runs the matrix-core GEMMs with each factor read
conjugated and transposed.  It must equal the VALU adjoint of one right-hand side at a time (FP64:
to rounding, 1e-12), satisfy the adjoint identity with the forward apply, and match the oracle's
direct adjoint sum (eq. 1 conjugate-transposed) on seeded rows.
"""
import numpy as np
import pytest

import workloads as W
from oracle.kernel import Kernel, direct_sum_adjoint
from oracle.metrics import rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _mod():
    import paper_1908_09376_amd as M
    return M


def to_dev(a: np.ndarray, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(DEV).to(dtype)


def from_dev(t) -> np.ndarray:
    return t.to(torch.complex128).cpu().numpy().T


def _one_at_a_time(F, g, precision):
    """The VALU adjoint (one right-hand side per call)."""
    return np.stack([from_dev(F.apply_adjoint(to_dev(g[:, [j]], g_dtype(precision))[0],
                                              precision=precision).unsqueeze(0))[:, 0]
                     for j in range(g.shape[1])], axis=1)


def g_dtype(precision):
    return torch.complex128 if precision == "fp64" else torch.complex64


@pytest.mark.parametrize("nrhs", [16, 64, 70])
def test_adjoint_mfma_equals_valu_and_oracle(nrhs):
    M = _mod()
    n = 64
    F = M.MIDBF(2, n, "fio_ellipse", precisions=1 | 2)
    g = W.complex_gaussian(n * n, nrhs, 22)
    print(f"[adj-mfma] 64^2 x {nrhs}", flush=True)
    F.profile(True)
    f64 = from_dev(F.apply_adjoint(to_dev(g), precision="fp64"))
    names = [r["name"] for r in F.profile_read()]
    F.profile(False)
    assert any(nm.startswith("adj_up_mfma_fp64") for nm in names), names
    assert any(nm.startswith("adj_middle_mfma_fp64") for nm in names), names
    ref = _one_at_a_time(F, g[:, :8], "fp64")
    assert rel_l2(f64[:, :8], ref) < 1e-12
    f32 = from_dev(F.apply_adjoint(to_dev(g, torch.complex64), precision="fp32"))
    assert rel_l2(f32, f64) < 1e-5
    rows = W.sample_rows(n * n, 0, 64)
    gd = direct_sum_adjoint(Kernel(2, n, "fio_ellipse"), g[:, :4], rows=rows)
    assert rel_l2(f64[rows, :4], gd) < 1e-5
    # adjoint identity with the forward apply, 64 right-hand sides each
    x = W.complex_gaussian(n * n, nrhs, 23)
    kx = from_dev(F.apply(to_dev(x)))
    lhs = np.sum(np.conj(g) * kx)
    rhs = np.sum(np.conj(f64) * x)
    assert abs(lhs - rhs) / abs(lhs) < 1e-12
    F.close()


def test_adjoint_mfma_256_piecewise_16rhs():
    """The 256^2 piecewise workload's backward shape (16 right-hand sides): matrix-core FP64 adjoint
    against the VALU adjoint column by column."""
    M = _mod()
    n = 256
    F = M.MIDBF(2, n, "fio_piecewise", precisions=1 | 2)
    g = W.complex_gaussian(n * n, 16, 4, 100)
    print("[adj-mfma] 256^2 piecewise x 16", flush=True)
    f64 = from_dev(F.apply_adjoint(to_dev(g), precision="fp64"))
    ref = _one_at_a_time(F, g, "fp64")
    err = rel_l2(f64, ref)
    print(f"[adj-mfma] 256^2 x 16 FP64 matrix cores vs VALU: {err:.2e}", flush=True)
    assert err < 1e-12
    f32 = from_dev(F.apply_adjoint(to_dev(g, torch.complex64), precision="fp32"))
    assert rel_l2(f32, f64) < 1e-5
    F.close()
