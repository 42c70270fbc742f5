"""3-D transforms built directly on the phase (Scenario 1), against the oracle (needs an MI355X)."""
import numpy as np
import pytest

import workloads as W
from oracle.kernel import Kernel, direct_sum

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [16, 32])
def test_iso3d_apply_and_adjoint(n):
    import paper_1908_09376_amd as M
    d = 3
    K = Kernel(d, n, "iso3d")
    N = K.N
    F = M.MIDBF(d, n, "iso3d", tol=1e-6, precisions=1 | 2)
    f = W.complex_gaussian(N, 2, 60, n)
    rows = W.sample_rows(N, 3, 64)
    ref = direct_sum(K, f, rows=rows)
    fd = torch.from_numpy(np.ascontiguousarray(f.T)).to("cuda:0")
    g = F.apply(fd, precision="fp64").cpu().numpy().T
    assert np.linalg.norm(g[rows] - ref) / np.linalg.norm(ref) < 1e-6
    g32 = F.apply(fd.to(torch.complex64), precision="fp32").to(torch.complex128).cpu().numpy().T
    assert np.linalg.norm(g32[rows] - ref) / np.linalg.norm(ref) < 1e-5
    # adjoint identity <K f, h> = <f, K^H h> through the transposed butterfly
    h = torch.from_numpy(np.ascontiguousarray(W.complex_gaussian(N, 2, 61, n).T)).to("cuda:0")
    ga = F.apply_adjoint(h, precision="fp64")
    lhs = torch.vdot(F.apply(fd, precision="fp64").reshape(-1), h.reshape(-1))
    rhs = torch.vdot(fd.reshape(-1), ga.reshape(-1))
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


def test_iso3d32_many_rhs_matrix_cores():
    """16 RHS at 32^3: the middle blocks are ~4064^2 (full-rank leaves), split over workgroups."""
    import paper_1908_09376_amd as M
    n, d = 32, 3
    K = Kernel(d, n, "iso3d")
    F = M.MIDBF(d, n, "iso3d", tol=1e-6, precisions=1 | 2)
    f = W.complex_gaussian(K.N, 16, 62)
    rows = W.sample_rows(K.N, 3, 32)
    ref = direct_sum(K, f, rows=rows)
    fd = torch.from_numpy(np.ascontiguousarray(f.T)).to("cuda:0").to(torch.complex64)
    g = F.apply(fd, precision="fp32").to(torch.complex128).cpu().numpy().T
    assert np.linalg.norm(g[rows] - ref) / np.linalg.norm(ref) < 1e-5
    prof = None
    F.profile(True, by_level=True)
    F.apply(fd, precision="fp32")
    prof = {r["name"]: r for r in F.profile_read()}
    F.profile(False)
    assert "middle_mfma_fp32" in prof
