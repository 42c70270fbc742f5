"""A factorization of K^H (midbf_params.adjoint), needs an MI355X.

The adjoint build factors the kernel conj(K(x, xi)) with the xi points as rows and the x points as
columns (eq. 1 conjugate-transposed), so its forward apply computes K^H g in every kept precision,
the split 16-bit ones included.  Each apply is compared with the oracle's direct adjoint sum on the
same seeded inputs, and the adjoint apply of such a handle (K^H)^H f = K f with the direct sum.
"""
import numpy as np
import pytest

import workloads as W
from oracle.kernel import Kernel, direct_sum, direct_sum_adjoint
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


def test_adjoint_kernel_entries():
    """The entries of K^H: conj(K(x_q, xi_p)) at (p, q), from the phase negated in FP64."""
    M = _mod()
    N = 32 * 32
    rows = W.index_sample(N, 150, 70)
    cols = W.index_sample(N, 170, 71)
    tr, tc = torch.from_numpy(rows).to(DEV), torch.from_numpy(cols).to(DEV)
    for phase in ("fio_ellipse", "fio_piecewise"):
        KH = M.kernel_entries(2, 32, phase, tr, tc, adjoint=True).cpu().numpy()
        ref = np.conj(Kernel(2, 32, phase).entries(cols, rows)).T
        assert KH.shape == (150, 170)
        assert np.abs(KH - ref).max() < 1e-12
        fwd = M.kernel_entries(2, 32, phase, tc, tr).cpu().numpy()
        assert np.abs(KH - np.conj(fwd).T).max() < 1e-14


@pytest.mark.parametrize("phase", ["fio_ellipse", "fio_piecewise"])
def test_adjoint_build_64(phase):
    M = _mod()
    n = 64
    K = Kernel(2, n, phase)
    print(f"[adj-build] {n}^2 {phase}", flush=True)
    F = M.MIDBF(2, n, phase, adjoint=True, precisions=1 | 2 | 4 | 8)
    g = W.complex_gaussian(K.N, 64, 72)
    fd = direct_sum_adjoint(K, g)
    f64 = from_dev(F.apply(to_dev(g)))
    assert rel_l2(f64, fd) < 1e-5
    f1 = from_dev(F.apply(to_dev(g[:, :1])[0]).unsqueeze(0))          # one right-hand side, VALU path
    assert rel_l2(f1, fd[:, :1]) < 1e-5
    for precision, tol in (("fp32", 1e-5), ("fp16x3", 1e-5), ("bf16x3", 1e-4)):
        f = from_dev(F.apply(to_dev(g, torch.complex64), precision=precision))
        assert rel_l2(f, fd) < tol, precision
    # the adjoint apply of a factorization of K^H is an apply of K
    h = W.complex_gaussian(K.N, 2, 73)
    assert rel_l2(from_dev(F.apply_adjoint(to_dev(h))), direct_sum(K, h)) < 1e-5
    F.close()


def test_adjoint_build_256_split16_sampled():
    """256^2 ellipse FIO at tolerance 1e-6: the split-FP16 apply of the K^H factorization (64
    right-hand sides) against the direct adjoint sum on seeded rows and against the FP64 adjoint
    apply of the forward factorization."""
    M = _mod()
    w = W.WORKLOADS["fio256"]
    K = Kernel(2, w.n, w.phase)
    print("[adj-build] 256^2 ellipse, fp16x3 x 64", flush=True)
    FH = M.MIDBF(2, w.n, w.phase, tol=w.tol, adjoint=True, precisions=1 | 8)
    FH.tune(64, "fp16x3")
    g = W.complex_gaussian(K.N, 64, 74)
    f16 = from_dev(FH.apply(to_dev(g, torch.complex64), precision="fp16x3"))
    rows = W.sample_rows(K.N, w.cfg, 64)
    fd = direct_sum_adjoint(K, g, rows=rows)
    assert rel_l2(f16[rows], fd) < 1e-5
    FH.close()
    F = M.MIDBF(2, w.n, w.phase, tol=w.tol, precisions=1)
    fa = from_dev(F.apply_adjoint(to_dev(g)))
    assert rel_l2(fa[rows], fd) < 1e-5
    assert rel_l2(f16, fa) < 1e-5
    F.close()


def test_adjoint_build_512x64_split16():
    """The metric's size, 512^2 with 64 right-hand sides: the autotuned split-FP16 apply of the K^H
    factorization (even L) against the direct adjoint sum on 64 seeded rows."""
    M = _mod()
    w = W.WORKLOADS["fio512x64"]
    K = Kernel(2, w.n, w.phase)
    print("[adj-build] 512^2 ellipse, fp16x3 x 64", flush=True)
    FH = M.MIDBF(2, w.n, w.phase, tol=w.tol, adjoint=True, precisions=8)
    st = FH.stats()
    print(f"[adj-build] ranks {st['k_min']}..{st['k_max']}", flush=True)
    assert st["L"] == 6
    FH.tune(64, "fp16x3")
    g = W.complex_gaussian(K.N, 64, 80)
    f16 = from_dev(FH.apply(to_dev(g, torch.complex64), precision="fp16x3"))
    rows = W.sample_rows(K.N, w.cfg, 64)
    fd = direct_sum_adjoint(K, g, rows=rows)
    err = rel_l2(f16[rows], fd)
    print(f"[adj-build] 512^2 x 64 fp16x3: rel L2 vs direct adjoint sum {err:.3e}", flush=True)
    assert err < 1e-5
    FH.close()


def test_adjoint_build_3d():
    """3-D lattice, the iso3d phase at 16^3: FP64 and 16-RHS FP32 matrix-core applies of the K^H
    factorization against the direct adjoint sum on seeded rows."""
    M = _mod()
    n = 16
    K = Kernel(3, n, "iso3d")
    F = M.MIDBF(3, n, "iso3d", tol=1e-6, adjoint=True, precisions=1 | 2)
    g = W.complex_gaussian(K.N, 16, 79)
    rows = W.sample_rows(K.N, 3, 64)
    fd = direct_sum_adjoint(K, g, rows=rows)
    assert rel_l2(from_dev(F.apply(to_dev(g)))[rows], fd) < 1e-5
    assert rel_l2(from_dev(F.apply(to_dev(g, torch.complex64), precision="fp32"))[rows], fd) < 1e-5
    F.close()


def test_adjoint_build_lowrank_phase():
    M = _mod()
    n = 32
    N = n * n
    U, V = W.random_lowrank_factors(N, 3, 75)
    F = M.MIDBF(2, n, "lowrank", U=torch.from_numpy(U).to(DEV), V=torch.from_numpy(V).to(DEV),
                adjoint=True, precisions=1 | 2)
    g = W.complex_gaussian(N, 3, 76)
    fd = direct_sum_adjoint(Kernel(2, n, ("lowrank", U, V)), g)
    assert rel_l2(from_dev(F.apply(to_dev(g))), fd) < 1e-5
    F.close()


@pytest.mark.parametrize("half", [False, True])
def test_adjoint_build_points(half):
    """Scattered points: the row tree holds the xi points and the column tree the x points (with
    half, the column tree's nodes are half empty)."""
    M = _mod()
    n, leaf = 32, 4
    x, xi = W.random_points(2, n, 77, half=half)
    K = Kernel(2, n, "linear", points=(x, xi))
    F = M.MIDBF(2, n, "linear", leaf_box=leaf, points=(torch.from_numpy(x).to(DEV), torch.from_numpy(xi).to(DEV)),
                adjoint=True, precisions=1 | 2)
    g = W.complex_gaussian(K.N, 2, 78)
    fd = direct_sum_adjoint(K, g)
    assert rel_l2(from_dev(F.apply(to_dev(g))), fd) < 1e-5
    assert rel_l2(from_dev(F.apply(to_dev(g, torch.complex64), precision="fp32")), fd) < 1e-5
    F.close()


def test_adjoint_build_not_saved(tmp_path):
    M = _mod()
    from paper_1908_09376_amd._lib import MidbfError
    F = M.MIDBF(2, 32, "fio_ellipse", adjoint=True, precisions=1)
    with pytest.raises(MidbfError, match="UNIMPLEMENTED"):
        F.save(str(tmp_path / "adj.midbf"))
    F.close()
