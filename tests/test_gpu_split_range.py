"""Split 16-bit applies across input scales, and at the 512^2 x 64 workload (needs an MI355X).

fp16 holds |x| < 65504 and keeps full precision in the lo part only above its
normal range, so the library holds every split vector scaled by a power of two
per right-hand side (exact in both directions).  These tests feed inputs whose
columns span 1e-4 .. 1e4, coherent inputs (a constant, plane waves, a point
source) whose partial sums grow linearly instead of like a square root, and
check every column against the FP64 apply and the oracle's direct sum (eq. 1).
The last test runs the metric's own configuration, 512^2 with 64 right-hand
sides on the autotuned kernels, against the direct sum on the seeded rows.
"""
import numpy as np
import pytest

import workloads as W
from oracle.kernel import Kernel, direct_sum, fft_linear
from oracle.metrics import rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
KEEP_ALL = 1 | 2 | 4 | 8


def _mod():
    import paper_1908_09376_amd as M
    return M


def to_dev(a: np.ndarray, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(DEV).to(dtype)


def from_dev(t) -> np.ndarray:
    return t.to(torch.complex128).cpu().numpy().T


def col_err(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Relative L2 error of every column."""
    return np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)


@pytest.fixture(scope="module")
def fio128():
    M = _mod()
    F = M.MIDBF(2, 128, "fio_ellipse", tol=1e-6, precisions=KEEP_ALL)
    for p in ("fp16x3", "bf16x3"):
        F.tune(64, p)
    # the interpolation coefficients packed into the 16-bit tiles stay far inside fp16's range
    t = F.stats()["t_abs_max"]
    print(f"[split-range] 128^2 largest |T| entry {t:.3f}", flush=True)
    assert 0.0 < t < 64.0
    return F


def _split_vs_fp64(F, f, precision):
    g = from_dev(F.apply(to_dev(f, torch.complex64), precision=precision))
    g64 = from_dev(F.apply(to_dev(f)))
    assert np.isfinite(g).all(), precision
    return g, g64


@pytest.mark.parametrize("scale", [1e-4, 1e4, 1e-20, 1e20])
def test_fp16x3_uniform_input_scale(fio128, scale):
    f = W.complex_gaussian(128 * 128, 64, 71) * scale
    print(f"[split-range] 128^2 x 64 fp16x3, f scaled by {scale:g}", flush=True)
    g, g64 = _split_vs_fp64(fio128, f, "fp16x3")
    assert col_err(g, g64).max() < 5e-6
    K = Kernel(2, 128, "fio_ellipse")
    rows = W.sample_rows(K.N, 0, 64)
    assert col_err(g[rows], direct_sum(K, f, rows=rows)).max() < 1e-5


@pytest.mark.parametrize("precision,tol", [("fp16x3", 5e-6), ("bf16x3", 1e-4)])
def test_split_mixed_column_scales(fio128, precision, tol):
    """Columns from 1e-4 to 1e4 in one block: each column keeps its own accuracy."""
    scales = np.logspace(-4, 4, 64)
    f = W.complex_gaussian(128 * 128, 64, 72) * scales[None, :]
    print(f"[split-range] 128^2 x 64 {precision}, column scales 1e-4 .. 1e4", flush=True)
    g, g64 = _split_vs_fp64(fio128, f, precision)
    assert col_err(g, g64).max() < tol
    K = Kernel(2, 128, "fio_ellipse")
    rows = W.sample_rows(K.N, 0, 64)
    assert col_err(g[rows], direct_sum(K, f, rows=rows)).max() < (1e-5 if precision == "fp16x3" else 1e-3)


def _coherent_inputs(n: int) -> np.ndarray:
    """Columns whose partial sums add up coherently: a constant, plane waves exp(-2 pi i x0 . xi)
    for a few lattice points x0 (for Phi = x . xi these focus all of |f| on one output point),
    a point source, and the same at amplitudes 1e3 and 1e-3."""
    N = n * n
    xi = np.stack(np.meshgrid(np.arange(n) - n // 2, np.arange(n) - n // 2, indexing="ij"), -1).reshape(N, 2)
    cols = [np.ones(N, dtype=np.complex128)]
    for a in ((0, 0), (5, 77), (n // 2, n // 2), (n - 1, 3)):
        x0 = np.array(a) / n
        cols.append(np.exp(-2j * np.pi * (xi @ x0)))
    e = np.zeros(N, dtype=np.complex128)
    e[N // 3] = 1.0
    cols.append(e)
    base = np.stack(cols, 1)
    return np.concatenate([base, base * 1e3, base * 1e-3], axis=1)


@pytest.mark.parametrize("precision,tol", [("fp16x3", 5e-6), ("bf16x3", 1e-4)])
def test_split_coherent_inputs_linear_phase(precision, tol):
    """Phi = x . xi with a constant or plane-wave input puts the whole sum, N |f|, on one output point
    and every partial sum on the way there is as large as it can be."""
    M = _mod()
    n = 128
    F = M.MIDBF(2, n, "linear", tol=1e-6, precisions=KEEP_ALL)
    f = _coherent_inputs(n)
    F.tune(f.shape[1], precision)
    print(f"[split-range] 128^2 linear, coherent inputs, {precision}", flush=True)
    g, g64 = _split_vs_fp64(F, f, precision)
    assert col_err(g, g64).max() < tol
    ref = fft_linear(2, n, f)
    assert col_err(g, ref).max() < (1e-5 if precision == "fp16x3" else 1e-3)


def test_split_coherent_inputs_fio(fio128):
    f = _coherent_inputs(128)
    print("[split-range] 128^2 fio, coherent inputs, fp16x3", flush=True)
    g, g64 = _split_vs_fp64(fio128, f, "fp16x3")
    assert col_err(g, g64).max() < 5e-6


def test_fp16x3_single_rhs_scaled(fio128):
    """One right-hand side (the split path then also goes through the scaled lattice copy)."""
    f = W.complex_gaussian(128 * 128, 1, 73) * 3e3
    g = from_dev(fio128.apply(to_dev(f, torch.complex64)[0], precision="fp16x3").unsqueeze(0))
    g64 = from_dev(fio128.apply(to_dev(f)[0]).unsqueeze(0))
    assert np.isfinite(g).all() and col_err(g, g64).max() < 5e-6


def test_metric_workload_512x64_against_direct_sum():
    """512^2, 64 right-hand sides, autotuned kernels: split-fp16 and FP32 within 1e-5 and split-bf16
    within 1e-3 of the FP64 direct sum on the 256 seeded rows (Sec. 4's sampled error)."""
    M = _mod()
    w = W.WORKLOADS["fio512x64"]
    print("[split-range] building 512^2 (FP32, bf16 and fp16 copies)", flush=True)
    F = M.MIDBF(w.d, w.n, w.phase, tol=w.tol, precisions=2 | 4 | 8)
    f = W.complex_gaussian(w.N, w.nrhs, w.cfg)
    rows = W.sample_rows(w.N, w.cfg)
    gd = direct_sum(Kernel(w.d, w.n, w.phase), f, rows=rows)
    fd = to_dev(f, torch.complex64)
    for precision, tol in (("fp16x3", 1e-5), ("fp32", 1e-5), ("bf16x3", 1e-3)):
        F.tune(w.nrhs, precision)
        print(f"[split-range] 512^2 x 64 {precision}", flush=True)
        g = from_dev(F.apply(fd, precision=precision))
        assert np.isfinite(g[rows]).all()
        err = rel_l2(g[rows], gd)
        print(f"[split-range] 512^2 x 64 {precision}: rel L2 vs direct sum {err:.3e}", flush=True)
        assert err < tol, (precision, err)
        assert col_err(g[rows], gd).max() < 2 * tol
    F.close()
