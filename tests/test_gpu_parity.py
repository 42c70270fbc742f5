"""Parity of the HIP path with the CPU oracle (needs an MI355X).

Every comparison is against the FP64 definition (the direct sum of eq. 1) or
a closed form computed by the oracle on the same seeded inputs; the library
is called through its C interface.
"""
import numpy as np
import pytest

import workloads as W
from oracle.kernel import Kernel, direct_sum, direct_sum_adjoint, fft_linear
from oracle.metrics import rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _mod():
    import paper_1908_09376_amd as M
    return M


def to_dev(a: np.ndarray, dtype=torch.complex128):
    """(N, r) column-major numpy -> (r, N) contiguous CUDA tensor."""
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(DEV).to(dtype)


def from_dev(t) -> np.ndarray:
    return t.to(torch.complex128).cpu().numpy().T


# ---- kernel entries -------------------------------------------------------

def _entries_reduced_exactly(d, n, phase, rows, cols):
    """exp(2 pi i Phi) with the bilinear part x . xi = a . (b - n/2) / n reduced mod 1 in Python
    integers (exact) and only the smooth part (|.| <~ 70 turns here) rounded in FP64."""
    grid = np.stack(np.meshgrid(*([np.arange(n)] * d), indexing="ij"), -1).reshape(-1, d)
    a = grid[rows].astype(object)
    b = (grid[cols] - n // 2).astype(object)
    lin = np.array([[int(sum(ai * bi for ai, bi in zip(ar, br))) % n for br in b] for ar in a],
                   dtype=np.float64) / n
    x = grid[rows].astype(np.float64) / n
    xi = (grid[cols] - n // 2).astype(np.float64)
    tp = 2.0 * np.pi
    if phase == "linear":
        smooth = np.zeros((len(rows), len(cols)))
    elif phase == "fio_ellipse":
        c1 = (2.0 + np.sin(tp * x[:, 0]) * np.sin(tp * x[:, 1])) / 16.0
        c2 = (2.0 + np.cos(tp * x[:, 0]) * np.cos(tp * x[:, 1])) / 16.0
        smooth = np.sqrt(c1[:, None] ** 2 * xi[None, :, 0] ** 2 + c2[:, None] ** 2 * xi[None, :, 1] ** 2)
    elif phase == "fio_piecewise":
        c = np.where(x[:, 0] < 0.5, (2.0 + np.sin(tp * x[:, 0])) / 16.0, (3.0 + np.cos(tp * x[:, 1])) / 16.0)
        smooth = c[:, None] * np.linalg.norm(xi, axis=1)[None, :]
    else:
        c = (3.0 + np.prod(np.sin(tp * x), axis=1)) / 100.0
        smooth = c[:, None] * np.linalg.norm(xi, axis=1)[None, :]
    return np.exp(2j * np.pi * np.mod(lin + smooth, 1.0))


@pytest.mark.parametrize("d,n,phase", [(2, 64, "fio_ellipse"), (2, 512, "fio_ellipse"), (2, 256, "fio_piecewise"),
                                       (2, 128, "linear"), (3, 32, "iso3d")])
def test_kernel_entries_match_oracle(d, n, phase):
    M = _mod()
    N = n ** d
    rows = W.index_sample(N, 300, 31, n)
    cols = W.index_sample(N, 300, 32, n)
    K = M.kernel_entries(d, n, phase, torch.from_numpy(rows).to(DEV), torch.from_numpy(cols).to(DEV))
    got = K.cpu().numpy()
    ref = Kernel(d, n, phase).entries(rows, cols)
    # |Phi| <= ~600 here: the oracle's unreduced FP64 phase carries ~2 pi |Phi| eps ~ 1e-12 of rounding
    assert np.abs(got - ref).max() < 2e-11
    # against the same phase with its bilinear part reduced exactly: only the smooth part's rounding
    # (~70 eps turns) and the sine / cosine remain on either side
    exact = _entries_reduced_exactly(d, n, phase, rows, cols)
    assert np.abs(got - exact).max() < 2e-13


def test_kernel_entries_lowrank():
    M = _mod()
    N = 32 * 32
    U, V = W.random_lowrank_factors(N, 5, 33)
    rows = W.index_sample(N, 200, 34)
    cols = W.index_sample(N, 200, 35)
    K = M.kernel_entries(2, 32, "lowrank", torch.from_numpy(rows).to(DEV), torch.from_numpy(cols).to(DEV),
                         U=torch.from_numpy(U).to(DEV), V=torch.from_numpy(V).to(DEV))
    ref = Kernel(2, 32, ("lowrank", U, V)).entries(rows, cols)
    assert np.abs(K.cpu().numpy() - ref).max() < 1e-12


# ---- batched interpolative decomposition -----------------------------------

@pytest.mark.parametrize("tol", [1e-6, 1e-9])
def test_id_batch_cpqr_bound_and_rank(tol):
    M = _mod()
    from oracle.midbf import Tree, column_id, mock_chebyshev_points
    K = Kernel(2, 128, "fio_ellipse")
    tr = Tree(2, 128, 8)
    Xs = []
    for j in range(6):
        cand = np.concatenate([tr.points(4, 4 * (7 * j + 3) + t) for t in range(4)])   # 16x16 box, 256 cands
        smp = mock_chebyshev_points(tr, 2, (5 * j + 1) % 16, 320)
        Xs.append(K.entries(cand, smp).T)                                               # row-side matrix
    X = np.stack(Xs)
    m, n = X.shape[1:]
    k, perm, T = M.id_batch(torch.from_numpy(X.copy()).to(DEV), tol)
    for b in range(len(Xs)):
        A = Xs[b]
        kb = int(k[b])
        p = perm[b]
        assert sorted(p.tolist()) == list(range(n))
        Tb = T[b].cpu().numpy()
        rec = np.zeros_like(A)
        rec[:, p] = A[:, p[:kb]] @ np.hstack([np.eye(kb), Tb])
        ref2 = (np.abs(A) ** 2).sum(axis=0).max()
        # ||X - X_skel [I T] Pi^T||_F = ||R22||_F <= sqrt(n-k) tol max_j ||X[:, j]||
        assert np.linalg.norm(rec - A) <= np.sqrt(n - kb) * tol * np.sqrt(ref2) * (1 + 1e-6) + 1e-12
        ko = column_id(A, tol)[0]
        assert abs(kb - ko) <= max(3, int(0.05 * ko)), (kb, ko)


def test_id_batch_exact_low_rank():
    M = _mod()
    rng = W.rng(36, 0)
    A = (rng.standard_normal((3, 90, 9)) + 1j * rng.standard_normal((3, 90, 9))) @ \
        (rng.standard_normal((3, 9, 70)) + 1j * rng.standard_normal((3, 9, 70)))
    k, perm, T = M.id_batch(torch.from_numpy(A.copy()).to(DEV), 1e-10)
    assert (k == 9).all()
    for b in range(3):
        rec = np.zeros_like(A[b])
        rec[:, perm[b]] = A[b][:, perm[b][:9]] @ np.hstack([np.eye(9), T[b].cpu().numpy()])
        assert rel_l2(rec, A[b]) < 1e-11


def _low_rank(rng, b, m, n, r):
    A = (rng.standard_normal((b, m, r)) + 1j * rng.standard_normal((b, m, r))) @ \
        (rng.standard_normal((b, r, n)) + 1j * rng.standard_normal((b, r, n)))
    return A


@pytest.mark.parametrize("m,n,r", [(64, 2048, 12), (4096, 32, 7), (37, 301, 5), (5, 40, 9), (1, 17, 1),
                                   (33, 1, 1)])
def test_id_batch_edge_shapes(m, n, r):
    """The largest candidate count (2048) and sample count (4096) the kernel takes, sizes off every
    block (rows not a multiple of the 32-row staging or the 4-row loads, columns not a multiple of the
    256 threads or the 16-pivot panels), fewer rows than the rank (wide: rank m), one row, one column.
    Exact low-rank inputs: the rank is min(r, m, n) and the ID reproduces the matrix."""
    M = _mod()
    A = _low_rank(W.rng(38, m + n), 2, m, n, r)
    k, perm, T = M.id_batch(torch.from_numpy(A.copy()).to(DEV), 1e-10)
    want = min(r, m, n)
    for b in range(2):
        assert int(k[b]) == want, (m, n, r, k)
        assert sorted(perm[b].tolist()) == list(range(n))
        kb = int(k[b])
        rec = np.zeros_like(A[b])
        rec[:, perm[b]] = A[b][:, perm[b][:kb]] @ np.hstack([np.eye(kb), T[b].cpu().numpy()])
        assert rel_l2(rec, A[b]) < 1e-10, (m, n, r)


def test_id_batch_zero_and_mixed_matrices():
    """A zero matrix has rank 0 (T empty, every column redundant); it may share a batch with others."""
    M = _mod()
    A = _low_rank(W.rng(39, 0), 3, 50, 40, 6)
    A[1] = 0.0
    k, perm, T = M.id_batch(torch.from_numpy(A.copy()).to(DEV), 1e-10)
    assert int(k[1]) == 0 and tuple(T[1].shape) == (0, 40)
    assert int(k[0]) == 6 and int(k[2]) == 6


def test_id_batch_refuses_beyond_its_sizes():
    M = _mod()
    for m, n in ((8, 2049), (4097, 8)):
        X = torch.zeros((1, m, n), dtype=torch.complex128, device=DEV)
        with pytest.raises(Exception):
            M.id_batch(X, 1e-6)


# ---- whole-transform parity ------------------------------------------------

def _build(n, phase, d=2, **kw):
    M = _mod()
    return M.MIDBF(d, n, phase, **kw)


@pytest.mark.parametrize("n", [16, 32, 64])
@pytest.mark.parametrize("phase", ["fio_ellipse", "fio_piecewise"])
def test_apply_fp64_matches_direct_sum_small(n, phase):
    F = _build(n, phase)
    K = Kernel(2, n, phase)
    f = W.complex_gaussian(K.N, 1, 0)
    g = from_dev(F.apply(to_dev(f)[0]).unsqueeze(0))
    gd = direct_sum(K, f)
    assert rel_l2(g, gd) < 1e-5


def test_fio64_fp64_and_fp32():
    # 64^2 ellipse phase, tolerance 1e-6, single RHS: full-vector error vs the direct sum
    w = W.WORKLOADS["fio64"]
    F = _build(w.n, w.phase, tol=w.tol)
    K = Kernel(2, w.n, w.phase)
    f = W.rhs_for(w)
    gd = direct_sum(K, f)
    g64 = from_dev(F.apply(to_dev(f)[0]).unsqueeze(0))
    g32 = from_dev(F.apply(to_dev(f, torch.complex64)[0], precision="fp32").unsqueeze(0))
    assert rel_l2(g64, gd) < 1e-5
    assert rel_l2(g32, gd) < 1e-5
    st = F.stats()
    assert st["L"] == 3 and st["b"] == 2 and st["hstar"] == 2


@pytest.mark.parametrize("n", [64, 128])
def test_linear_phase_matches_fft(n):
    F = _build(n, "linear")
    f = W.complex_gaussian(n * n, 3, 37)
    g = from_dev(F.apply(to_dev(f)))
    assert rel_l2(g, fft_linear(2, n, f)) < 1e-5


def test_adjoint_identity_and_direct_adjoint():
    F = _build(64, "fio_ellipse")
    K = Kernel(2, 64, "fio_ellipse")
    f = W.complex_gaussian(K.N, 2, 38)
    h = W.complex_gaussian(K.N, 2, 39)
    Kf = from_dev(F.apply(to_dev(f)))
    KHh = from_dev(F.apply_adjoint(to_dev(h)))
    lhs = np.vdot(h, Kf)
    rhs = np.vdot(KHh, f)
    assert abs(lhs - rhs) / abs(lhs) < 1e-12
    assert rel_l2(KHh, direct_sum_adjoint(K, h)) < 1e-5
    KHh32 = from_dev(F.apply_adjoint(to_dev(h, torch.complex64), precision="fp32"))
    assert rel_l2(KHh32, direct_sum_adjoint(K, h)) < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_multi_rhs_equals_single(precision):
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    F = _build(64, "fio_ellipse")
    f = W.complex_gaussian(64 * 64, 11, 40)
    many = from_dev(F.apply(to_dev(f, dt), precision=precision))
    ones = np.stack([from_dev(F.apply(to_dev(f[:, j:j + 1], dt)[0], precision=precision).unsqueeze(0))[:, 0]
                     for j in range(11)], axis=1)
    assert rel_l2(many, ones) < (1e-14 if precision == "fp64" else 1e-6)


def test_apply_is_deterministic():
    F = _build(64, "fio_ellipse")
    f = to_dev(W.complex_gaussian(64 * 64, 2, 41), torch.complex64)
    a = F.apply(f, precision="fp32")
    b = F.apply(f, precision="fp32")
    assert torch.equal(a, b)


def test_fio256_sampled_rows_fp64_fp32():
    w = W.WORKLOADS["fio256"]
    F = _build(w.n, w.phase, tol=w.tol)
    K = Kernel(2, w.n, w.phase)
    f = W.rhs_for(w)
    rows = W.sample_rows(K.N, w.cfg)
    gd = direct_sum(K, f, rows=rows)
    g64 = from_dev(F.apply(to_dev(f)[0]).unsqueeze(0))
    g32 = from_dev(F.apply(to_dev(f, torch.complex64)[0], precision="fp32").unsqueeze(0))
    assert rel_l2(g64[rows], gd) < 1e-5
    assert rel_l2(g32[rows], gd) < 1e-5


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp16x3", 5e-6), ("bf16x3", 1e-4)])
def test_many_rhs_tiles(precision, tol):
    """257 right-hand sides: five 64-column tiles on the matrix cores, the last holding one column."""
    F = _build(64, "fio_ellipse", precisions=1 | 2 | 4 | 8)
    f = W.complex_gaussian(64 * 64, 257, 50, 64)
    g64 = from_dev(F.apply(to_dev(f)))
    g = from_dev(F.apply(to_dev(f, torch.complex64), precision=precision))
    assert g.shape == g64.shape and np.isfinite(g).all()
    assert rel_l2(g, g64) < tol
    assert rel_l2(g[:, -1:], g64[:, -1:]) < 2 * tol


def test_split_adjoint_refused():
    """The split 16-bit copies serve the forward transform only: an adjoint in them is refused with
    MIDBF_ERR_UNIMPLEMENTED, and the FP32 adjoint of the same handle still runs."""
    M = _mod()
    from paper_1908_09376_amd._lib import MidbfError
    F = _build(64, "fio_ellipse", precisions=1 | 2 | 8)
    g = torch.zeros((64, 64 * 64), dtype=torch.complex64, device=DEV)
    with pytest.raises(MidbfError, match="UNIMPLEMENTED"):
        F.apply_adjoint(g, precision="fp16x3")
    assert torch.isfinite(F.apply_adjoint(g, precision="fp32").abs()).all()


def test_errors_reported():
    M = _mod()
    from paper_1908_09376_amd._lib import MidbfError
    with pytest.raises(MidbfError):
        M.MIDBF(2, 60, "fio_ellipse")          # 60 is not 8 * 2^L
    F = _build(32, "fio_ellipse", precisions=1)
    with pytest.raises(MidbfError):
        F.apply(torch.zeros(1024, dtype=torch.complex64, device=DEV), precision="fp32")
    # a caller's output block is checked before any launch
    f = torch.zeros(1024, dtype=torch.complex128, device=DEV)
    with pytest.raises(TypeError):
        F.apply(f, out=torch.zeros(1024, dtype=torch.complex64, device=DEV))
    with pytest.raises(ValueError):
        F.apply(f, out=torch.zeros(1000, dtype=torch.complex128, device=DEV))
    with pytest.raises(ValueError):
        F.apply_adjoint(f, out=torch.zeros((2, 1024), dtype=torch.complex128, device=DEV))
    # a negative count is rejected by midbf_ranks
    import ctypes
    from paper_1908_09376_amd import _lib
    buf = (ctypes.c_int * 4)()
    assert _lib.lib.midbf_ranks(F._h, 0, 0, buf, -1) == -1
    assert b"count" in _lib.lib.midbf_last_error()
    # the C ABI refuses an empty block, a short leading dimension and null vectors before any launch
    g = torch.empty_like(f)
    fp, gp = ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(g.data_ptr())
    assert _lib.lib.midbf_apply(F._h, fp, gp, 0, 1024, 0, None) == -1
    assert b"nrhs" in _lib.lib.midbf_last_error()
    assert _lib.lib.midbf_apply(F._h, fp, gp, 1, 1000, 0, None) == -1
    assert b"ld" in _lib.lib.midbf_last_error()
    assert _lib.lib.midbf_apply(F._h, None, gp, 1, 1024, 0, None) == -1
    assert _lib.lib.midbf_apply(F._h, fp, gp, 1, 1024, 0, None) == 0          # the same call, well formed


# ---- matrix-core path (many right-hand sides, FP32) -------------------------

@pytest.mark.parametrize("n,nrhs", [(64, 16), (64, 64), (64, 70), (128, 64), (256, 33)])
def test_mfma_many_rhs_fp32(n, nrhs):
    F = _build(n, "fio_ellipse")
    K = Kernel(2, n, "fio_ellipse")
    f = W.complex_gaussian(K.N, nrhs, 42, n)
    g32 = from_dev(F.apply(to_dev(f, torch.complex64), precision="fp32"))
    g64 = from_dev(F.apply(to_dev(f)))
    assert rel_l2(g32, g64) < 1e-5
    rows = W.sample_rows(K.N, 0, 128)
    gd = direct_sum(K, f, rows=rows)
    assert rel_l2(g32[rows], gd) < 1e-5
    # every right-hand side individually
    per = np.linalg.norm(g32[rows] - gd, axis=0) / np.linalg.norm(gd, axis=0)
    assert per.max() < 2e-5


@pytest.mark.parametrize("variant", range(10))
def test_mfma_every_tile_variant(variant):
    F = _build(128, "fio_ellipse")
    f = W.complex_gaussian(128 * 128, 40, 43)
    g64 = from_dev(F.apply(to_dev(f)))
    F.set_variants([variant] * 3, precision="fp32")
    g32 = from_dev(F.apply(to_dev(f, torch.complex64), precision="fp32"))
    assert rel_l2(g32, g64) < 1e-5


def test_autotuner_picks_valid_variants():
    F = _build(64, "fio_ellipse")
    v = F.tune(64, "fp32")
    assert len(v) == 3 and all(0 <= x < 10 for x in v)
    f = W.complex_gaussian(64 * 64, 64, 44)
    g32 = from_dev(F.apply(to_dev(f, torch.complex64), precision="fp32"))
    assert rel_l2(g32, from_dev(F.apply(to_dev(f)))) < 1e-5


# ---- split-bf16 matrix-core path ---------------------------------------------

@pytest.mark.parametrize("n,nrhs", [(64, 64), (128, 20), (256, 64)])
def test_bf16x3_apply(n, nrhs):
    F = _build(n, "fio_ellipse")
    K = Kernel(2, n, "fio_ellipse")
    f = W.complex_gaussian(K.N, nrhs, 45, n)
    gb = from_dev(F.apply(to_dev(f, torch.complex64), precision="bf16x3"))
    g64 = from_dev(F.apply(to_dev(f)))
    err = rel_l2(gb, g64)
    assert err < 1e-4, err           # split-bf16 target is 1e-3 against the direct sum
    rows = W.sample_rows(K.N, 0, 64)
    assert rel_l2(gb[rows], direct_sum(K, f, rows=rows)) < 1e-3


@pytest.mark.parametrize("variant", range(11))
def test_bf16x3_every_variant(variant):
    F = _build(128, "fio_ellipse")
    f = W.complex_gaussian(128 * 128, 64, 46)
    g64 = from_dev(F.apply(to_dev(f)))
    F.set_variants([variant] * 3, precision="bf16x3")
    gb = from_dev(F.apply(to_dev(f, torch.complex64), precision="bf16x3"))
    assert rel_l2(gb, g64) < 1e-4
    assert F.tune(64, "bf16x3")[0] in range(11)


# ---- split-fp16 matrix-core path ---------------------------------------------

@pytest.mark.parametrize("n,nrhs", [(64, 64), (128, 20), (256, 64)])
def test_fp16x3_apply(n, nrhs):
    """fp16 hi + lo keeps ~2^-22 per split value: FP32-level error against the FP64 apply."""
    F = _build(n, "fio_ellipse", precisions=1 | 2 | 8)
    K = Kernel(2, n, "fio_ellipse")
    f = W.complex_gaussian(K.N, nrhs, 47, n)
    gh = from_dev(F.apply(to_dev(f, torch.complex64), precision="fp16x3"))
    g64 = from_dev(F.apply(to_dev(f)))
    assert rel_l2(gh, g64) < 5e-6
    rows = W.sample_rows(K.N, 0, 64)
    assert rel_l2(gh[rows], direct_sum(K, f, rows=rows)) < 1e-5
    assert F.stats()["bytes_fp16"] > 0


@pytest.mark.parametrize("variant", range(11))
def test_fp16x3_every_variant(variant):
    F = _build(128, "fio_ellipse", precisions=1 | 8)
    f = W.complex_gaussian(128 * 128, 64, 48)
    g64 = from_dev(F.apply(to_dev(f)))
    F.set_variants([variant] * 3, precision="fp16x3")
    gh = from_dev(F.apply(to_dev(f, torch.complex64), precision="fp16x3"))
    assert rel_l2(gh, g64) < 5e-6
    assert F.tune(64, "fp16x3")[0] in range(11)


@pytest.mark.parametrize("n,nrhs", [(64, 70), (256, 64), (256, 20)])
@pytest.mark.parametrize("variant", [9, 10])
def test_fp16x3_two_workgroup_middle_odd_levels(n, nrhs, variant):
    """Split variant 10 runs the middle kinds with two 512-thread workgroups per CU (two-tile B
    stages).  L odd (64^2: L = 3, 256^2: L = 5) gives single-piece middle blocks and ragged right-hand
    side tiles (70 = 64 + 6, 20); the result must match the FP64 apply as variant 9's does."""
    F = _build(n, "fio_ellipse", precisions=1 | 8)
    f = W.complex_gaussian(n * n, nrhs, 49, n)
    g64 = from_dev(F.apply(to_dev(f)))
    F.set_variants([variant] * 3, precision="fp16x3")
    gh = from_dev(F.apply(to_dev(f, torch.complex64), precision="fp16x3"))
    assert rel_l2(gh, g64) < 5e-6, (n, nrhs, variant)


@pytest.mark.parametrize("precision", ["fp16x3", "bf16x3"])
@pytest.mark.parametrize("n,nrhs", [(64, 70), (128, 64), (256, 20)])
def test_split_exchange_top_up_to_middle(precision, n, nrhs):
    """The top up step hands the middle its output already split into hi / lo halves when both run
    source-table kernels (variants 7-10); the halves come from the same conversions as the middle's
    own split, so the apply is bitwise the one with FP32 pairs (MIDBF_SPLIT_EXCHANGE=0).  Mixed
    variant sets where one side is outside 7-10 turn the exchange off by themselves."""
    import os
    F = _build(n, "fio_ellipse", precisions=1 | 4 | 8)
    f = W.complex_gaussian(n * n, nrhs, 83, n)
    fd = to_dev(f, torch.complex64)
    g64 = from_dev(F.apply(to_dev(f)))
    for vs in ([9, 8, 10], [10, 10, 10], [7, 6, 7], [9, 8, 5], [2, 8, 10]):
        F.set_variants(vs, precision=precision)
        print(f"[exchange] {precision} {n}^2 x {nrhs} variants {vs}", flush=True)
        g = F.apply(fd, precision=precision)
        os.environ["MIDBF_SPLIT_EXCHANGE"] = "0"
        try:
            g_pairs = F.apply(fd, precision=precision)
        finally:
            del os.environ["MIDBF_SPLIT_EXCHANGE"]
        assert torch.equal(g, g_pairs), (precision, n, nrhs, vs)
        assert rel_l2(from_dev(g), g64) < (5e-6 if precision == "fp16x3" else 1e-4), (precision, vs)


@pytest.mark.parametrize("nrhs", [64, 70])
def test_fp16x3_lattice_input_path(nrhs):
    """When the first up step keeps every leaf point (64^2: every leaf decomposition is full rank),
    the table-driven split kernels (variants 7-10) transpose the input into the row-major copy and
    the step above reads it through lattice rows; the other variants keep the first-step copy.
    Both must match the FP64 apply; the profile shows which path ran."""
    n = 64
    F = _build(n, "fio_ellipse", precisions=1 | 8)
    assert int(F.ranks(1, 0).min()) == 64         # no redundant leaf points on the column side
    f = W.complex_gaussian(n * n, nrhs, 64, n)
    g64 = from_dev(F.apply(to_dev(f)))
    for v, lattice in ((9, True), (10, True), (7, True), (0, False)):
        F.set_variants([v] * 3, precision="fp16x3")
        F.profile(True, by_level=True)
        g = from_dev(F.apply(to_dev(f, torch.complex64), precision="fp16x3"))
        names = [r["name"] for r in F.profile_read()]
        F.profile(False)
        assert ("transpose_fp16x3_in" in names) == lattice, (v, names)
        assert rel_l2(g, g64) < 5e-6, v


def test_split16_precisions_need_their_copy():
    F = _build(64, "fio_ellipse", precisions=1 | 2)
    from paper_1908_09376_amd._lib import MidbfError
    f = to_dev(W.complex_gaussian(64 * 64, 16, 49), torch.complex64)
    with pytest.raises(MidbfError, match="ERR_ARG"):
        F.apply(f, precision="fp16x3")


# ---- rank-deficient leaves ---------------------------------------------------

@pytest.mark.parametrize("precision,variant", [("fp32", None), ("bf16x3", 0), ("bf16x3", 8), ("fp16x3", 2),
                                               ("fp16x3", 7), ("fp16x3", 9)])
def test_compressible_leaves_many_rhs(precision, variant):
    """A slowly varying low-rank phase: the leaf column IDs keep few of their 64 columns, so the
    first up step multiplies T by the redundant rows of the caller's column-major input (70
    right-hand sides: a second, ragged block of 64)."""
    M = _mod()
    n = 64
    N = n * n
    U, V = W.random_lowrank_factors(N, 2, 61)
    U, V = U * 0.1, V * 0.1
    F = M.MIDBF(2, n, "lowrank", U=torch.from_numpy(U).to(DEV), V=torch.from_numpy(V).to(DEV),
                precisions=1 | 2 | 4 | 8)
    k0 = F.ranks(1, 0)
    assert 0 < k0.max() < 64
    if variant is not None:
        F.set_variants([variant] * 3, precision=precision)
    f = W.complex_gaussian(N, 70, 62)
    g = from_dev(F.apply(to_dev(f, torch.complex64), precision=precision))
    g64 = from_dev(F.apply(to_dev(f)))
    assert rel_l2(g, g64) < (1e-4 if precision == "bf16x3" else 5e-6)
    rows = W.sample_rows(N, 4, 64)
    gd = direct_sum(Kernel(2, n, ("lowrank", U, V)), f, rows=rows)
    assert rel_l2(g64[rows], gd) < 1e-5


# ---- FP64 matrix cores ----------------------------------------------------------

def _single_fp64(F, f, j):
    return from_dev(F.apply(to_dev(f[:, j:j + 1])[0]).unsqueeze(0))[:, 0]


@pytest.mark.parametrize("n,nrhs", [(64, 16), (128, 64), (256, 33)])
def test_mfma_fp64_equals_single_rhs(n, nrhs):
    """FP64 with 16 or more RHS runs on v_mfma_f64 (Gauss's three products); each column equals the
    FP64 VALU apply of that column alone up to FP64 rounding, and the direct sum within the ID error."""
    F = _build(n, "fio_ellipse")
    f = W.complex_gaussian(n * n, nrhs, 51, n)
    many = from_dev(F.apply(to_dev(f)))
    for j in (0, nrhs // 2, nrhs - 1):
        one = _single_fp64(F, f, j)
        assert np.linalg.norm(many[:, j] - one) / np.linalg.norm(one) < 1e-12
    K = Kernel(2, n, "fio_ellipse")
    rows = W.sample_rows(K.N, 0, 64)
    assert rel_l2(many[rows], direct_sum(K, f, rows=rows)) < 1e-5


@pytest.mark.parametrize("variant", range(5))
def test_mfma_fp64_every_variant(variant):
    F = _build(128, "fio_ellipse")
    f = W.complex_gaussian(128 * 128, 70, 52)
    F.set_variants([variant] * 3, precision="fp64")
    many = from_dev(F.apply(to_dev(f)))
    for j in (0, 69):
        one = _single_fp64(F, f, j)
        assert np.linalg.norm(many[:, j] - one) / np.linalg.norm(one) < 1e-12
    assert all(v in range(5) for v in F.tune(64, "fp64"))
