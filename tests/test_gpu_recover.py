"""Phase recovery on the GPU against the oracle (needs an MI355X).

The library and the oracle draw their samples in the same splitmix64 orders,
so the accepted rows and columns, the integer shifts, the threshold and the
flagged nodes are compared exactly; the factors U, V are not unique (pivots
chosen on rounding-level residuals, signs of the bases), so the comparison is
on U V^T, on eps^K against K, and on the closed-form phase where one exists.
"""
import numpy as np
import pytest

import workloads as W
from oracle.kernel import Kernel, x_points, xi_points
from oracle.metrics import eps_K
from oracle.phase import reconciled_low_rank_factorization, recovery_path_lattice

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _mod():
    import paper_1908_09376_amd as M
    return M


def _sampler(Kfun, N):
    def sample(is_row, index):
        return Kfun([index], np.arange(N))[0] if is_row else Kfun(np.arange(N), [index])[:, 0]
    return sample


def _oracle(d, n, Kfun, xi, r, q, seed):
    N = n ** d
    kr = lambda i: Kfun([i], np.arange(N))[0]
    kc = lambda j: Kfun(np.arange(N), [j])[:, 0]
    P1 = recovery_path_lattice(d, n, (0,) * d)
    P2 = recovery_path_lattice(d, n, (n // 2,) * d)
    return reconciled_low_rank_factorization(kr, kc, N, P1, P2, xi, r, q, seed)


def _compare(info, H, oinfo):
    assert info["tau"] == H.tau
    assert info["disc_rows"] == len(H.Dr) - 1 and info["disc_cols"] == len(H.Dc) - 1
    assert np.array_equal(info["R"], oinfo["R"])
    assert np.array_equal(info["C"], oinfo["C"])
    assert np.array_equal(info["m"], oinfo["m"])
    assert np.array_equal(info["a"], oinfo["a"])


@pytest.mark.parametrize("n", [16, 32])
def test_recover_iso3d_integer_lattice(n):
    """The 3-D phase x.xi + c(x)|xi| on the integer frequency lattice (32^3: the recovered-phase workload)."""
    M = _mod()
    K = Kernel(3, n, "iso3d")
    N = K.N
    U, V, info = M.phase_recover(3, n, _sampler(K.entries, N), r=8, q=2, seed=500 + n)
    Uo, Vo, H, oinfo = _oracle(3, n, K.entries, xi_points(3, n), 8, 2, 500 + n)
    _compare(info, H, oinfo)
    U, V = U.cpu().numpy(), V.cpu().numpy()
    S = W.index_sample(N, 256, 3, 501)
    T = W.index_sample(N, 256, 3, 502)
    assert np.abs(U[S] @ V[T].T - Uo[S] @ Vo[T].T).max() < 1e-9
    # closed form: both anchors sit where Phi = 0, rank(Phi) = 4 <= r, so U V^T = Phi
    x, xi = x_points(3, n)[S], xi_points(3, n)[T]
    c = (3 + np.prod(np.sin(2 * np.pi * x), axis=1)) / 100
    Phi = x @ xi.T + c[:, None] * np.linalg.norm(xi, axis=1)[None, :]
    assert np.abs(U[S] @ V[T].T - Phi).max() < 1e-9
    assert eps_K(K.entries(S, S), U, V, S) < 1e-12


def _jump_phase(n):
    d = 2
    N = n ** d
    a = np.array(np.unravel_index(np.arange(N), (n,) * d)).T
    x = a / n
    xi = (a - n // 2) / n * 0.9

    def Kfun(I, J):
        I, J = np.atleast_1d(I), np.atleast_1d(J)
        Phi = x[I] @ xi[J].T + 0.35 * (x[I, 0] >= 0.5)[:, None] + 0.3 * (xi[J, 1] >= 0.2)[None, :]
        return np.exp(2j * np.pi * Phi)
    return Kfun, xi


def test_recover_discontinuous_phase_blocks_and_tau_schedule():
    """Jumps seen by the root column and the root row: the tau schedule rises to 0.3 and the
    row side splits into two blocks (Partition2); inside Lemma 2.2 otherwise, so no shifts."""
    M = _mod()
    n = 32
    N = n * n
    Kfun, xi = _jump_phase(n)
    U, V, info = M.phase_recover(2, n, _sampler(Kfun, N), r=8, q=2, seed=5, X2=xi)
    Uo, Vo, H, oinfo = _oracle(2, n, Kfun, xi, 8, 2, 5)
    _compare(info, H, oinfo)
    assert info["tau"] > 0.25 and info["disc_rows"] == 1
    assert info["rejected_rows"] == 0 and info["rejected_cols"] == 0
    U, V = U.cpu().numpy(), V.cpu().numpy()
    S = W.index_sample(N, 200, 1, 2)
    assert np.abs(U[S] @ V[S].T - Uo[S] @ Vo[S].T).max() < 1e-9
    assert eps_K(Kfun(S, S), U, V, S) < 1e-12


def test_recover_errors():
    M = _mod()
    from paper_1908_09376_amd._lib import MidbfError
    K = Kernel(2, 16, "fio_ellipse")
    with pytest.raises(MidbfError, match="ERR_ARG"):
        M.phase_recover(2, 16, _sampler(K.entries, 256), r=20)

    def bad(is_row, index):
        raise RuntimeError("sampler down")
    with pytest.raises(RuntimeError, match="sampler down"):
        M.phase_recover(2, 16, bad, r=4)


def test_iso3d32_recovered_phase_transform_end_to_end():
    """The 32^3 workload: phase recovered from rows / columns of K, MIDBF built on exp(2 pi i U V^T),
    16 right-hand sides applied in FP32 (matrix cores) and FP64, checked against the direct sum of
    the true K on seeded sampled rows."""
    M = _mod()
    n, d = 32, 3
    K = Kernel(d, n, "iso3d")
    N = K.N
    U, V, info = M.phase_recover(d, n, _sampler(K.entries, N), r=8, q=2, seed=3500)
    F = M.MIDBF(d, n, "lowrank", tol=1e-6, U=U, V=V, precisions=1 | 2)
    st = F.stats()
    assert st["L"] == 2 and st["b"] == 1
    f = W.complex_gaussian(N, 16, 3)
    rows = W.sample_rows(N, 3, 64)
    ref = K.entries(rows, np.arange(N)) @ f
    f32 = torch.from_numpy(np.ascontiguousarray(f.T)).to("cuda:0").to(torch.complex64)
    g32 = F.apply(f32, precision="fp32").to(torch.complex128).cpu().numpy().T
    assert np.linalg.norm(g32[rows] - ref) / np.linalg.norm(ref) < 1e-5
    f64 = torch.from_numpy(np.ascontiguousarray(f.T)).to("cuda:0")
    g64 = F.apply(f64, precision="fp64").cpu().numpy().T
    assert np.linalg.norm(g64[rows] - ref) / np.linalg.norm(ref) < 1e-6
    # the FP32 16-RHS apply equals 16 single FP32 applies up to FP32 rounding
    g1 = F.apply(f32[3].contiguous(), precision="fp32").to(torch.complex128).cpu().numpy()
    assert np.linalg.norm(g1 - g32[:, 3]) / np.linalg.norm(g1) < 1e-5
