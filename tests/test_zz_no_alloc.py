"""midbf_apply_noalloc (the apply that allocates nothing) against midbf_apply (needs an MI355X).

Both calls run the same kernels with the same launch shapes; only the home of
the level vectors differs (the library's static device scratch instead of the
handle's workspace), so their outputs must agree bit for bit.  Each case makes
two no-allocation calls in a row, the second with a smaller input, so that
the second one runs over the first one's leftovers in the shared scratch.
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _mod():
    import paper_1908_09376_amd as M
    return M


def _rhs(n, nrhs, key, dtype):
    f = W.complex_gaussian(n * n, nrhs, 90, key)
    t = torch.from_numpy(np.ascontiguousarray(f.T)).to(DEV).to(dtype)
    return t.reshape(nrhs, n * n) if nrhs > 1 else t.reshape(n * n)


def _check_pair(M, big, small, precision, nrhs_big, nrhs_small, tune=False):
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    for k, (F, nrhs) in enumerate(((big, nrhs_big), (small, nrhs_small))):
        if tune:
            F.tune(nrhs, precision)
        f = _rhs(F.n, nrhs, 10 * k + nrhs, dt)
        print(f"[noalloc] N={F.n}^2 nrhs={nrhs} {precision}", flush=True)
        ref = F.apply(f, precision=precision)
        got = torch.full_like(f, float("nan"))
        F.apply_noalloc(f, out=got, precision=precision)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (precision, F.n, nrhs)


def test_noalloc_fp64_single_rhs_then_smaller():
    M = _mod()
    big = M.MIDBF(2, 128, "fio_ellipse", tol=1e-6)
    small = M.MIDBF(2, 64, "fio_piecewise", tol=1e-6)
    _check_pair(M, big, small, "fp64", 1, 1)


def test_noalloc_fp32_few_rhs_then_fewer():
    M = _mod()
    F = M.MIDBF(2, 128, "fio_ellipse", tol=1e-6)
    _check_pair(M, F, F, "fp32", 5, 2)


def test_noalloc_matrix_cores_fp32_then_smaller():
    M = _mod()
    big = M.MIDBF(2, 64, "fio_ellipse", tol=1e-6)
    small = M.MIDBF(2, 64, "linear", tol=1e-6)
    _check_pair(M, big, small, "fp32", 40, 16, tune=True)


def test_noalloc_split_fp16_then_smaller():
    M = _mod()
    keep = 1 | 2 | 8
    big = M.MIDBF(2, 64, "fio_ellipse", tol=1e-6, precisions=keep)
    small = M.MIDBF(2, 64, "linear", tol=1e-6, precisions=keep)
    _check_pair(M, big, small, "fp16x3", 32, 20, tune=True)


def test_noalloc_rejects_beyond_its_scratch():
    M = _mod()
    from paper_1908_09376_amd import _lib as L
    F = M.MIDBF(2, 128, "linear", tol=1e-6)
    nrhs = 512                       # the lattice copy alone is 128^2 * 512 * 16 B = 128 MiB
    f = torch.zeros(nrhs, F.N, dtype=torch.complex128, device=DEV)
    with pytest.raises(L.MidbfError) as e:
        F.apply_noalloc(f, precision="fp64")
    assert e.value.code == -2 and "scratch" in str(e.value)
    # a regular apply of the same size still works afterwards, and so does a small no-allocation one
    g = F.apply(f[:1].reshape(-1), precision="fp64")
    h = F.apply_noalloc(f[:1].reshape(-1), precision="fp64")
    torch.cuda.synchronize()
    assert torch.equal(g, h)
