"""Factor files: save, load, and every apply equal to the saved handle's bit for bit (needs an MI355X).

A loaded factorization reads the decompositions (ranks, pivot orders, FP64 T blocks) instead of
computing them and packs everything else as the build does, so its applies must equal those of the
handle that was saved, in every precision, exactly.
"""
import numpy as np
import pytest

import workloads as W
from oracle.kernel import Kernel, direct_sum
from oracle.metrics import rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _mod():
    import paper_1908_09376_amd as M
    return M


def to_dev(a: np.ndarray, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(DEV).to(dtype)


def _same(a, b):
    return torch.equal(torch.view_as_real(a), torch.view_as_real(b))


def test_save_load_applies_equal_bitwise(tmp_path):
    M = _mod()
    n = 64
    F = M.MIDBF(2, n, "fio_ellipse", precisions=1 | 2)
    path = str(tmp_path / "fio64.midbf")
    print("[saveload] 64^2 save", flush=True)
    F.save(path)
    G = M.MIDBF.load(path, precisions=1 | 2 | 8)
    sF, sG = F.stats(), G.stats()
    for key in ("L", "b", "hstar", "ids", "entries", "k_min", "k_max", "index_bytes"):
        assert sF[key] == sG[key], key
    for side in (0, 1):
        for s in range(sF["b"]):
            assert np.array_equal(F.ranks(side, s), G.ranks(side, s))
    f = W.complex_gaussian(n * n, 3, 19)
    for prec, dt in (("fp64", torch.complex128), ("fp32", torch.complex64)):
        x = to_dev(f, dt)
        assert _same(F.apply(x, precision=prec), G.apply(x, precision=prec)), prec
        assert _same(F.apply_adjoint(x, precision=prec), G.apply_adjoint(x, precision=prec)), prec
    # the split copy made on loading equals the one of a fresh build of the same factorization
    H = M.MIDBF(2, n, "fio_ellipse", precisions=1 | 8)
    f64 = to_dev(W.complex_gaussian(n * n, 64, 20), torch.complex64)
    for X in (G, H):
        X.set_variants([9, 8, 9], precision="fp16x3")
    assert _same(G.apply(f64, precision="fp16x3"), H.apply(f64, precision="fp16x3"))
    rows = W.sample_rows(n * n, 0, 64)
    g = G.apply(to_dev(f)).to(torch.complex128).cpu().numpy().T
    assert rel_l2(g[rows], direct_sum(Kernel(2, n, "fio_ellipse"), f, rows=rows)) < 1e-5
    for X in (F, G, H):
        X.close()


def test_save_load_lowrank_phase_and_fixed_rank(tmp_path):
    """The low-rank phase's U and V travel in the file (the caller's copies are gone by then), and
    the fixed-rank parameter comes back with the parameters."""
    M = _mod()
    n = 32
    N = n * n
    U, V = W.random_lowrank_factors(N, 3, 34)
    Ut, Vt = torch.from_numpy(U).to(DEV), torch.from_numpy(V).to(DEV)
    F = M.MIDBF(2, n, "lowrank", U=Ut, V=Vt, fixed_rank=40, precisions=1 | 2)
    path = str(tmp_path / "lr32.midbf")
    F.save(path)
    f = to_dev(W.complex_gaussian(N, 2, 21))
    want = F.apply(f)
    F.close()
    del Ut, Vt
    torch.cuda.synchronize()
    G = M.MIDBF.load(path, precisions=1)
    assert G._p.fixed_rank == 40 and G._p.r == 3
    assert _same(G.apply(f), want)
    G.close()


def test_save_needs_fp64_and_load_refuses_damaged_files(tmp_path):
    M = _mod()
    from paper_1908_09376_amd._lib import MidbfError
    F = M.MIDBF(2, 32, "fio_ellipse", precisions=2)
    with pytest.raises(MidbfError, match="ERR_ARG"):
        F.save(str(tmp_path / "x.midbf"))
    F.close()
    F = M.MIDBF(2, 32, "fio_ellipse", precisions=1)
    path = tmp_path / "ok.midbf"
    F.save(str(path))
    F.close()
    data = path.read_bytes()
    # cut short: the last record and the ending are missing
    (tmp_path / "cut.midbf").write_bytes(data[: len(data) // 2])
    with pytest.raises(MidbfError, match="ERR_IO"):
        M.MIDBF.load(str(tmp_path / "cut.midbf"))
    # a pivot order that is not a permutation: the first pivot of the first decomposition repeats the
    # second (header 64 B, then nid (8), m and 0 (8), n[nid], k[nid], pivot orders)
    nid = 4 ** 3
    off = 64 + 16 + 8 * nid
    b = bytearray(data)
    b[off: off + 4] = b[off + 4: off + 8]
    (tmp_path / "perm.midbf").write_bytes(bytes(b))
    with pytest.raises(MidbfError, match="ERR_IO"):
        M.MIDBF.load(str(tmp_path / "perm.midbf"))
