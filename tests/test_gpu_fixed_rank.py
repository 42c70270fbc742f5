"""The fixed-rank variant (Sec. 3.5, closing paragraph) against the oracle's (needs an MI355X).

With a fixed rank every decomposition keeps min(rank, samples, candidates) columns, so the ranks and
the stored entry count follow from the geometry alone: they must equal the oracle's exactly.  The
pivots come from different column-pivoted QRs (sketch-chosen panels on the GPU, classical on the
CPU), so the apply is compared with the direct sum (eq. 1) against the oracle's own error there.
"""
import numpy as np
import pytest

import workloads as W
from oracle.kernel import Kernel, direct_sum
from oracle.metrics import rel_l2
from oracle.midbf import MIDBF as OracleMIDBF

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


@pytest.mark.parametrize("n,rank", [(32, 40), (64, 20), (64, 112)])
def test_fixed_rank_matches_oracle_ranks_entries_and_error(n, rank):
    M = _mod()
    K = Kernel(2, n, "fio_ellipse")
    print(f"[fixed-rank] {n}^2 rank {rank}", flush=True)
    O = OracleMIDBF(K, rank=rank)
    F = M.MIDBF(2, n, "fio_ellipse", fixed_rank=rank, precisions=1 | 2)
    st = F.stats()
    ot = O.rank_table()
    for side, name in ((0, "rows"), (1, "cols")):
        for s in range(st["b"]):
            assert sorted(F.ranks(side, s).tolist()) == sorted(ot[name][s]), (side, s)
    assert st["entries"] == O.entry_count()
    f = W.complex_gaussian(K.N, 2, 17)
    rows = W.sample_rows(K.N, 0, 128)
    gd = direct_sum(K, f, rows=rows)
    e_or = rel_l2(O.apply(f)[rows], gd)
    g = from_dev(F.apply(to_dev(f)))
    e_gpu = rel_l2(g[rows], gd)
    print(f"[fixed-rank] {n}^2 rank {rank}: GPU {e_gpu:.3e}, oracle {e_or:.3e}", flush=True)
    assert e_gpu < 3.0 * e_or + 1e-13
    g32 = from_dev(F.apply(to_dev(f, torch.complex64), precision="fp32"))
    assert rel_l2(g32, g) < 1e-5
    F.close()


def test_fixed_rank_split_many_rhs():
    """Uniform ranks through the split-fp16 matrix-core path, 64 right-hand sides."""
    M = _mod()
    n = 64
    F = M.MIDBF(2, n, "fio_ellipse", fixed_rank=112, precisions=1 | 8)
    F.tune(64, "fp16x3")
    f = W.complex_gaussian(n * n, 64, 18)
    g64 = from_dev(F.apply(to_dev(f)))
    g = from_dev(F.apply(to_dev(f, torch.complex64), precision="fp16x3"))
    assert rel_l2(g, g64) < 5e-6
    F.close()


def test_fixed_rank_rejects_negative():
    M = _mod()
    with pytest.raises(Exception):
        M.MIDBF(2, 32, "fio_ellipse", fixed_rank=-1)
