"""The apply captured in a hipGraph (midbf_apply_graph_*) against the eager apply (needs an MI355X).

Each graph is replayed several times with other eager applies of the same
handle and host synchronizations in between; every replay must equal the
eager midbf_apply of the same input bit for bit (same kernels, same launch
shapes), and the inputs of later replays are changed in place to show that
the graph reads the buffers it was given.
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _rhs(n, nrhs, key, dtype):
    f = W.complex_gaussian(n * n, nrhs, 95, key)
    t = torch.from_numpy(np.ascontiguousarray(f.T)).to(DEV).to(dtype)
    return t.reshape(nrhs, n * n) if nrhs > 1 else t.reshape(n * n)


@pytest.mark.parametrize("n,nrhs,precision", [(128, 64, "fp16x3"), (128, 64, "bf16x3"), (64, 20, "fp32"),
                                              (64, 1, "fp64"), (64, 3, "fp32")])
def test_graph_replays_equal_eager(n, nrhs, precision):
    import paper_1908_09376_amd as M
    F = M.MIDBF(2, n, "fio_ellipse", tol=1e-6, precisions=1 | 2 | 4 | 8)
    if nrhs >= 16:
        F.tune(nrhs, precision)
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    f = _rhs(n, nrhs, 1, dt)
    G = M.ApplyGraph(F, f, precision=precision)
    other = _rhs(n, nrhs, 2, dt)
    for rep in range(4):
        print(f"[graph] N={n}^2 nrhs={nrhs} {precision} replay {rep}", flush=True)
        ref = F.apply(f, precision=precision)
        F.apply(other, precision=precision)            # eager work on the same handle between replays
        torch.cuda.synchronize()
        got = G.launch().clone()
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (precision, rep)
        f.mul_(-0.5).add_(other)                        # new input in place for the next replay
    G.close()
