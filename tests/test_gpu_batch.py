"""Batched uneven transforms in one persistent launch (needs an MI355X).

The batch runs the same level-kernel bodies as a single apply, as tasks of
one queue taken by persistent workgroups; every output is compared with the
transform's own midbf_apply (bitwise: the same bodies on the same data) and
with the oracle's FP64 direct sum (eq. 1), and every run must finish with no
abandoned dependency wait.
"""
import numpy as np
import pytest

import workloads as W
from oracle.kernel import Kernel, direct_sum
from oracle.metrics import rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SMALL = [(16, "fio_ellipse"), (64, "fio_piecewise"), (32, "fio_ellipse"), (128, "linear"), (32, "linear"),
         (64, "fio_ellipse")]


def _mod():
    import paper_1908_09376_amd as M
    return M


def to_dev(a: np.ndarray, dtype):
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(DEV).to(dtype)


@pytest.fixture(scope="module")
def small():
    M = _mod()
    return [M.MIDBF(2, n, ph, tol=1e-6) for n, ph in SMALL]


def _inputs(nrhs_list, dtype, key):
    return [to_dev(W.complex_gaussian(n * n, r, key, j), dtype).reshape(-1, n * n).squeeze(0)
            for j, ((n, _), r) in enumerate(zip(SMALL, nrhs_list))]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_batch_equals_individual_applies(small, precision, nrhs):
    M = _mod()
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    fs = _inputs([nrhs] * len(SMALL), dt, 40 + nrhs)
    outs = M.apply_batched(small, fs, precision=precision)
    for F, f, g in zip(small, fs, outs):
        ref = F.apply(f, precision=precision)
        assert torch.equal(g, ref)


def test_batch_mixed_nrhs_fp64(small):
    M = _mod()
    nr = [1, 2, 1, 5, 1, 3]
    fs = _inputs(nr, torch.complex128, 44)
    outs = M.apply_batched(small, fs, precision="fp64")
    for F, f, g in zip(small, fs, outs):
        ref = F.apply(f, precision="fp64")
        assert (torch.linalg.norm(g - ref) / torch.linalg.norm(ref)).item() < 1e-13


def test_batch_matches_direct_sum(small):
    M = _mod()
    fs_np = [W.complex_gaussian(n * n, 1, 45, j) for j, (n, _) in enumerate(SMALL)]
    fs = [to_dev(f, torch.complex128).reshape(-1) for f in fs_np]
    outs = M.apply_batched(small, fs, precision="fp64")
    for (n, ph), f, g in zip(SMALL, fs_np, outs):
        ref = direct_sum(Kernel(2, n, ph), f)
        assert rel_l2(g.cpu().numpy()[:, None], ref) < 1e-5


def test_batch_shared_handle_equals_individual_applies(small):
    """Transforms given one handle (their segments interleaved in the queue) each equal their own apply."""
    M = _mod()
    F = small[3]                                   # 128^2, linear phase
    n = SMALL[3][0]
    fs = [to_dev(W.complex_gaussian(n * n, 1, 49, j), torch.complex128).reshape(-1) for j in range(5)]
    extra = _inputs([1] * 6, torch.complex128, 50)[0]
    outs = M.apply_batched([F] * 5 + [small[0]], fs + [extra], precision="fp64")
    for c in range(5):
        assert torch.equal(outs[c], F.apply(fs[c], precision="fp64")), c
    assert torch.equal(outs[5], small[0].apply(extra, precision="fp64"))


def test_batch_graph_replays_follow_inputs(small):
    """Replays of the captured graph, with eager work between them, each equal the eager applies."""
    M = _mod()
    fs = _inputs([1] * len(SMALL), torch.complex64, 46)
    B = M.Batch(small, fs, precision="fp32", graph=True)
    st = B.stats()
    assert st["graph"] == 1 and st["stages"] == sum(2 * F.stats()["b"] + 1 for F in small)
    assert st["rounds"] == max(2 * F.stats()["b"] + 1 for F in small)
    assert st["launches"] == 1 and st["workgroups"] >= 1
    for rep in range(4):
        for f in fs:
            f.mul_(1.5 - 0.25j)          # eager work on the inputs between replays
        torch.cuda.synchronize()
        outs = B.run()
        torch.cuda.synchronize()
        for F, f, g in zip(small, fs, outs):
            assert torch.equal(g, F.apply(f, precision="fp32")), rep
        torch.cuda.synchronize()
    assert B.stats()["timeouts"] == 0
    B.close()


def test_batch_direct_launch_equals_graph(small):
    M = _mod()
    fs = _inputs([1] * len(SMALL), torch.complex64, 47)
    Bg = M.Batch(small, fs, precision="fp32", graph=True)
    Bd = M.Batch(small, fs, precision="fp32", graph=False)
    og = [g.clone() for g in Bg.run()]
    torch.cuda.synchronize()
    od = Bd.run()
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(og, od))
    assert Bd.stats()["graph"] == 0


def test_batch_errors(small):
    M = _mod()
    from paper_1908_09376_amd._lib import MidbfError
    fs = _inputs([1] * len(SMALL), torch.complex64, 48)
    with pytest.raises(MidbfError, match="UNIMPLEMENTED"):
        M.apply_batched(small, fs, precision="bf16x3")
    with pytest.raises(MidbfError, match="ERR_ARG"):
        M.Batch([], [], precision="fp32")
    with pytest.raises(ValueError):
        M.apply_batched(small, fs, outs=[torch.empty(3, dtype=torch.complex64, device=DEV)] * len(fs),
                        precision="fp32")


def test_uneven_batch_of_32_transforms():
    """The uneven batch: 32 transforms with N in {64^2, 128^2, 256^2}, one RHS each, FP32."""
    M = _mod()
    ns = W.batch_sizes(32)
    cache = {}
    Fs = []
    for n in ns:
        if int(n) not in cache:
            cache[int(n)] = M.MIDBF(2, int(n), "fio_ellipse", tol=1e-6, precisions=2 | 1)
        Fs.append(cache[int(n)])
    fs_np = [W.batch_rhs(j, int(n)) for j, n in enumerate(ns)]
    fs = [to_dev(f, torch.complex64).reshape(-1) for f in fs_np]
    B = M.Batch(Fs, fs, precision="fp32", graph=True)
    for rep in range(3):                 # the queue resets itself between runs
        outs = B.run()
        torch.cuda.synchronize()
        for j, (F, f, g) in enumerate(zip(Fs, fs, outs)):
            assert torch.equal(g, F.apply(f, precision="fp32")), (rep, j)
    st = B.stats()
    assert st["timeouts"] == 0 and st["launches"] == 1
    # against the FP64 definition on seeded sampled rows of three transforms (one per size)
    for n in sorted(cache):
        j = int(np.nonzero(ns == n)[0][0])
        rows = W.sample_rows(n * n, 2, 64)
        ref = direct_sum(Kernel(2, n, "fio_ellipse"), fs_np[j], rows=rows)
        got = outs[j].to(torch.complex128).cpu().numpy()[rows][:, None]
        assert rel_l2(got, ref) < 1e-5, (n, rel_l2(got, ref))
    B.close()
