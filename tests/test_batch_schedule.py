"""The persistent batch's queue protocol on host threads (CPU only, no GPU work).

midbf_schedule_simulate builds the batch's task queue with the library's own
builder and runs the protocol of the persistent kernel with host threads in
place of workgroups: take a segment of tasks from an atomic counter, wait for
the segment's transform to finish its previous level, count its tasks
complete.  With any number of workers, far fewer than segments included, and
with transforms of equal N interleaved (shared factorizations), every task
must complete with no stalled wait.
"""
import ctypes as C

import numpy as np
import pytest

import workloads as W


def _levels_items(ns, nrhs_tiles=1):
    """Level launches of a transform on an n x n lattice (leaf 8x8): b up levels and b down levels of
    P^L groups, and the middle's P*M blocks (L odd) or M blocks (L even)."""
    levels, items = [], []
    for n in ns:
        L = int(round(np.log2(n // 8)))
        b = (L + 1) // 2
        groups = 4 ** L
        middle = 4 ** (L + 1) // 4 ** (L % 2 == 0)
        seq = [groups] * b + [middle] + [groups] * b
        levels.append(len(seq))
        items.extend(x * nrhs_tiles for x in seq)
    return levels, items


def _simulate(levels, items, workers, chunk, seed=1, share=None):
    from paper_1908_09376_amd import _lib
    lv = (C.c_int * len(levels))(*levels)
    it = (C.c_longlong * len(items))(*items)
    sh = (C.c_int * len(levels))(*share) if share is not None else None
    done, stalls = C.c_longlong(), C.c_longlong()
    st = _lib.lib.midbf_schedule_simulate(len(levels), lv, it, sh, workers, chunk, 5000, seed, C.byref(done),
                                          C.byref(stalls))
    assert st == 0, _lib.lib.midbf_last_error()
    return done.value, stalls.value


@pytest.mark.parametrize("workers,chunk", [(1, 1), (3, 8), (8, 8), (37, 1), (256, 8)])
@pytest.mark.parametrize("shared", [False, True])
def test_uneven_batch_queue_completes(workers, chunk, shared):
    """The 32-transform batch; shared: transforms of equal N share one factorization (interleaved)."""
    ns = [int(n) for n in W.batch_sizes(32)]
    levels, items = _levels_items(ns)
    share = [ns.index(n) for n in ns] if shared else None
    done, stalls = _simulate(levels, items, workers, chunk, share=share)
    assert done == sum(items)
    assert stalls == 0


def test_more_workers_than_tasks_and_ragged_levels():
    levels = [1, 3, 5, 2]
    items = [1, 7, 2, 9, 3, 3, 1, 4, 1, 1, 2]
    done, stalls = _simulate(levels, items, workers=64, chunk=3, seed=7)
    assert done == sum(items) and stalls == 0


def test_simulation_rejects_bad_arguments():
    from paper_1908_09376_amd import _lib
    lv = (C.c_int * 1)(1)
    it = (C.c_longlong * 1)(5)
    d, s = C.c_longlong(), C.c_longlong()
    assert _lib.lib.midbf_schedule_simulate(1, lv, it, None, 0, 1, 100, 0, C.byref(d), C.byref(s)) == -1
    it0 = (C.c_longlong * 1)(0)           # a level launch without workgroups
    assert _lib.lib.midbf_schedule_simulate(1, lv, it0, None, 2, 1, 100, 0, C.byref(d), C.byref(s)) == -2
