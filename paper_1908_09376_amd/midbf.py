"""Python front end of the MIDBF library: the C calls with torch tensors.

Vectors are torch CUDA tensors of shape (N,) or (nrhs, N) (each right-hand
side contiguous = column-major N x nrhs with ld = N): complex128 for the
FP64 apply, complex64 for FP32 and split-BF16.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

from . import _lib as L


def _stream_ptr(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _params(d, n, phase, tol, leaf_box, oversample_t, k_cap, U=None, V=None, precisions=0,
            workspace_bytes=0, fixed_rank=0, points=None, helmholtz_h=0.0, adjoint=False) -> L.Params:
    p = L.Params()
    p.d, p.n, p.tol = d, n, tol
    p.leaf_box, p.oversample_t, p.k_cap = leaf_box, oversample_t, k_cap
    p.phase = L.PHASES[phase]
    p.U_dev = U.data_ptr() if U is not None else None
    p.V_dev = V.data_ptr() if V is not None else None
    p.r = U.shape[1] if U is not None else 0
    p.precisions = precisions
    p.build_workspace_bytes = workspace_bytes
    p.fixed_rank = fixed_rank
    if points is not None:
        p.x_points = points[0].data_ptr()
        p.xi_points = points[1].data_ptr()
        p.n_points = points[0].shape[0]
    p.helmholtz_h = helmholtz_h
    p.adjoint = 1 if adjoint else 0
    return p


_PREC = {"fp64": L.FP64, "fp32": L.FP32, "bf16x3": L.SPLIT_BF16, "fp16x3": L.SPLIT_FP16}


class MIDBF:
    """A built factorization K ~ U^L...U^h S V^h...V^L (midbf_build); with adjoint=True a factorization
    of K^H, whose apply computes K^H g in every kept precision."""

    def __init__(self, d: int, n: int, phase: str, tol: float = 1e-6, leaf_box: int = 8,
                 oversample_t: int = 5, k_cap: int = 0, U: torch.Tensor | None = None,
                 V: torch.Tensor | None = None, precisions: int = 0, workspace_bytes: int = 0,
                 fixed_rank: int = 0, points=None, helmholtz_h: float = 0.0, adjoint: bool = False,
                 stream=None):
        self.d, self.n, self.N = d, n, n ** d
        self.adjoint = bool(adjoint)
        if phase == "lowrank":
            U = U.to(torch.float64).contiguous()
            V = V.to(torch.float64).contiguous()
        if points is not None:
            # scattered points: two N x d FP64 sets (N = n^d unless given by their length); n then
            # only sets the tree depth
            points = tuple(t.to(torch.float64).contiguous() for t in points)
            self.N = points[0].shape[0]
            for t in points:
                if not t.is_cuda or t.dim() != 2 or t.shape != (self.N, d):
                    raise ValueError("points: two CUDA tensors of the same shape (N, d)")
        self._UV = (U, V, points)    # kept alive: the library reads them during the build
        self._p = _params(d, n, phase, tol, leaf_box, oversample_t, k_cap, U, V, precisions,
                          workspace_bytes, fixed_rank, points, helmholtz_h, adjoint)
        h = C.c_void_p()
        L.check(L.lib.midbf_build(C.byref(self._p), _stream_ptr(stream), C.byref(h)))
        self._h = h

    def save(self, path: str, stream=None) -> None:
        """Write the factorization to a file (midbf_save; needs the FP64 copy)."""
        L.check(L.lib.midbf_save(self._h, os.fsencode(path), _stream_ptr(stream)))

    @classmethod
    def load(cls, path: str, precisions: int = 0, stream=None) -> "MIDBF":
        """A factorization read from a file written by save (midbf_load), keeping `precisions`."""
        p = L.Params()
        h = C.c_void_p()
        L.check(L.lib.midbf_load(os.fsencode(path), precisions, _stream_ptr(stream), C.byref(p), C.byref(h)))
        self = cls.__new__(cls)
        self.d, self.n, self.N = p.d, p.n, p.n ** p.d
        self.adjoint = False                  # factor files hold forward factorizations
        self._UV = (None, None)
        self._p = p
        self._h = h
        return self

    def close(self):
        if getattr(self, "_h", None):
            L.lib.midbf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- apply ------------------------------------------------------------
    def _prep(self, x: torch.Tensor, precision: str):
        want = torch.complex128 if precision == "fp64" else torch.complex64
        if x.dtype != want or not x.is_cuda or not x.is_contiguous():
            raise TypeError(f"expected a contiguous CUDA {want} tensor")
        if x.shape[-1] != self.N or x.dim() > 2:
            raise ValueError("expected shape (N,) or (nrhs, N)")
        return (1 if x.dim() == 1 else x.shape[0])

    def _out(self, x: torch.Tensor, out: torch.Tensor | None) -> torch.Tensor:
        """The output block: a new tensor like x, or the caller's, checked against x before any launch."""
        if out is None:
            return torch.empty_like(x)
        if out.dtype != x.dtype or not out.is_cuda or not out.is_contiguous():
            raise TypeError(f"out must be a contiguous CUDA {x.dtype} tensor")
        if out.shape != x.shape or out.device != x.device:
            raise ValueError("out must have the input's shape and device")
        return out

    def apply(self, f: torch.Tensor, out: torch.Tensor | None = None, precision: str = "fp64",
              stream=None) -> torch.Tensor:
        """g = K f (midbf_apply)."""
        nrhs = self._prep(f, precision)
        g = self._out(f, out)
        L.check(L.lib.midbf_apply(self._h, f.data_ptr(), g.data_ptr(), nrhs, self.N, _PREC[precision],
                                  _stream_ptr(stream)))
        return g

    def apply_noalloc(self, f: torch.Tensor, out: torch.Tensor | None = None, precision: str = "fp64",
                      stream=None) -> torch.Tensor:
        """g = K f with the library's static device scratch instead of a workspace (midbf_apply_noalloc)."""
        nrhs = self._prep(f, precision)
        g = self._out(f, out)
        L.check(L.lib.midbf_apply_noalloc(self._h, f.data_ptr(), g.data_ptr(), nrhs, self.N, _PREC[precision],
                                          _stream_ptr(stream)))
        return g

    def apply_adjoint(self, g: torch.Tensor, out: torch.Tensor | None = None, precision: str = "fp64",
                      stream=None) -> torch.Tensor:
        """f = K^H g (midbf_apply_adjoint)."""
        nrhs = self._prep(g, precision)
        f = self._out(g, out)
        L.check(L.lib.midbf_apply_adjoint(self._h, g.data_ptr(), f.data_ptr(), nrhs, self.N,
                                          _PREC[precision], _stream_ptr(stream)))
        return f

    # -- inspection ---------------------------------------------------------
    def stats(self) -> dict:
        s = L.Stats()
        L.check(L.lib.midbf_factor_stats(self._h, C.byref(s)))
        return {name: getattr(s, name) for name, _ in L.Stats._fields_}

    def tune(self, nrhs: int, precision: str = "fp32", stream=None) -> list[int]:
        """Pick the fastest matrix-core tile variants for nrhs right-hand sides (midbf_tune)."""
        out = (C.c_int * 3)()
        L.check(L.lib.midbf_tune(self._h, nrhs, _PREC[precision], _stream_ptr(stream), out))
        return list(out)

    def set_variants(self, variants, precision: str = "fp32") -> None:
        arr = (C.c_int * 3)(*variants)
        L.check(L.lib.midbf_set_variants(self._h, _PREC[precision], arr))

    def profile(self, on: bool = True, by_level: bool = False) -> None:
        """Bracket every level-kernel launch with HIP events (midbf_profile_enable)."""
        L.check(L.lib.midbf_profile_enable(self._h, (2 if by_level else 1) if on else 0))

    def profile_read(self) -> list[dict]:
        """Per-kernel launches, total ms, algorithmic bytes and flops since the last read."""
        buf = (L.KernelTime * 64)()
        cnt = C.c_int()
        L.check(L.lib.midbf_profile_read(self._h, buf, 64, C.byref(cnt)))
        return [{"name": buf[i].name.decode(), "launches": buf[i].launches, "total_ms": buf[i].total_ms,
                 "bytes": buf[i].bytes, "flops": buf[i].flops, "stored_bytes": buf[i].stored_bytes}
                for i in range(min(cnt.value, 64))]

    def ranks(self, side: int, step: int) -> np.ndarray:
        st = self.stats()
        count = (2 ** self.d) ** (st["L"] + 1)
        out = np.zeros(count, dtype=np.int32)
        L.check(L.lib.midbf_ranks(self._h, side, step, out.ctypes.data_as(C.POINTER(C.c_int)), count))
        return out


def _batch_arrays(handles, fs, outs, precision):
    count = len(handles)
    if len(fs) != count or len(outs) != count:
        raise ValueError("one input and one output per handle")
    for f, g in zip(fs, outs):
        if g.shape != f.shape or g.dtype != f.dtype or not g.is_contiguous() or g.device != f.device:
            raise ValueError("each output must match its input's shape, dtype and device")
    hs = (C.c_void_p * count)(*[h._h for h in handles])
    fp = (C.c_void_p * count)(*[f.data_ptr() for f in fs])
    gp = (C.c_void_p * count)(*[g.data_ptr() for g in outs])
    nr = (C.c_int * count)(*[h._prep(f, precision) for h, f in zip(handles, fs)])
    return count, hs, fp, gp, nr


def apply_batched(handles: list[MIDBF], fs: list[torch.Tensor], outs: list[torch.Tensor] | None = None,
                  precision: str = "fp64", stream=None) -> list[torch.Tensor]:
    """g_j = K_j f_j for independent transforms in one persistent launch (midbf_apply_batched).

    Synchronizes the stream.
    """
    outs = [torch.empty_like(f) for f in fs] if outs is None else outs
    count, hs, fp, gp, nr = _batch_arrays(handles, fs, outs, precision)
    L.check(L.lib.midbf_apply_batched(count, hs, fp, gp, nr, _PREC[precision], _stream_ptr(stream)))
    return outs


class ApplyGraph:
    """g = K f for fixed buffers f, out, captured once in a hipGraph and replayed (midbf_apply_graph_*).

    The factorization and both tensors are referenced here and kept alive; the
    tile variants in effect at creation are fixed into the graph.
    """

    def __init__(self, F: MIDBF, f: torch.Tensor, out: torch.Tensor | None = None, precision: str = "fp32",
                 stream=None):
        nrhs = F._prep(f, precision)
        self.out = F._out(f, out)
        self._keep = (F, f, self.out)
        g = C.c_void_p()
        L.check(L.lib.midbf_apply_graph_create(F._h, f.data_ptr(), self.out.data_ptr(), nrhs, F.N,
                                               _PREC[precision], _stream_ptr(stream), C.byref(g)))
        self._g = g

    def launch(self, stream=None) -> torch.Tensor:
        L.check(L.lib.midbf_graph_launch(self._g, _stream_ptr(stream)))
        return self.out

    def close(self):
        if getattr(self, "_g", None):
            L.lib.midbf_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """A reusable batch g_j = K_j f_j of uneven transforms (midbf_batch_create / _run).

    One persistent launch per run: every level launch of every transform is a
    stage of one task queue, ordered by level, consumed by the workgroups that
    fit on the device at once.
    The handles and the tensors fs, outs are referenced by the batch and kept
    alive here; run() enqueues one replay (of the captured hipGraph when
    graph=True) on the stream.
    """

    def __init__(self, handles: list[MIDBF], fs: list[torch.Tensor], outs: list[torch.Tensor] | None = None,
                 precision: str = "fp32", graph: bool = True, stream=None):
        self.outs = [torch.empty_like(f) for f in fs] if outs is None else outs
        self._keep = (list(handles), list(fs), self.outs)
        count, hs, fp, gp, nr = _batch_arrays(handles, fs, self.outs, precision)
        b = C.c_void_p()
        L.check(L.lib.midbf_batch_create(count, hs, fp, gp, nr, _PREC[precision], 1 if graph else 0,
                                         _stream_ptr(stream), C.byref(b)))
        self._b = b

    def run(self, stream=None) -> list[torch.Tensor]:
        L.check(L.lib.midbf_batch_run(self._b, _stream_ptr(stream)))
        return self.outs

    def stats(self) -> dict:
        """Shape of the batch and the count of abandoned dependency waits (synchronizes the device)."""
        s = L.BatchStats()
        L.check(L.lib.midbf_batch_get_stats(self._b, C.byref(s)))
        return {name: getattr(s, name) for name, _ in L.BatchStats._fields_}

    def close(self):
        if getattr(self, "_b", None):
            L.lib.midbf_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kernel_entries(d: int, n: int, phase: str, rows: torch.Tensor, cols: torch.Tensor,
                   U: torch.Tensor | None = None, V: torch.Tensor | None = None, adjoint: bool = False,
                   stream=None) -> torch.Tensor:
    """K(rows, cols) (or K^H(rows, cols) with adjoint) as a complex128 (len(rows), len(cols)) tensor
    (midbf_kernel_entries)."""
    p = _params(d, n, phase, 1e-6, 1, 1, 0, U, V, adjoint=adjoint)
    rows = rows.to(torch.int32).contiguous()
    cols = cols.to(torch.int32).contiguous()
    out = torch.empty((rows.numel(), cols.numel()), dtype=torch.complex128, device=rows.device)
    L.check(L.lib.midbf_kernel_entries(C.byref(p), rows.data_ptr(), rows.numel(), cols.data_ptr(),
                                       cols.numel(), out.data_ptr(), _stream_ptr(stream)))
    return out


def id_batch(X: torch.Tensor, tol: float, k_cap: int = 0, stream=None):
    """Batched CPQR interpolative decomposition of X (batch, m, n) complex128 (midbf_id_batch).

    Returns (k (batch,), perm (batch, n), T list of (k_b, n-k_b) tensors).  X is overwritten.
    """
    b, m, n = X.shape
    k = torch.empty(b, dtype=torch.int32, device=X.device)
    perm = torch.empty((b, n), dtype=torch.int32, device=X.device)
    T = torch.empty((b, m * n), dtype=torch.complex128, device=X.device)
    L.check(L.lib.midbf_id_batch(X.data_ptr(), b, m, n, tol, k_cap, k.data_ptr(), perm.data_ptr(),
                                 T.data_ptr(), _stream_ptr(stream)))
    kk = k.cpu().numpy()
    Ts = [T[i, : kk[i] * (n - kk[i])].reshape(kk[i], n - kk[i]) for i in range(b)]
    return kk, perm.cpu().numpy(), Ts


def recovery_path(pts: np.ndarray, root: int = 0, stream=None) -> np.ndarray:
    """(N-1) x 2 recovery path (pred, node) of a point set (midbf_recovery_path, Alg. 5)."""
    a = np.ascontiguousarray(pts, dtype=np.float64)
    N, d = a.shape
    P = np.zeros((N - 1, 2), dtype=np.int32)
    L.check(L.lib.midbf_recovery_path(a.ctypes.data_as(C.POINTER(C.c_double)), N, d, root,
                                      P.ctypes.data_as(C.POINTER(C.c_int)), _stream_ptr(stream)))
    return P.astype(np.int64)


def phase_recover(d: int, n: int, sample, r: int = 8, q: int = 2, tau: float = 0.25, seed: int = 0,
                  X2: np.ndarray | None = None, stream=None, points=None):
    """[U, V] with exp(2 pi i U V^T) ~ K from rows / columns of K (phase_recover).

    sample(is_row, index) returns row `index` (is_row True) or column `index`
    of K as N complex values; it runs on the host when the library asks.
    Returns (U, V, info): (N, r) float64 CUDA tensors and a dict of the
    recovery's threshold, flagged nodes, accepted samples and integer shifts.
    """
    N = n ** d if points is None else len(points[0])
    dev = torch.device("cuda", torch.cuda.current_device())
    U = torch.empty((N, r), dtype=torch.float64, device=dev)
    V = torch.empty((N, r), dtype=torch.float64, device=dev)
    err = []

    def cb(_user, is_row, index, out):
        try:
            vals = np.asarray(sample(bool(is_row), int(index)), dtype=np.complex128).reshape(N)
            buf = np.ctypeslib.as_array(out, shape=(2 * N,))
            buf[0::2] = vals.real
            buf[1::2] = vals.imag
            return 0
        except Exception as e:          # reported after the call returns
            err.append(e)
            return 1

    cfun = L.SAMPLE_CB(cb)
    x2 = None
    if X2 is not None:
        x2a = np.ascontiguousarray(X2, dtype=np.float64).reshape(N, d)
        x2 = x2a.ctypes.data_as(C.POINTER(C.c_double))
    info = L.RecoverInfo()
    if points is not None:
        # scattered points (phase_recover_points): host coordinate copies for the paths and the fit
        xa = np.ascontiguousarray(points[0], dtype=np.float64).reshape(N, d)
        wa = np.ascontiguousarray(points[1], dtype=np.float64).reshape(N, d)
        st = L.lib.phase_recover_points(d, N, xa.ctypes.data_as(C.POINTER(C.c_double)),
                                        wa.ctypes.data_as(C.POINTER(C.c_double)), cfun, None, r, q, tau, seed,
                                        _stream_ptr(stream), U.data_ptr(), V.data_ptr(), C.byref(info))
    else:
        st = L.lib.phase_recover(d, n, None, x2, cfun, None, r, q, tau, seed, _stream_ptr(stream),
                                 U.data_ptr(), V.data_ptr(), C.byref(info))
    if err:
        raise err[0]
    L.check(st)
    nr, nc = info.n_rows, info.n_cols
    out = {"tau": info.tau, "disc_rows": info.disc_rows, "disc_cols": info.disc_cols,
           "disc_rows_initial": info.disc_rows_initial, "disc_cols_initial": info.disc_cols_initial,
           "rejected_rows": info.rejected_rows, "rejected_cols": info.rejected_cols,
           "callbacks": info.callbacks,
           "R": np.array(info.rows[:nr], dtype=np.int64), "C": np.array(info.cols[:nc], dtype=np.int64),
           "m": np.array([list(info.shift[a])[:d] for a in range(nr)], dtype=np.int64).reshape(nr, d),
           "a": np.array([info.shift[a][d] for a in range(nr)], dtype=np.int64)}
    return U, V, out
