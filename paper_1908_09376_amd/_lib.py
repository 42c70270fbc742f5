"""ctypes binding of libmidbf.so (include/midbf.h): argument marshalling only.

Every computation runs in the library's HIP kernels; PyTorch supplies device
memory and the stream.  Importing this module fails loudly if the library
has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmidbf.so")

MIDBF_OK = 0
STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_SHAPE", -3: "ERR_OOM", -4: "ERR_RANK_SATURATED",
          -5: "ERR_RECOVERY", -6: "ERR_HIP", -7: "ERR_UNIMPLEMENTED", -8: "ERR_IO"}

PHASES = {"linear": 0, "fio_ellipse": 1, "fio_piecewise": 2, "iso3d": 3, "lowrank": 4, "helmholtz": 5}
FP64, FP32, SPLIT_BF16, SPLIT_FP16 = 0, 1, 2, 3
KEEP_FP64, KEEP_FP32, KEEP_BF16, KEEP_FP16 = 1, 2, 4, 8


class Params(C.Structure):
    _fields_ = [("d", C.c_int), ("n", C.c_int), ("tol", C.c_double), ("leaf_box", C.c_int),
                ("oversample_t", C.c_int), ("k_cap", C.c_int), ("phase", C.c_int),
                ("U_dev", C.c_void_p), ("V_dev", C.c_void_p), ("r", C.c_int),
                ("precisions", C.c_uint), ("build_workspace_bytes", C.c_size_t), ("fixed_rank", C.c_int),
                ("x_points", C.c_void_p), ("xi_points", C.c_void_p), ("n_points", C.c_longlong),
                ("helmholtz_h", C.c_double), ("adjoint", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("L", C.c_int), ("b", C.c_int), ("hstar", C.c_int), ("ids", C.c_longlong),
                ("entries", C.c_longlong), ("bytes_fp64", C.c_longlong), ("bytes_fp32", C.c_longlong),
                ("bytes_bf16", C.c_longlong), ("index_bytes", C.c_longlong), ("k_min", C.c_int),
                ("k_max", C.c_int), ("build_seconds", C.c_double), ("bytes_fp16", C.c_longlong),
                ("t_abs_max", C.c_double), ("id_ms", C.c_double), ("id_flops", C.c_double),
                ("id_bytes", C.c_double)]


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_longlong), ("total_ms", C.c_double),
                ("bytes", C.c_double), ("flops", C.c_double), ("stored_bytes", C.c_double)]


class BatchStats(C.Structure):
    _fields_ = [("stages", C.c_int), ("rounds", C.c_int), ("items", C.c_longlong), ("graph", C.c_int),
                ("lds_bytes", C.c_longlong), ("bytes", C.c_double), ("flops", C.c_double),
                ("launches", C.c_int), ("workgroups", C.c_int), ("timeouts", C.c_longlong)]


class RecoverInfo(C.Structure):
    _fields_ = [("tau", C.c_double), ("disc_rows", C.c_int), ("disc_cols", C.c_int), ("n_rows", C.c_int),
                ("n_cols", C.c_int), ("rejected_rows", C.c_int), ("rejected_cols", C.c_int),
                ("callbacks", C.c_longlong), ("rows", C.c_longlong * 64), ("cols", C.c_longlong * 64),
                ("shift", (C.c_int * 4) * 64), ("disc_rows_initial", C.c_int), ("disc_cols_initial", C.c_int)]


NOALLOC_SCRATCH_BYTES = 64 << 20   # MIDBF_NOALLOC_SCRATCH_BYTES

SAMPLE_CB = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.c_longlong, C.POINTER(C.c_double))


class MidbfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1908_09376_amd.build_lib` (no CPU fallback exists)")
    lib = C.CDLL(LIB_PATH)
    vp, i, ll = C.c_void_p, C.c_int, C.c_longlong
    sig = {
        "midbf_build": (i, [C.POINTER(Params), vp, C.POINTER(vp)]),
        "midbf_save": (i, [vp, C.c_char_p, vp]),
        "midbf_load": (i, [C.c_char_p, C.c_uint, vp, C.POINTER(Params), C.POINTER(vp)]),
        "midbf_apply": (i, [vp, vp, vp, i, ll, i, vp]),
        "midbf_apply_adjoint": (i, [vp, vp, vp, i, ll, i, vp]),
        "midbf_apply_noalloc": (i, [vp, vp, vp, i, ll, i, vp]),
        "midbf_apply_graph_create": (i, [vp, vp, vp, i, ll, i, vp, C.POINTER(vp)]),
        "midbf_graph_launch": (i, [vp, vp]),
        "midbf_graph_destroy": (None, [vp]),
        "midbf_apply_batched": (i, [i, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(i), i, vp]),
        "midbf_batch_create": (i, [i, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(i), i, i, vp,
                                   C.POINTER(vp)]),
        "midbf_batch_run": (i, [vp, vp]),
        "midbf_batch_get_stats": (i, [vp, C.POINTER(BatchStats)]),
        "midbf_batch_destroy": (None, [vp]),
        "midbf_schedule_simulate": (i, [i, C.POINTER(i), C.POINTER(ll), C.POINTER(i), i, i, i, C.c_uint,
                                        C.POINTER(ll), C.POINTER(ll)]),
        "midbf_factor_stats": (i, [vp, C.POINTER(Stats)]),
        "midbf_ranks": (i, [vp, i, i, C.POINTER(i), ll]),
        "midbf_kernel_entries": (i, [C.POINTER(Params), vp, i, vp, i, vp, vp]),
        "midbf_id_batch": (i, [vp, i, i, i, C.c_double, i, vp, vp, vp, vp]),
        "midbf_tune": (i, [vp, i, i, vp, C.POINTER(i)]),
        "midbf_set_variants": (i, [vp, i, C.POINTER(i)]),
        "midbf_profile_enable": (i, [vp, i]),
        "midbf_profile_read": (i, [vp, C.POINTER(KernelTime), i, C.POINTER(i)]),
        "phase_recover": (i, [i, i, C.POINTER(C.c_double), C.POINTER(C.c_double), SAMPLE_CB, vp, i, i, C.c_double,
                              C.c_uint64, vp, vp, vp, C.POINTER(RecoverInfo)]),
        "phase_recover_points": (i, [i, ll, C.POINTER(C.c_double), C.POINTER(C.c_double), SAMPLE_CB, vp, i, i,
                                     C.c_double, C.c_uint64, vp, vp, vp, C.POINTER(RecoverInfo)]),
        "midbf_recovery_path": (i, [C.POINTER(C.c_double), ll, i, ll, C.POINTER(C.c_int), vp]),
        "midbf_destroy": (None, [vp]),
        "midbf_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def check(status: int) -> None:
    if status != MIDBF_OK:
        raise MidbfError(status, lib.midbf_last_error().decode())


EXPORTED = ["midbf_build", "midbf_save", "midbf_load", "midbf_apply", "midbf_apply_adjoint", "midbf_apply_noalloc", "midbf_apply_batched",
            "midbf_apply_graph_create", "midbf_graph_launch", "midbf_graph_destroy",
            "midbf_batch_create", "midbf_batch_run", "midbf_batch_get_stats",
            "midbf_batch_destroy", "midbf_schedule_simulate",
            "midbf_factor_stats", "midbf_ranks", "midbf_kernel_entries", "midbf_id_batch",
            "midbf_tune", "midbf_set_variants", "midbf_profile_enable", "midbf_profile_read", "midbf_destroy", "midbf_last_error",
            "phase_recover", "phase_recover_points", "midbf_recovery_path"]
