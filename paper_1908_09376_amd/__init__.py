"""MI355X-native MIDBF: multidimensional interpolative decomposition butterfly
factorization (Chen, Zhang, Ho, Yang) in hand-written HIP for gfx950.

The library (libmidbf.so, C interface in include/midbf.h) builds the factors
on the GPU (FP64 kernel entries and batched column-pivoted QR interpolative
decompositions) and applies g = K f and f = K^H g level by level.

The binding is loaded on first use, so that `build_lib` can run before the
library exists.
"""
_EXPORTS = ("MIDBF", "ApplyGraph", "Batch", "apply_batched", "id_batch", "kernel_entries", "phase_recover",
            "recovery_path")


def __getattr__(name):
    if name in _EXPORTS:
        from . import midbf
        return getattr(midbf, name)
    if name == "midbf_matvec":
        from .autograd import midbf_matvec
        return midbf_matvec
    raise AttributeError(name)
