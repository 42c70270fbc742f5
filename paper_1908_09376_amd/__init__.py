"""MI355X-native MIDBF: multidimensional interpolative decomposition butterfly
factorization (Chen, Zhang, Ho, Yang) in hand-written HIP for gfx950.

The library (libmidbf.so, C interface in include/midbf.h) builds the factors
on the GPU (FP64 kernel entries and batched column-pivoted QR interpolative
decompositions) and applies g = K f and f = K^H g level by level.
"""
from .midbf import MIDBF, apply_batched, id_batch, kernel_entries  # noqa: F401
