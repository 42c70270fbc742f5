"""CPU oracle for the MIDBF hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 NumPy/SciPy implementation of what the GPU library
computes, written from the paper (Chen, Zhang, Ho, Yang, "Multidimensional
phase recovery and interpolative decomposition butterfly factorization").
Only the tests, the package's smoke check and the benchmark's CPU-baseline
leg may import it.  It shares no code with the HIP library and never imports
it; the product path must not route through it.

Modules
  kernel   -- lattices, phase functions, kernel entries, the direct sum (eq. 1)
              and the FFT closed form for Phi = x . xi.
  midbf    -- the plain CPU MIDBF: trees (Sec. 3.1), linear-scaling ID
              (Sec. 3.2), LRCS / MSCS / recursive MSCS (Sec. 3.3-3.5) and the
              apply of the factor product, its adjoint and densification.
  phase    -- phase recovery (Sec. 2): RecoveryVector2 (Alg. 4), recovery
              paths (Alg. 5), Partition2, RecoveryMatrix2 (Alg. 6),
              randomized SVD (Alg. 1) and LowRankFactorization (Alg. 7).
  metrics  -- the error measures of Section 4.

Parity status (each function's docstring names its pins):
  every function is pinned by a test under tests/ against closed forms,
  brute force or worked examples, except where a docstring says
  "parity unpinned".
"""
