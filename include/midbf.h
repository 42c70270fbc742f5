/*
 * midbf.h -- C interface of the MI355X MIDBF library (libmidbf.so).
 *
 * The library evaluates the oscillatory transform
 *     g(x) = sum_{xi in Omega} exp(2 pi i Phi(x, xi)) f(xi),   x in X      (Section 1, eq. 1)
 * with the multidimensional interpolative decomposition butterfly
 * factorization (MIDBF, Section 3): K ~ U^L ... U^h S V^h ... V^L.
 *
 * Point sets.  X = {0..n-1}^d / n and Omega = {0..n-1}^d - n/2 (integers),
 * d = 2 or 3.  Points are numbered in C order (last coordinate fastest);
 * vectors f and g are indexed by these numbers.
 *
 * Conventions for every call:
 *   - Pointers named *_dev are device pointers (hipMalloc'ed or torch CUDA
 *     tensors); all other pointers are host pointers.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *     Applies are asynchronous on `stream`; build and phase_recover may
 *     synchronize it.
 *   - Complex vectors are interleaved (re, im): complex128 for MIDBF_FP64,
 *     complex64 for MIDBF_FP32, MIDBF_SPLIT_BF16 and MIDBF_SPLIT_FP16.  A block of nrhs vectors
 *     is column-major: element (point p, rhs r) at [r * ld + p], ld >= N.
 *   - No call throws; each returns a midbf_status and, on failure, leaves a
 *     message for midbf_last_error() (per thread).
 *   - The handle owns its device factors; the caller owns every buffer it
 *     passes.  Calls on one handle must not overlap on different streams.
 */
#ifndef MIDBF_H
#define MIDBF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct midbf_plan* midbf_handle;
typedef struct midbf_batch_s* midbf_batch;
typedef struct midbf_graph_s* midbf_graph;

typedef enum {
    MIDBF_OK = 0,
    MIDBF_ERR_ARG = -1,             /* invalid argument or null pointer            */
    MIDBF_ERR_SHAPE = -2,           /* sizes inconsistent (n not leaf * 2^L, ...)  */
    MIDBF_ERR_OOM = -3,             /* device allocation failed                    */
    MIDBF_ERR_RANK_SATURATED = -4,  /* an ID kept as many pivots as samples        */
    MIDBF_ERR_RECOVERY = -5,        /* phase recovery failed (tau schedule ran out) */
    MIDBF_ERR_HIP = -6,             /* a HIP runtime call failed                   */
    MIDBF_ERR_UNIMPLEMENTED = -7,
    MIDBF_ERR_IO = -8          /* a factor file could not be written or read, or is not one */
} midbf_status;

/* Phase functions (Scenario 1 of Table 1: O(1) entry access). */
typedef enum {
    MIDBF_PHASE_LINEAR = 0,        /* Phi = x . xi                                          */
    MIDBF_PHASE_FIO_ELLIPSE = 1,   /* Section 4, Example 1: x.xi + sqrt(c1^2 xi1^2 + c2^2 xi2^2),
                                      c1 = (2 + sin 2pi x1 sin 2pi x2)/16,
                                      c2 = (2 + cos 2pi x1 cos 2pi x2)/16  (d = 2)          */
    MIDBF_PHASE_FIO_PIECEWISE = 2, /* x.xi + c(x)|xi|, c = (2 + sin 2pi x1)/16 if x1 < 1/2,
                                      else (3 + cos 2pi x2)/16  (d = 2)                    */
    MIDBF_PHASE_ISO3D = 3,         /* x.xi + c(x)|xi|, c = (3 + prod_q sin 2pi x_q)/100 (d = 3) */
    MIDBF_PHASE_LOWRANK = 4,       /* Phi = U V^T from phase_recover (Section 2.3.5, Alg. 7) */
    MIDBF_PHASE_HELMHOLTZ = 5      /* Phi = h |x - xi|_2, scattered points only (Sec. 4, Example 3:
                                      the oscillatory part of the Helmholtz Green's function)     */
} midbf_phase_kind;

typedef enum {
    MIDBF_FP64 = 0,          /* FP64 factors and arithmetic                              */
    MIDBF_FP32 = 1,          /* FP32 factors, FP32 accumulation                          */
    MIDBF_SPLIT_BF16 = 2,    /* factors and inputs split into bf16 hi + lo, three bf16
                                products per real product, FP32 accumulation (MFMA)      */
    MIDBF_SPLIT_FP16 = 3     /* the same with fp16 hi + lo: ~2^-22 per split value.  fp16
                                holds |x| < 65504: the library keeps every vector it splits
                                scaled by a power of two per right-hand side (exact), taken
                                from max |f| of that column and the points behind each entry,
                                so any finite input works; the build refuses an fp16 copy
                                whose factor entries reach 2^15 (midbf_stats.t_abs_max)    */
} midbf_precision;

/* Bits of midbf_params.precisions: which factor copies the build keeps.  A
 * split copy (BF16 or FP16) holds the factors as MFMA fragment tiles, plus,
 * for the down steps above the leaves, one dense block per group of 2^d
 * sibling decompositions; the middle factor is also kept once as its phases
 * (4 bytes per entry, shared by both split types).  Factors are built in FP64
 * and rounded once into each kept copy. */
#define MIDBF_KEEP_FP64 1u
#define MIDBF_KEEP_FP32 2u
#define MIDBF_KEEP_BF16 4u
#define MIDBF_KEEP_FP16 8u

typedef struct {
    int d;               /* 2 or 3                                                     */
    int n;               /* points per dimension; n = leaf_box * 2^L with L >= 1        */
    double tol;          /* ID tolerance epsilon of the rank rule (Sec. 3.5), e.g. 1e-6 */
    int leaf_box;        /* leaf side in points, n0 = leaf_box^d (paper: 8)            */
    int oversample_t;    /* t of the linear-scaling ID: t*k samples (Sec. 3.2; paper 5) */
    int k_cap;           /* rank cap per ID; 0 = no cap beyond min(samples, candidates) */
    midbf_phase_kind phase;
    const double* U_dev; /* MIDBF_PHASE_LOWRANK: N x r row-major FP64 (x side)          */
    const double* V_dev; /* MIDBF_PHASE_LOWRANK: N x r row-major FP64 (xi side)         */
    int r;               /* rank of U V^T                                               */
    unsigned precisions; /* MIDBF_KEEP_* bits; 0 = FP64, FP32 and split-bf16            */
    size_t build_workspace_bytes; /* cap on transient build memory; 0 = 48 GiB          */
    int fixed_rank;      /* > 0: the fixed-rank variant (Sec. 3.5, closing paragraph):
                            every ID keeps min(fixed_rank, samples, candidates) columns
                            whatever tol says, so each level's ranks are known before
                            the build; 0: the adaptive rank rule with tol                */
    const double* x_points;  /* scattered points (Sec. 3.5, closing paragraph; Sec. 4 Ex. 2):
                                N = n^d points x, N x d row-major FP64, device            */
    const double* xi_points; /* and N frequencies xi, the same layout.  Both set: each set
                                is moved and scaled uniformly into [0, 1]^d by its bounding
                                cube and partitioned on the boxes of the n^d lattice's tree
                                (depth log2(n / leaf_box)); a node without points holds
                                none, leaves hold uneven counts.  Phase
                                MIDBF_PHASE_LINEAR (Phi = x . xi on the given coordinates),
                                MIDBF_PHASE_HELMHOLTZ or MIDBF_PHASE_LOWRANK (U, V rows per
                                point).  Vectors are
                                indexed by point number.  FP64 and FP32 copies only.  Both
                                null: the lattices {0..n-1}^d / n and {0..n-1}^d - n/2      */
    long long n_points;      /* scattered points: N, the size of each set (0: n^d); n then
                                only sets the tree depth log2(n / leaf_box)                */
    double helmholtz_h;      /* MIDBF_PHASE_HELMHOLTZ: h                                    */
    int adjoint;             /* nonzero: factor K^H instead of K, i.e. the kernel
                                conj(K(x, xi)) with the xi points as rows and the x points
                                as columns (the same trees, the phase negated and its
                                arguments swapped), so that midbf_apply computes K^H g in
                                every kept precision, the split 16-bit ones included.  This
                                is a factorization of K^H to the tolerance, not the exact
                                conjugate transpose of a forward factorization (that is
                                midbf_apply_adjoint, FP64 and FP32).  Factor files hold
                                forward factorizations only.                                */
} midbf_params;

typedef struct {
    int L, b, hstar;            /* tree depth, MSCS steps, level of the last IDs        */
    long long ids;              /* interpolative decompositions performed              */
    long long entries;          /* complex entries stored (T blocks plus middle)       */
    long long bytes_fp64, bytes_fp32, bytes_bf16;  /* bytes of each factor copy        */
    long long index_bytes;      /* permutation and offset tables read by an apply      */
    int k_min, k_max;           /* ranks over all IDs                                  */
    double build_seconds;       /* wall time of midbf_build                            */
    long long bytes_fp16;       /* bytes of the split-fp16 factor copy                 */
    double t_abs_max;           /* largest |Re| or |Im| of an interpolation coefficient
                                   (entry of T) in the 16-bit copies; 0 without them   */
    double id_ms;               /* HIP-event time of the batched ID launches            */
    double id_flops;            /* sum over IDs of 8 m n k (m samples, n candidates,
                                   k rank): the column-pivoted QR's real flops          */
    double id_bytes;            /* sum over IDs of 16 m n: each complex FP64 sample
                                   matrix read once                                     */
} midbf_stats;

/*
 * midbf_build -- factor K = (exp(2 pi i Phi(x, xi))) on the lattices
 * (Sections 3.1-3.5): Z-ordered trees, then for steps s = 0..b-1 (b = ceil(L/2))
 * batched interpolative decompositions of every block (row node at level L-s,
 * column node at level s+1) and its transpose, from Mock-Chebyshev samples
 * with FP64 column-pivoted QR and the adaptive rank rule
 * k = #{j : |R_jj| > tol |R_11|}; then the middle factor from the last skeletons.
 * Runs on the GPU of the current device; synchronizes `stream`.
 * Errors: MIDBF_ERR_ARG / _SHAPE for bad params, _OOM, _RANK_SATURATED if
 * doubling the samples could not lift a saturated ID, _HIP.
 */
midbf_status midbf_build(const midbf_params* p, void* stream, midbf_handle* out);

/*
 * midbf_save -- write the factorization to `path` so that a later run skips the build
 * (the build costs far more than an apply: T_fac against T_app in Table 2).  The file holds
 * the parameters, for the low-rank phase U and V, and per step and side the sample count,
 * the candidate count, rank and pivot order of every decomposition and its FP64 T block
 * (Sec. 3.2: V = [I T] Pi^T); the middle factor and every other precision are derived from
 * these on loading.  Needs the FP64 copy (MIDBF_KEEP_FP64).  Synchronizes `stream`.
 * Little-endian binary; not portable across format versions (the magic carries the version).
 * Errors: MIDBF_ERR_ARG (null argument, no FP64 copy), MIDBF_ERR_IO (cannot write), _HIP.
 */
midbf_status midbf_save(midbf_handle h, const char* path, void* stream);

/*
 * midbf_load -- rebuild a factorization from a file written by midbf_save, keeping the
 * `precisions` copies (MIDBF_KEEP_* bits, 0 = the midbf_build default).  The decompositions
 * are read instead of computed; the packing, the middle factor and the split tiles are made
 * as in midbf_build, so every apply equals the saved handle's bit for bit.  params_out
 * (may be null) receives the parameters (U_dev, V_dev then point at the handle's own copies).
 * The whole header is checked before the device is touched, and every record before it is
 * used (counts, ranks, pivot orders are permutations).
 * Errors: MIDBF_ERR_IO (cannot open, not a factor file, truncated or inconsistent), the
 * midbf_build errors.
 */
midbf_status midbf_load(const char* path, unsigned precisions, void* stream, midbf_params* params_out,
                        midbf_handle* out);

/*
 * midbf_apply -- g = K~ f for nrhs right-hand sides (the factor product of
 * Sec. 3.5 applied right to left).  f_dev, g_dev: N x nrhs column-major with
 * leading dimension ld (complex128 for MIDBF_FP64, complex64 otherwise).
 * The precision's factor copy must have been kept.  Workspace for nrhs is
 * allocated on the first call with that many right-hand sides.  Errors:
 * MIDBF_ERR_ARG for a null handle or vector, nrhs < 1, ld < N, or a
 * precision whose copy was not kept; nothing is launched then.
 */
midbf_status midbf_apply(midbf_handle h, const void* f_dev, void* g_dev, int nrhs, long long ld,
                         midbf_precision prec, void* stream);

/* Bytes of device scratch behind midbf_apply_noalloc (per GPU, held by the
 * library from the first such call on that GPU until the process ends). */
#define MIDBF_NOALLOC_SCRATCH_BYTES (64u << 20)

/*
 * midbf_apply_noalloc -- midbf_apply for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, layouts, kernels and results as
 * midbf_apply; the level vectors (and, on the matrix-core paths, the
 * lattice-order copy and the down pass's contribution block) live in one static
 * device array of MIDBF_NOALLOC_SCRATCH_BYTES per GPU instead of the handle's
 * workspace.  No hipMalloc, hipFree or other allocating call is made, and no
 * profiler events are taken (a handle's profiler records nothing for it).
 * Nothing in the scratch needs to start at zero: every element a kernel reads
 * was written earlier in the same call.
 * Limit: 2 * max_level_rows * nrhs * c, plus N * nrhs * c on the matrix-core
 * paths with nrhs > 1 (the lattice copy), plus max_candidate_rows * nrhs * c
 * where the matrix-core down pass writes per-decomposition contributions
 * (FP32 and FP64 matrix cores, split tile variants 0-4), each part rounded
 * up to 256, with c = 16 (FP64) or 8; larger applies return MIDBF_ERR_SHAPE
 * with the size needed (one right-hand side at N = 256^2 needs ~8 MB).
 * Concurrency: every call on one GPU shares that GPU's array, so calls that
 * overlap on one GPU (different streams or threads) race; serialize them.
 * Errors: as midbf_apply, plus MIDBF_ERR_SHAPE beyond the limit and
 * MIDBF_ERR_HIP if the scratch's device address cannot be obtained.
 */
midbf_status midbf_apply_noalloc(midbf_handle h, const void* f_dev, void* g_dev, int nrhs, long long ld,
                                 midbf_precision prec, void* stream);

/*
 * midbf_apply_graph_create -- capture the launch sequence of
 * midbf_apply(h, f_dev, g_dev, nrhs, ld, prec) into a hipGraph (the many-RHS
 * apply of Sec. 3.5's factor product, replayed without host launch overhead).
 * The handle's workspace for nrhs right-hand sides is allocated before the
 * capture, and the tile variants in effect now (midbf_tune,
 * midbf_set_variants) are fixed into the graph.  The graph refers to f_dev,
 * g_dev and the handle's factors and workspace: they must outlive it, and a
 * replay must not overlap another apply of the same handle and precision.
 * Synchronizes `stream`.  Errors: as midbf_apply; MIDBF_ERR_HIP if capture
 * or instantiation fails.
 * midbf_graph_launch enqueues one replay on `stream` (asynchronous);
 * midbf_graph_destroy releases the graph (not the buffers).
 */
midbf_status midbf_apply_graph_create(midbf_handle h, const void* f_dev, void* g_dev, int nrhs, long long ld,
                                      midbf_precision prec, void* stream, midbf_graph* out);
midbf_status midbf_graph_launch(midbf_graph g, void* stream);
void midbf_graph_destroy(midbf_graph g);

/*
 * midbf_apply_adjoint -- f = K~^H g: conjugate-transposed factors in reverse
 * order (the transposed butterfly).  Same layouts as midbf_apply.  FP64 and
 * FP32 (matrix cores from 16 right-hand sides); a split 16-bit precision is
 * refused with MIDBF_ERR_UNIMPLEMENTED (K^H in those comes from a handle
 * built with midbf_params.adjoint, applied with midbf_apply).
 */
midbf_status midbf_apply_adjoint(midbf_handle h, const void* g_dev, void* f_dev, int nrhs, long long ld,
                                 midbf_precision prec, void* stream);

/*
 * midbf_apply_batched -- count independent transforms (different handles,
 * possibly different N): g_j = K~_j f_j as one persistent launch
 * (midbf_batch_create + midbf_batch_run, then destroy; the call therefore
 * synchronizes `stream`).  hs, f_devs, g_devs, nrhs are
 * host arrays of length count; each f/g block is column-major with ld = N_j.
 * FP64 or FP32.
 */
midbf_status midbf_apply_batched(int count, const midbf_handle* hs, const void* const* f_devs,
                                 void* const* g_devs, const int* nrhs, midbf_precision prec,
                                 void* stream);

/*
 * Batches of forward transforms of uneven N (the batched apply of many
 * transforms; the factor product of Sec. 3.5 per transform).
 *
 * midbf_batch_create -- prepare g_j = K~_j f_j for j < count as ONE
 * persistent launch per run.  The workgroups of every level launch of every
 * transform become tasks of one queue, ordered by level (every transform's
 * first level, then every second level, ...).  As many workgroups as fit on
 * the device at once take tasks in queue order with an atomic counter; a
 * task waits until its transform's previous level has completed (a
 * completion count per level, release / acquire at device scope), runs the
 * level kernel's body, and counts itself complete.  Tasks depend only on
 * earlier tasks, so the earliest unfinished one can always proceed: no
 * deadlock, whatever the number of resident workgroups.  Waits poll with a
 * bounded count; one that runs out is abandoned and counted
 * (midbf_batch_stats.timeouts) instead of hanging.  The last workgroup of a
 * run resets the queue for the next run, so a run is a single kernel node
 * (graph replays need no reset).  Tasks are handed out in segments of a few
 * consecutive workgroups; within a level, the segments of transforms given
 * the same handle are interleaved block by block, so segments that read the
 * same factor blocks run at about the same time and the repeated reads hit
 * the caches.  Each output equals midbf_apply of its own transform.
 * hs, f_devs, g_devs, nrhs: host arrays of
 * length count; f/g blocks column-major with ld = N_j; FP64 (complex128) or
 * FP32 (complex64), through the VALU level kernels.  use_graph != 0 captures
 * the launches in a hipGraph at creation; midbf_batch_run replays it.  The
 * batch owns its level buffers and references the handles and the f/g
 * buffers, which must outlive it.  Runs of one batch must not overlap.
 * Errors: _ARG, _UNIMPLEMENTED (split-bf16, or candidate vectors beyond the
 * LDS budget), _OOM, _HIP.
 */
typedef struct {
    int stages;                 /* level launches folded into the batch              */
    int rounds;                 /* levels of the deepest transform                   */
    long long items;            /* tasks (level-launch workgroups) of one run        */
    int graph;                  /* 1 if replayed from a captured hipGraph            */
    long long lds_bytes;        /* dynamic LDS per workgroup                         */
    double bytes, flops;        /* algorithmic bytes and flops of one run            */
    int launches;               /* kernel launches per run (1)                       */
    int workgroups;             /* persistent workgroups (resident capacity)         */
    long long timeouts;         /* dependency waits abandoned at the poll limit, over
                                   all runs so far (0 in a correct run)              */
} midbf_batch_stats;

midbf_status midbf_batch_create(int count, const midbf_handle* hs, const void* const* f_devs,
                                void* const* g_devs, const int* nrhs, midbf_precision prec,
                                int use_graph, void* stream, midbf_batch* out);
/* Enqueue one run of the batch on `stream` (asynchronous). */
midbf_status midbf_batch_run(midbf_batch b, void* stream);
/* Synchronizes the device (it reads the timeout count). */
midbf_status midbf_batch_get_stats(midbf_batch b, midbf_batch_stats* out);

/*
 * midbf_schedule_simulate -- host check of the persistent batch's queue
 * protocol (no GPU work): builds the queue of `count` transforms, transform j
 * having levels[j] level launches with the task counts given in order in
 * items (sum of levels[] entries) and sharing group share[j] (transforms of
 * one group are interleaved; NULL: none shared), in segments of `chunk`
 * tasks, and runs the protocol with `workers` host threads in place of
 * workgroups (any number, also fewer than segments), each segment pausing at
 * random.  A dependency wait longer than limit_ms counts as a stall.  Outputs
 * the tasks completed and the stalls.  Errors: MIDBF_ERR_ARG, MIDBF_ERR_SHAPE
 * (a level launch without tasks).
 */
midbf_status midbf_schedule_simulate(int count, const int* levels, const long long* items, const int* share,
                                     int workers, int chunk, int limit_ms, unsigned seed, long long* completed,
                                     long long* stalls);
/* Free the batch; waits for the device like hipFree. */
void midbf_batch_destroy(midbf_batch b);

/*
 * Phase recovery (Section 2; Scenario 2 of Table 1: K is reachable only
 * through O(1) of its rows and columns).
 *
 * midbf_sample_cb -- the caller's sampler: write row `index` (is_row != 0,
 * K(x_index, :)) or column `index` (K(:, xi_index)) of K as N complex128
 * values (interleaved re, im) to the host buffer `out`; return 0 on success.
 */
typedef int (*midbf_sample_cb)(void* user, int is_row, long long index, double* out);

#define PHASE_RECOVER_MAX_SAMPLES 64

typedef struct {
    double tau;                    /* discontinuity threshold after the schedule (Sec. 2.3.4) */
    int disc_rows, disc_cols;      /* flagged nodes on the root column / root row            */
    int n_rows, n_cols;            /* accepted sampled rows / columns                        */
    int rejected_rows, rejected_cols;
    long long callbacks;           /* rows and columns fetched through the sampler           */
    long long rows[PHASE_RECOVER_MAX_SAMPLES], cols[PHASE_RECOVER_MAX_SAMPLES];
    int shift[PHASE_RECOVER_MAX_SAMPLES][4];   /* per accepted row: integer m (d entries), a  */
    int disc_rows_initial, disc_cols_initial;  /* flagged nodes at the initial tau, before the
                                                  schedule raises it (Table 4's counts)        */
} phase_recover_info;

/*
 * phase_recover -- a real N x r pair (U, V) with exp(2 pi i U V^T) ~ K
 * (Alg. 7: RecoveryMatrix2 (Alg. 6, built on Alg. 4 along recovery paths),
 * then the randomized SVD of Alg. 1), for the lattices of this library:
 * x = {0..n-1}^d / n, xi = {0..n-1}^d - n/2.  The recovery paths are the
 * dimension-ordered comb trees rooted at x = 0 and xi = 0.  X1, X2: host
 * N x d row-major coordinates of the x and xi points, or NULL for the
 * lattice coordinates (X2 enters the integer-shift fit below).
 *
 * The GPU form is Alg. 7 with branch reconciliation, for phases whose steps
 * along rows exceed the unwrap limit of Alg. 4 on an integer frequency
 * lattice: a recovered row or column is used only if every path step inside
 * its block stays below 0.4 in magnitude; each accepted row is fitted
 * against the accepted sampled columns by an integer shift m . xi + a (kept
 * only if the fit is exact) and shifted; Alg. 1 takes its pivots and extra
 * rows / columns inside the accepted samples.  Samples are drawn in
 * splitmix64-seeded orders (sorted by splitmix64(seed + 2 i + stream),
 * stream 0 rows, 1 columns), the discontinuity nodes first.  Inside the
 * regime of Lemma 2.2 nothing is rejected and every shift is zero.
 *
 * r: rank (1..16); q: oversampling, r*q <= 32 rows and columns are sampled;
 * tau: initial discontinuity threshold (1/4; raised by 1/40 while more than
 * 16 nodes are flagged, up to 1/2).  U_dev, V_dev: caller-owned device
 * buffers of N x r FP64, row-major (the layout of midbf_params.U_dev / V_dev).
 * info may be NULL.  Synchronizes `stream`.
 * Errors: _ARG, _RECOVERY (the sampler failed, or too few rows / columns
 * passed the screening), _OOM, _HIP.
 */
midbf_status phase_recover(int d, int n, const double* X1, const double* X2, midbf_sample_cb cb, void* user,
                           int r, int q, double tau, uint64_t seed, void* stream, double* U_dev,
                           double* V_dev, phase_recover_info* info);

/*
 * phase_recover_points -- phase_recover for scattered point sets (Sec. 3.5,
 * closing paragraph; Sec. 4 Example 2): X1 and X2 are the host N x d row-major
 * coordinates of the x and xi points (both required).  The recovery paths are
 * those of midbf_recovery_path rooted at point 0 of each set; flagged nodes are
 * taken in path order; everything else is phase_recover's.
 * Errors: as phase_recover.
 */
midbf_status phase_recover_points(int d, long long N, const double* X1, const double* X2, midbf_sample_cb cb,
                                  void* user, int r, int q, double tau, uint64_t seed, void* stream, double* U_dev,
                                  double* V_dev, phase_recover_info* info);

/*
 * midbf_recovery_path -- the recovery path of a point set (Alg. 5, Def. 2.3):
 * the minimum spanning tree of the Euclidean distances (the Delaunay graph
 * the paper builds first holds every edge of it, so the tree is the same),
 * computed on the device by Prim's algorithm (ties to the smaller point
 * number), then a breadth-first order from `root` with neighbours visited by
 * increasing number.  pts: host N x d row-major coordinates (d = 2 or 3);
 * P_out: host (N - 1) x 2 int32, row t = (predecessor, node), in
 * non-decreasing depth.  Synchronizes `stream`.  Errors: _ARG, _OOM, _HIP.
 */
midbf_status midbf_recovery_path(const double* pts, long long N, int d, long long root, int* P_out, void* stream);

/* Sizes and ranks of a built factorization. */
midbf_status midbf_factor_stats(midbf_handle h, midbf_stats* out);

/*
 * midbf_ranks -- copy the ranks of step `step` (0..b-1) of side `side`
 * (0 = row IDs / U factors, 1 = column IDs / V factors) into out[0..count).
 * IDs are numbered node * P^(step+1) + partner.
 */
midbf_status midbf_ranks(midbf_handle h, int side, int step, int* out, long long count);

/*
 * midbf_kernel_entries -- out_dev[i * ncols + j] = K(x_rows[i], xi_cols[j])
 * (complex128) for point numbers rows_dev[0..nrows) and cols_dev[0..ncols),
 * with the phase of p (Sec. 3 preamble: entry evaluation from Phi in FP64,
 * reduced mod 1 before the exponential); with p->adjoint set, the entries of
 * K^H instead, conj(K(x_cols[j], xi_rows[i])).
 */
midbf_status midbf_kernel_entries(const midbf_params* p, const int* rows_dev, int nrows,
                                  const int* cols_dev, int ncols, void* out_dev, void* stream);

/*
 * midbf_id_batch -- the batched FP64 interpolative decomposition on caller
 * matrices (Sec. 3.2 with the rank rule of Sec. 3.5): for b = 0..batch-1,
 * X_b = X_dev + b*m*n (m x n, row-major complex128, overwritten) is
 * factored as X_b[:, perm] ~ X_b[:, perm[:k]] [I T].  Outputs: k_dev[b],
 * perm_dev[b*n + j] (0-based column numbers, skeleton first) and
 * T_dev + b*m*n holding T (k x (n-k), row-major, leading dimension n-k).
 * Constraint: m <= 4096, n <= 2048.
 */
midbf_status midbf_id_batch(void* X_dev, int batch, int m, int n, double tol, int k_cap,
                            int* k_dev, int* perm_dev, void* T_dev, void* stream);

/*
 * Per-kernel timing of the applies (the paper's T_app, Sec. 4, split by
 * kernel).  With profiling enabled, every level-kernel launch of
 * midbf_apply / midbf_apply_adjoint is bracketed by HIP events on the
 * apply's stream.  midbf_profile_read synchronizes those events and
 * aggregates by kernel name: launches, total milliseconds, and the
 * algorithmic bytes (factor entries once, index tables, input and output
 * vectors) and flops (8 per complex multiply-add) of those launches.  It
 * writes up to max_entries records, sets *count to the number of distinct
 * kernels, and clears the records.  on = 2 also splits each kernel by MSCS
 * step (names end in _s<step>).
 */
typedef struct {
    char name[48];
    long long launches;
    double total_ms;
    double bytes;
    double flops;
    double stored_bytes;   /* the same traffic as laid out: tile padding and the identity
                              entries of dense blocks included (>= bytes) */
} midbf_kernel_time;

midbf_status midbf_profile_enable(midbf_handle h, int on);
midbf_status midbf_profile_read(midbf_handle h, midbf_kernel_time* out, int max_entries, int* count);

/*
 * midbf_tune -- autotuner of the many-right-hand-side (matrix-core) apply:
 * times every tile variant (rows per wave, K chunk, pipelining, workgroup
 * width) of the up, down and middle kernels on this factorization with nrhs
 * right-hand sides and keeps the fastest per kernel kind and MSCS step
 * (one warm-up apply per variant, then the faster of two timed applies).
 * Allocates and frees two N x nrhs buffers; synchronizes `stream`.  If
 * variants != NULL, writes the choice for the top step of up and down and
 * for the middle to variants[0..3).  midbf_set_variants installs one variant
 * per kind for every step (MIDBF_ERR_ARG for an unknown precision or a
 * variant out of range: FP32 0-9, FP64 0-4, split 16-bit 0-10).  nrhs below
 * the matrix-core threshold leaves the choice unchanged.  FP64, FP32,
 * MIDBF_SPLIT_BF16 and MIDBF_SPLIT_FP16 keep separate choices.  For the split
 * applies, variants 7-10 of the up kind read per-level source-row tables
 * built with the plan; when the first up step keeps every leaf point, they
 * also replace that step by the (scaled) transpose of the input into the
 * apply's row-major copy.  When the top up step and the middle both run
 * variants 7-10, the up step writes its output already split into hi / lo
 * halves for the middle (the same conversions, so the result is bitwise the
 * same); the environment variable MIDBF_SPLIT_EXCHANGE=0, read when an apply
 * is planned, keeps FP32 pairs instead.
 */
midbf_status midbf_tune(midbf_handle h, int nrhs, midbf_precision prec, void* stream, int* variants);
midbf_status midbf_set_variants(midbf_handle h, midbf_precision prec, const int* variants);

/* Release the factorization and its workspaces. */
void midbf_destroy(midbf_handle h);

/* Message of the last failed call on this thread ("" if none). */
const char* midbf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MIDBF_H */
