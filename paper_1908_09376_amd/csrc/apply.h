// Level kernels of the apply: argument blocks and launch entry.
#pragma once

#include "plan.h"

namespace midbf {

constexpr int APPLY_RT = 8;     // right-hand sides per workgroup, multi-RHS FP32 VALU path
constexpr int APPLY_RT64 = 4;   // the same for FP64

struct ApplyGeom {
    int d, n, P, L, leaf, n0;
};

constexpr int MAX_P = 8;        // P = 2^d children per node, d <= 3

// Ranks and previous-level-buffer offsets of the P child pieces that make up
// the candidate vector of group (a, partner) at step s >= 1.  The loads are
// issued together, so the P round trips overlap.
__device__ inline void child_pieces(int (&len)[MAX_P], long long (&off)[MAX_P], int P, long long a,
                                    long long partner, long long Ps, const int* k_prev,
                                    const long long* yoff_prev) {
#pragma unroll
    for (int t = 0; t < MAX_P; ++t) {
        if (t < P) {
            const long long idp = ((long long)P * a + t) * Ps + partner;
            len[t] = k_prev[idp];
            off[t] = yoff_prev[idp];
        }
    }
}

// Range guard of the split 16-bit applies.  fp16 holds |x| < 65504 ~ 2^16
// and keeps a lo part's full precision only for |x| >~ 2^-3 (its normal range
// starts at 2^-14), so the vectors an apply splits are held in HBM scaled by
// powers of two, which is exact in both directions:
//   - every vector v of the apply's chain (the input copy, the up levels' y,
//     the middle's and down levels' z) stores v * 2^(h_v - cexp[r]) for
//     right-hand side r, where cexp[r] is the binary exponent of max |f(:, r)|
//     (max = m 2^cexp, 1/2 <= m < 1), taken from the input once per apply;
//   - entries of v are (interpolated) sums over the p_v lattice points of the
//     column node they belong to of unit-modulus kernel entries times f, so
//     |v| <= p_v max |f(:, r)| up to the decompositions' interpolation growth
//     (the l1 norms of the up side's composed rows measure below 0.2 p_v),
//     and h_v <= SPLIT16_HEADROOM - ceil(log2 p_v) keeps the scaled entries
//     below 2^SPLIT16_HEADROOM, a factor 8 under 65504, while typical entries
//     (~ sqrt(p_v) max|f| / 5) stay well above 2^-3;
//   - a kernel whose output copies input rows (up: y = y_skel + T y_red; down:
//     skeleton rows, sibling sums) keeps its input's scale, so consecutive
//     vectors joined by such kernels share one h (the smallest bound among
//     them); the middle kernels (pure products, also the dense down blocks)
//     change it by a uniform power of two applied while staging
//     (MidArgs::bscale);
//   - only the copies at the ends touch per-column scales: the input copy
//     (TransposeIn or the leaf copy) multiplies by 2^(h - cexp[r]), the output
//     transpose by 2^(cexp[r] - h).
// cexp == null: no scaling.
struct SplitScale {
    const int* cexp;
    int hs;
};
constexpr int SPLIT16_HEADROOM = 13;

// 2^(hs - cexp[r]) (dir = +1) or its inverse (dir = -1); the exponent is
// clamped to +-100, so both are normal FP32 values.  1 without scaling.
__device__ inline float split_scale_of(const SplitScale& sc, int r, int dir) {
    if (!sc.cexp) return 1.f;
    const int e = max(-100, min(100, dir * (sc.hs - sc.cexp[r])));
    return __int_as_float((e + 127) << 23);
}

// Tables of one level (one step, one side) as seen by a kernel.
struct LevelArgs {
    const int* k;
    const int* n;
    const long long* perm_off;
    const int* perm;
    const long long* y_off;
    const void* const* T;    // per-ID factor block of the precision in use
    const int* src;          // split 16-bit up side: input row of every candidate position, or null
    const int* slot;         // scattered points: leaf slot table of this side's tree (point or -1), or null
};

struct UpArgs {
    ApplyGeom G;
    LevelArgs lev;
    int s;
    long long Ps;            // P^s
    const void* ext;         // s == 0: external input block (column-major, ld)
    long long ld;
    const void* in;          // s >= 1: previous level buffer
    const int* k_prev;
    const long long* yoff_prev;
    void* out;               // this level's buffer
    int nrhs;
    int ncand_max;           // largest candidate count of the level (LDS strip size)
    int nred_max;            // bound on the redundant inputs n - k of the level's decompositions
    int lattice_in;          // 1: `in` is the row-major input copy and lev.src holds lattice points
                             // (only the source-row-table kernels accept it)
    SplitScale sc;           // split 16-bit leaf copy: scale of the copied input (SplitScale)
    float presplit;          // split 16-bit top up step: > 0 writes its output already split, times
                             // this power of two, for the middle (MidArgs::presplit); 0: FP32 pairs
};

struct DownArgs {
    ApplyGeom G;
    LevelArgs lev;
    int s;
    long long Ps;
    const void* in;          // this level's buffer
    void* ext;               // s == 0: external output block
    long long ld;
    void* out;               // s >= 1: previous level buffer
    const int* k_prev;
    const long long* yoff_prev;
    int nrhs;
    int ncand_max;
    int kmax;                // largest rank of the level
};

struct MidArgs {
    const int* nr;
    const int* nc;
    const long long* off;
    const void* S;
    int pieces;
    const long long* in_off;
    const int* in_len;
    const long long* out_off;
    const int* out_len;
    const void* in;
    void* out;
    int nrhs;
    int in_max, out_max;     // largest column / row count of a block (matrix-core index tables)
    int chunk;               // VALU path: input entries staged in LDS per pass
    int mchunks;             // matrix-core FP32 path: workgroups splitting the rows of one block
    const int* ang;          // split 16-bit: the blocks' phase tiles (see mfma.h), or null
    float bscale;            // split 16-bit: power of two applied to the input while staging (SplitScale)
    int presplit;            // split 16-bit: the input was written already split and scaled by the top
                             // up step (per entry hi(re) | hi(im) << 16, then lo(re) | lo(im) << 16,
                             // in the 8 bytes of an FP32 pair), so staging only moves halves
};

// Input and output row numbers of middle block bi (the concatenations of its
// pieces in the level buffers) written to LDS; pieces <= MAX_P, and the piece
// tables are loaded together.
template <int NT>
__device__ inline void middle_rows(int* crow_in, int* crow_out, const MidArgs& A, long long bi) {
    long long oi[MAX_P], oo[MAX_P];
    int li[MAX_P], lo[MAX_P];
#pragma unroll
    for (int t = 0; t < MAX_P; ++t) {
        if (t < A.pieces) {
            oi[t] = A.in_off[bi * A.pieces + t];
            oo[t] = A.out_off[bi * A.pieces + t];
            li[t] = A.in_len[bi * A.pieces + t];
            lo[t] = A.out_len[bi * A.pieces + t];
        }
    }
    int s_in = 0, s_out = 0;
#pragma unroll
    for (int t = 0; t < MAX_P; ++t) {
        if (t < A.pieces) {
            for (int c = threadIdx.x; c < li[t]; c += NT) crow_in[s_in + c] = (int)(oi[t] + c);
            for (int c = threadIdx.x; c < lo[t]; c += NT) crow_out[s_out + c] = (int)(oo[t] + c);
            s_in += li[t];
            s_out += lo[t];
        }
    }
}

enum class LevelKernel { Up, Down, Middle, AdjUp, AdjMiddle, AdjDown, DownSum, Transpose, DownGroup, DownDense,
                         UpLeafCopy, DownLeaf, TransposeIn, ColExp };

// The per right-hand side exponents of SplitScale: blocks (b, r) write the
// largest |re| or |im| of slice b of column r of the external complex64 block
// to part[r * S + b]; then one block reduces each column's S slice maxima and
// writes cexp[r] (0 for a zero or non-finite column).
struct ColExpArgs {
    const void* src;
    long long ld, N;
    int nrhs, S;
    float* part;
    int* cexp;
};

// Block transpose between a row-major N x nrhs copy (element (p, r) at
// [p * nrhs + r]) and the external column-major layout (element (p, r) at
// [r * ld + p]): Transpose writes the external block from the copy (src
// row-major), TransposeIn the copy from the external block (src column-major).
struct TransposeArgs {
    const void* src;
    void* dst;
    long long ld;
    long long N;
    int nrhs;
    SplitScale sc;           // complex64: TransposeIn multiplies by 2^(hs - cexp[r]), Transpose by 2^(cexp[r] - hs)
};

void launch_level_kernel(LevelKernel which, int prec, int rt, const void* args, dim3 grid, size_t smem,
                         hipStream_t s);

// A batch of forward transforms as one persistent launch.  Each level launch
// of each transform is a stage; its tasks (one per workgroup of that launch)
// are handed out in segments of up to a chunk of consecutive items, in queue
// order: level by level, and within a level the transforms that share a
// factorization item block by item block, so that their segments reading the
// same factor blocks are handed out together.  A segment waits until its
// transform's previous level (stage dep) has completed all its items.
struct BatchStage {
    int kind;                // 0 up, 1 middle, 2 down (forward transform)
    int tiles;               // right-hand-side tiles per group
    long long items;         // tasks: groups (or middle blocks) x tiles
    int dep;                 // stage of the same transform's previous level, or -1
    union {
        UpArgs up;
        MidArgs mid;
        DownArgs down;
    } a;
};

struct BatchSegment {
    int stage;
    int count;               // items item0 .. item0 + count - 1 of the stage
    long long item0;
};

// Control block of a persistent run, 32-bit words: next segment to hand out,
// workgroups finished, waits that hit the spin limit (kept across runs), one
// spare, then one completion count per stage.  The last workgroup of a run
// clears every word but the timeout count for the next run.
constexpr int BATCH_CTL_HEAD = 4;

struct PersistArgs {
    const BatchStage* st;
    const BatchSegment* seg;
    int nseg;
    unsigned* ctl;
    int nst;
    long long spin_limit;    // polls of a dependency before a wait is abandoned (counted as a timeout)
};

// Workgroups of the persistent kernel that fit on the current device at once
// (occupancy x compute units) with `smem` bytes of dynamic LDS.
int persistent_capacity(int prec, int rt, size_t smem);
void launch_persistent(int prec, int rt, const PersistArgs& P, int grid, size_t smem, hipStream_t s);

}  // namespace midbf
