// Matrix-core (MFMA) level kernels for many right-hand sides.
#pragma once

#include <algorithm>

#include "apply.h"

namespace midbf {

constexpr int MFMA_NRHS = 64;        // right-hand sides per workgroup
constexpr int MFMA_MIN_NRHS = 16;    // below this the VALU kernels are used
constexpr int MFMA_CROW_MAX = 4096;  // FP32: largest candidate vector / middle block side (LDS index tables)
constexpr int BF16_CROW_MAX = 2048;  // split-bf16: the same

constexpr int MFMA_VARIANTS = 10;     // tile variants (rows per wave, K chunk, pipelining)
constexpr int MFMA64_VARIANTS = 5;    // the same for FP64 (one row tile per wave)

// One matrix-core level kernel.  count = IDs (up, down), groups (down-sum) or
// middle blocks (each split over MidArgs::mchunks workgroups).  Going down, each ID writes its
// contribution to `scratch` (total_n x nrhs complex64) and the down-sum kernel
// adds the 2^d contributions of every group into the previous level buffer /
// external output.
void launch_mfma_kernel(LevelKernel which, int variant, const void* args, long long count, int nrhs, void* scratch,
                        hipStream_t s, bool fp64 = false);

// The external <-> row-major transposes around a matrix-core apply.
void launch_transpose(const TransposeArgs& A, bool fp64, hipStream_t s);
// The external column-major complex64 block -> the row-major copy (A.src external, A.dst the copy).
void launch_transpose_in(const TransposeArgs& A, hipStream_t s);
// SplitScale exponents of the input block (two launches, see ColExpArgs).
void launch_col_exponents(const ColExpArgs& A, hipStream_t s);
// Slices per column of the exponent pass (ColExpArgs::S; part holds nrhs * S floats).
inline int col_exp_slices(long long N) { return (int)std::min<long long>(64, (N + 4095) / 4096); }
// The first up step when every leaf decomposition keeps all its points (no T):
// per leaf, the caller's block is staged once and copied to the P partners'
// skeleton rows.  groups = leaves; complex64.
void launch_up_leaf_copy(const UpArgs& A, long long groups, int nrhs, hipStream_t s);

// Split 16-bit variants of the up / down / middle kernels (factors stored as
// MFMA fragment tiles; tile_off gives each middle block's first tile), for
// elem = SPLIT16_BF16 or SPLIT16_FP16.  DownDense runs the middle kernels on
// the group blocks of a down step (MidArgs; tile_off = their first tiles).
constexpr int BF16_VARIANTS = 11;
// Ranks up to which the split down kernels keep z in LDS (variants 5-9 then
// run the grouped down pass, LevelKernel::DownGroup).
constexpr int SPLIT16_RESIDENT_K = 256;
enum { SPLIT16_BF16 = 0, SPLIT16_FP16 = 1 };
void launch_bf16_kernel(int elem, LevelKernel which, int variant, const void* args, long long count, int nrhs,
                        void* scratch, const long long* tile_off, hipStream_t s);

// Fragment tiles (16 x 32, 4 KB each) of an M x K block.
long long bf16_tiles(int M, int K);
constexpr long long BF16_TILE_BYTES = 4096;
// Pack T of each decomposition of a build wave (FP64 slab) into tiles: the
// column side stores A = T (k x (n-k)), the row side (transposed = true) A = T^T.
// tmax (or null): atomic max of the entries' |re| and |im| as FP32 bits (the
// range of the 16-bit copies; |x| of a non-negative float orders like its bits).
void pack_bf16_slab(int elem, const double2* X, long long x_stride, const int* k_w, const int* n_w, int count,
                    bool transposed, void* out, const long long* tile_off, unsigned* tmax, hipStream_t s);
// Pack the dense candidate-order block of every group of P sibling row
// decompositions (one step, going down) from the siblings' own tiles; per group
// nr = n rows, nc = sum of k columns, first tile at tile_off.
// The input row of every candidate position of the IDs [0, nid) of one up
// level (LevelSide::d_src): candidate c of ID id is the lattice point c of its
// leaf at s = 0, else row c of the concatenated child pieces of the previous
// level; out[perm_off[id] + p] = row of candidate perm[perm_off[id] + p].
// Candidate sets up to BF16_CROW_MAX.
void pack_src_rows(const ApplyGeom& G, int s, long long Ps, const int* n, const long long* perm_off, const int* perm,
                   const int* k_prev, const long long* yoff_prev, long long nid, int* out, hipStream_t st);
// out[i] = skel[src[i]], i < count: a source-row table whose rows are y rows of
// a first up step that keeps every leaf point, turned into lattice points.
void pack_src_lattice(const int* skel, const int* src, long long count, int* out, hipStream_t st);
void pack_group_tiles(int elem, int P, const int* k, const long long* perm_off, const int* perm, void* const* T,
                      const int* nr, const int* nc, const long long* tile_off, long long groups, void* out,
                      hipStream_t s);
// The middle blocks K(rows, cols) = exp(2 pi i Phi) stored by their phases:
// per 16 x 32 tile, lane l holds the eight entries of row l % 16, columns
// 8 (l / 16) + i, as frac(Phi) - [frac(Phi) >= 1/2] in units of 2^-32 turns
// (int32, 32 B per lane, 2 KB per tile; tiles at the blocks' tile_off).
// pts: per block its nr row points, then its nc column points, at pts_off.
constexpr long long ANGLE_TILE_BYTES = 2048;
void pack_angle_tiles(const PhaseDesc& ph, const int* nr, const int* nc, const long long* pts_off, const int* pts,
                      const long long* tile_off, long long count, void* out, hipStream_t s);
// Pack column-major FP32 middle blocks into tiles.
void pack_bf16_blocks(int elem, const float2* S, const long long* s_off, const int* nr, const int* nc,
                      long long count, void* out, const long long* tile_off, hipStream_t s);

}  // namespace midbf
