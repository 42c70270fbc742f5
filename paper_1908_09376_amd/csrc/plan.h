// Host-side plan of a factorization: trees, per-step decomposition tables,
// factor storage and apply workspaces.
#pragma once

#include <string>
#include <utility>
#include <vector>

#include "common.h"
#include "phase.h"

namespace midbf {

enum { SIDE_ROW = 0, SIDE_COL = 1 };
enum { PREC_FP64 = 0, PREC_FP32 = 1, PREC_BF16 = 2, PREC_FP16 = 3, NPREC = 4 };

inline bool is_split16(int prec) { return prec == PREC_BF16 || prec == PREC_FP16; }

// One unrolled MSCS step of one side (Sec. 3.5): decompositions of the
// blocks (node at level la = L-s, partner at level lb = s+1), numbered
// id = node * P^lb + partner.
struct LevelSide {
    int s = 0, side = 0, la = 0, lb = 0;
    long long nid = 0;
    int m = 0;                            // samples per decomposition
    std::vector<int> k, n;                // rank and candidate count per ID
    std::vector<long long> perm_off, y_off;
    long long total_k = 0, total_n = 0, entries = 0, bf16_bytes = 0;   // bf16_bytes: one split-16 tile copy
    int kmin = 0, kmax = 0, nmax = 0;
    // device copies
    int* d_k = nullptr;
    int* d_n = nullptr;
    long long* d_perm_off = nullptr;
    long long* d_y_off = nullptr;
    int* d_perm = nullptr;                // candidate positions, skeleton first
    int* d_skel = nullptr;                // skeleton lattice point numbers at y_off
    // Split 16-bit, column side: for each candidate position p of an ID (perm
    // order, at perm_off), the row its input comes from: the lattice point at
    // s = 0, else the row of the previous level buffer.  Null: not built.
    int* d_src = nullptr;
    // The same table for s = 1 as lattice points, when the first step keeps
    // every leaf point (its y rows are copies of the input): the split up
    // kernels then read a row-major copy of the input directly.
    int* d_src_lat = nullptr;
    void** d_T[NPREC] = {};               // per-ID pointer to its T block
    // Split 16-bit, row side, s >= 1: per group of P siblings (IDs g P + t) the
    // dense candidate-order block [Pi_0 [I; T_0^T] ... Pi_{P-1} [I; T_{P-1}^T]]
    // (n x sum k) as fragment tiles, with piece tables in the middle's form:
    // inputs = the siblings' z vectors, outputs = the candidate rows (the
    // children's pieces of the previous level).  groups = 0: not built.
    long long groups = 0, g_tiles = 0, g_entries = 0;
    int g_nr_max = 0, g_nc_max = 0;
    int* d_g_nr = nullptr;
    int* d_g_nc = nullptr;
    long long* d_g_tile_off = nullptr;
    long long* d_g_in_off = nullptr;
    int* d_g_in_len = nullptr;
    long long* d_g_out_off = nullptr;
    int* d_g_out_len = nullptr;
    void* g_T[NPREC] = {};
    std::vector<void*> chunks;            // device allocations owned by this level
    // the FP64 T chunks (one per build wave, IDs in order) and their entry counts
    std::vector<std::pair<double2*, long long>> t64;
};

// Middle factor: one dense block per (row group, column group) pair.
struct Middle {
    long long nblk = 0;
    int pieces = 1;                       // 1 (L odd) or P (L even)
    std::vector<int> nr, nc;
    std::vector<long long> off;
    long long total = 0;
    int nr_max = 0, nc_max = 0;
    int* d_nr = nullptr;
    int* d_nc = nullptr;
    long long* d_off = nullptr;
    // per block and piece: vector offset/length of the column (input) and row (output) pieces
    long long* d_in_off = nullptr;
    int* d_in_len = nullptr;
    long long* d_out_off = nullptr;
    int* d_out_len = nullptr;
    void* S[NPREC] = {};                                // column-major blocks at off (split-16: fragment tiles)
    long long* d_tile_off = nullptr;                    // first bf16 tile of each block
    long long bf16_bytes = 0;
    void* ang = nullptr;                                // phase tiles of the blocks (split 16-bit applies)
    long long ang_bytes = 0;
};

struct Workspace {
    void* buf[2] = {nullptr, nullptr};
    size_t bytes = 0;
    void* scratch = nullptr;      // per-ID candidate contributions (matrix-core path going down)
    size_t scratch_bytes = 0;
    void* lat = nullptr;          // N x nrhs row-major copy of the output (matrix-core path)
    size_t lat_bytes = 0;
    void* aux = nullptr;          // split 16-bit: per right-hand side input maxima and exponents
    size_t aux_bytes = 0;
};

// Per-launch HIP-event timing of the apply kernels (midbf_profile_*).
struct ProfRecord {
    std::string name;
    hipEvent_t a, b;
    double bytes, flops;   // algorithmic bytes moved and flops of the launch
    double stored;         // bytes as laid out in memory (>= bytes: tile padding, identity entries)
};

struct Profiler {
    bool on = false;
    bool by_level = false;   // append the step index to kernel names
    std::vector<ProfRecord> recs;
    std::vector<hipEvent_t> pool;
};

}  // namespace midbf

struct midbf_plan {
    midbf_params p{};
    midbf::PhaseDesc ph{};
    int d = 0, n = 0, P = 0, L = 0, b = 0, hstar = 0, leaf = 0, n0 = 0;
    long long N = 0;
    std::vector<midbf::LevelSide> rows, cols;
    midbf::Middle mid;
    midbf::Workspace ws[midbf::NPREC];
    midbf_stats stats{};
    unsigned keep = 0;
    long long max_total_k = 0, max_total_n = 0;
    unsigned* d_tmax = nullptr;   // build only: largest |re|, |im| of the T entries packed into 16-bit tiles
    double* own_U = nullptr;      // low-rank phase: the plan's own copies of U and V (N x r)
    double* own_V = nullptr;
    // scattered points: own coordinate copies (x, xi; N x d) and, per side (row: the x tree,
    // column: the xi tree), the leaves' slot tables (leaf a, slot c < n0 -> point number, or -1
    // past the leaf's points) and the host trees (points leaf by leaf, leaf starts)
    bool points = false;
    double* own_xp = nullptr;
    double* own_wp = nullptr;
    int* d_slot[2] = {nullptr, nullptr};
    std::vector<double> tree_pts[2];      // coordinates in [0, 1)^d
    std::vector<int> tree_order[2];
    std::vector<long long> tree_start[2];
    int max_n = 0, max_k = 0;
    midbf::Profiler prof;
    // matrix-core tile variant per kernel kind (up, down, middle) and MSCS step (FP32, split-bf16, split-fp16)
    static constexpr int VMAXLEV = 16;
    int mfma_variant[3][VMAXLEV] = {};
    int mfma64_variant[3][VMAXLEV] = {};
    int bf16_variant[3][VMAXLEV] = {};
    int fp16_variant[3][VMAXLEV] = {};
};
