// Apply orchestration and the C interface (include/midbf.h).
#include <algorithm>
#include <atomic>
#include <cctype>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>

#include "apply.h"
#include "build.h"
#include "mfma.h"
#include "recover.h"

// Device scratch of midbf_apply_noalloc: level vectors, the matrix-core down
// pass's contribution block and the lattice-order copy of one apply.  Each
// GPU the library runs on holds its own copy until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns for
// the current device (noalloc_scratch below), never through this name.
static __device__ __align__(256) unsigned char scratch[MIDBF_NOALLOC_SCRATCH_BYTES];

namespace midbf {

namespace {

thread_local std::string g_last_error;

midbf_status fail(midbf_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

template <class F> midbf_status guarded(F&& f) {
    try {
        f();
        return MIDBF_OK;
    } catch (const Error& e) {
        return fail(e.code, e.what());
    } catch (const std::bad_alloc&) {
        return fail(MIDBF_ERR_OOM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(MIDBF_ERR_HIP, e.what());
    }
}

int prec_index(midbf_precision p) {
    switch (p) {
        case MIDBF_FP64: return PREC_FP64;
        case MIDBF_FP32: return PREC_FP32;
        case MIDBF_SPLIT_BF16: return PREC_BF16;
        case MIDBF_SPLIT_FP16: return PREC_FP16;
    }
    throw Error(MIDBF_ERR_ARG, "unknown precision");
}

LevelArgs level_args(const LevelSide& lv, int prec) {
    return LevelArgs{lv.d_k, lv.d_n, lv.d_perm_off, lv.d_perm, lv.d_y_off, (const void* const*)lv.d_T[prec], lv.d_src,
                     nullptr};
}

LevelArgs level_args(const midbf_plan* h, const LevelSide& lv, int prec) {
    LevelArgs a = level_args(lv, prec);
    if (h->points) a.slot = h->d_slot[lv.side];
    return a;
}

size_t csize(int prec) { return prec == PREC_FP64 ? 16 : 8; }

constexpr size_t LDS_LIMIT = 64 * 1024;    // dynamic LDS of the VALU level kernels

const char* kernel_name(LevelKernel k) {
    switch (k) {
        case LevelKernel::Up: return "up";
        case LevelKernel::Down: return "down";
        case LevelKernel::Middle: return "middle";
        case LevelKernel::AdjUp: return "adj_up";
        case LevelKernel::AdjMiddle: return "adj_middle";
        case LevelKernel::AdjDown: return "adj_down";
        case LevelKernel::DownSum: return "down_sum";
        case LevelKernel::Transpose: return "transpose";
        case LevelKernel::DownGroup: return "down_group";
        case LevelKernel::DownDense: return "down_dense";
        case LevelKernel::UpLeafCopy: return "up_copy";
        case LevelKernel::DownLeaf: return "down_leaf";
        case LevelKernel::TransposeIn: return "transpose";
        case LevelKernel::ColExp: return "col_exp";
    }
    return "?";
}

hipEvent_t take_event(Profiler& P) {
    if (P.pool.empty()) {
        hipEvent_t e;
        MIDBF_HIP(hipEventCreate(&e));
        return e;
    }
    hipEvent_t e = P.pool.back();
    P.pool.pop_back();
    return e;
}

// Launch one level kernel; with profiling on, bracket it with events on the
// same stream and record its algorithmic bytes and flops.  mfma_count > 0
// selects the matrix-core kernel with that many workgroups in x.
void launch_checked(midbf_plan* h, const Workspace& ws, LevelKernel which, int prec, int rt, const void* args,
                    dim3 grid, size_t smem, hipStream_t st, double bytes, double flops, long long mfma_count = 0,
                    int nrhs = 0, int level = -1, bool profile = true, double stored = -1.0) {
    MIDBF_CHECK(mfma_count > 0 || smem <= LDS_LIMIT, MIDBF_ERR_UNIMPLEMENTED,
                "candidate vectors of this factorization exceed the apply kernels' LDS budget");
    auto go = [&] {
        if (which == LevelKernel::Transpose) {
            launch_transpose(*(const TransposeArgs*)args, prec == PREC_FP64, st);
            return;
        }
        if (which == LevelKernel::TransposeIn) {
            launch_transpose_in(*(const TransposeArgs*)args, st);
            return;
        }
        if (which == LevelKernel::ColExp) {
            launch_col_exponents(*(const ColExpArgs*)args, st);
            return;
        }
        if (which == LevelKernel::UpLeafCopy) {
            launch_up_leaf_copy(*(const UpArgs*)args, mfma_count, nrhs, st);
            return;
        }
        if (mfma_count > 0) {
            const int kind = (which == LevelKernel::Up || which == LevelKernel::AdjUp)           ? 0
                             : (which == LevelKernel::Middle || which == LevelKernel::AdjMiddle) ? 2
                                                                                                 : 1;
            const int lv = std::max(0, std::min(level, midbf_plan::VMAXLEV - 1));
            // (DownGroup and DownDense are split-16 only; DownDense runs the middle
            // kernels on the group blocks, whose first-tile table travels in MidArgs::off)
            if (is_split16(prec) && which != LevelKernel::DownSum) {
                const auto& var = prec == PREC_FP16 ? h->fp16_variant : h->bf16_variant;
                // the top up step and the middle exchange split vectors only when both run
                // source-table kernels (split variants 7-10); else both keep FP32 pairs
                const int top = std::max(0, std::min(h->b - 1, midbf_plan::VMAXLEV - 1));
                const bool xv = var[0][top] >= 7 && var[0][top] <= 10 && var[2][0] >= 7 && var[2][0] <= 10;
                const void* ka = args;
                UpArgs ua;
                MidArgs ma;
                if (which == LevelKernel::Up && ((const UpArgs*)args)->presplit > 0.f && !xv) {
                    ua = *(const UpArgs*)args;
                    ua.presplit = 0.f;
                    ka = &ua;
                }
                if (which == LevelKernel::Middle && ((const MidArgs*)args)->presplit && !xv) {
                    ma = *(const MidArgs*)args;
                    ma.presplit = 0;
                    ka = &ma;
                }
                launch_bf16_kernel(prec == PREC_FP16 ? SPLIT16_FP16 : SPLIT16_BF16, which, var[kind][lv], ka,
                                   mfma_count, nrhs, ws.scratch,
                                   which == LevelKernel::DownDense ? ((const MidArgs*)args)->off
                                                                   : h->mid.d_tile_off,
                                   st);
            }
            else
                launch_mfma_kernel(which, (prec == PREC_FP64 ? h->mfma64_variant : h->mfma_variant)[kind][lv], args,
                                   mfma_count, nrhs, ws.scratch, st, prec == PREC_FP64);
        }
        else launch_level_kernel(which, prec, rt, args, grid, smem, st);
    };
    Profiler& P = h->prof;
    if (!P.on || !profile) {
        go();
        return;
    }
    ProfRecord r;
    const char* pname = prec == PREC_FP64   ? "_fp64"
                        : prec == PREC_BF16 ? "_bf16x3"
                        : prec == PREC_FP16 ? "_fp16x3"
                                            : "_fp32";
    if (which == LevelKernel::Transpose || which == LevelKernel::TransposeIn || which == LevelKernel::ColExp) {
        r.name = std::string(kernel_name(which)) + pname;
        if (which == LevelKernel::TransposeIn) r.name += "_in";
        else if (which == LevelKernel::Transpose && P.by_level) r.name += "_out";
    } else {
        r.name = std::string(kernel_name(which)) + (mfma_count > 0 && !is_split16(prec) ? "_mfma" : "") + pname +
                 (mfma_count > 0 ? "" : "_rt" + std::to_string(rt));
        if (P.by_level && level >= 0) r.name += "_s" + std::to_string(level);
    }
    r.a = take_event(P);
    r.b = take_event(P);
    r.bytes = bytes;
    r.stored = stored < 0.0 ? bytes : stored;
    r.flops = flops;
    MIDBF_HIP(hipEventRecord(r.a, st));
    go();
    MIDBF_HIP(hipEventRecord(r.b, st));
    P.recs.push_back(r);
}

// Bytes of each workspace part an apply of nrhs right-hand sides needs: the
// two level-vector buffers (each), the matrix-core down pass's contribution
// block and the N x nrhs lattice-order copy.
struct WorkspaceNeed {
    size_t buf, scratch, lat, aux;
};

WorkspaceNeed workspace_need(const midbf_plan* h, int prec, int nrhs, bool scratch, bool lat) {
    WorkspaceNeed w;
    w.buf = (size_t)std::max<long long>(h->max_total_k, 1) * nrhs * csize(prec);
    w.scratch = scratch ? (size_t)std::max<long long>(h->max_total_n, 1) * nrhs * csize(prec) : 0;
    w.lat = lat ? (size_t)h->N * nrhs * csize(prec) : 0;
    // split 16-bit: slice maxima and exponents of the range guard (SplitScale)
    w.aux = is_split16(prec) ? (size_t)nrhs * (col_exp_slices(h->N) + 1) * 4 : 0;
    return w;
}

void ensure_workspace(midbf_plan* h, int prec, int nrhs, bool scratch, bool lat) {
    Workspace& w = h->ws[prec];
    const WorkspaceNeed need = workspace_need(h, prec, nrhs, scratch, lat);
    if (w.bytes < need.buf) {
        if (w.buf[0]) MIDBF_HIP(hipFree(w.buf[0]));
        if (w.buf[1]) MIDBF_HIP(hipFree(w.buf[1]));
        w.buf[0] = w.buf[1] = nullptr;
        w.bytes = 0;
        MIDBF_HIP(hipMalloc(&w.buf[0], need.buf));
        MIDBF_HIP(hipMalloc(&w.buf[1], need.buf));
        w.bytes = need.buf;
    }
    if (scratch && w.scratch_bytes < need.scratch) {
        if (w.scratch) MIDBF_HIP(hipFree(w.scratch));
        w.scratch = nullptr;
        w.scratch_bytes = 0;
        MIDBF_HIP(hipMalloc(&w.scratch, need.scratch));
        w.scratch_bytes = need.scratch;
    }
    if (lat && w.lat_bytes < need.lat) {
        if (w.lat) MIDBF_HIP(hipFree(w.lat));
        w.lat = nullptr;
        w.lat_bytes = 0;
        MIDBF_HIP(hipMalloc(&w.lat, need.lat));
        w.lat_bytes = need.lat;
    }
    if (need.aux && w.aux_bytes < need.aux) {
        if (w.aux) MIDBF_HIP(hipFree(w.aux));
        w.aux = nullptr;
        w.aux_bytes = 0;
        MIDBF_HIP(hipMalloc(&w.aux, need.aux));
        w.aux_bytes = need.aux;
    }
}

// One level launch of an apply: which kernel, its argument block, shape and
// the algorithmic bytes and flops it accounts for.
struct LaunchDesc {
    LevelKernel which;
    union {
        UpArgs up;
        MidArgs mid;
        DownArgs down;
        TransposeArgs tr;
        ColExpArgs ce;
    } a;
    dim3 grid;
    size_t smem;
    double bytes, flops;
    double stored;          // bytes as laid out (padded tiles, identity entries), if above `bytes`; else 0
    long long mfma_count;   // > 0: matrix-core kernel with that many workgroups
    int level;
};

// The launch sequence of one application of the factor product
// (adjoint = false) or of its conjugate transpose (adjoint = true), with the
// level vectors in bufs[0..1] (and the matrix-core down pass's per-ID
// contributions in scratch), rt right-hand sides per VALU workgroup.
// chunk_middle splits the middle into launches of at most 65535 blocks (grid
// limit of a direct launch).  With lat (N x nrhs), the last down-sum writes
// its rows there (row-major, lattice order: whole 512-byte rows instead of
// strided columns) and a final transpose writes the output block.  (The leaf
// up kernels read the input block directly: measured faster than a transpose
// in front of them.)
std::vector<LaunchDesc> plan_apply(midbf_plan* h, const void* in_ext, void* out_ext, int nrhs, long long ld, int prec,
                                   bool adjoint, bool mfma, void* const* buf, bool chunk_middle, int rt,
                                   void* lat = nullptr, void* aux = nullptr) {
    const double fl = is_split16(prec) ? 24.0 : 8.0;   // flops per complex entry and RHS (split-16: three products)
    const int tiles = (nrhs + rt - 1) / rt;
    const size_t cs = csize(prec);
    const ApplyGeom G{h->d, h->n, h->P, h->L, h->leaf, h->n0};
    const auto& up = adjoint ? h->rows : h->cols;
    const auto& down = adjoint ? h->cols : h->rows;
    const long long groups = ipow(h->P, h->L);
    std::vector<LaunchDesc> out;
    // Split 16-bit with a lattice copy, when the first up step keeps every leaf
    // point: that step only copies input rows, so the input is transposed into
    // the row-major copy instead and the step above reads it through its
    // lattice source-row table.
    // (only the source-row-table up kernels, split variants 7-10, read it)
    const int v_up1 = (prec == PREC_FP16 ? h->fp16_variant : h->bf16_variant)[0][1];
    const bool lat_in = is_split16(prec) && mfma && lat && !adjoint && h->b >= 2 && up[0].entries == 0 &&
                        up[1].d_src_lat != nullptr && v_up1 >= 7 && v_up1 < BF16_VARIANTS;
    // Split 16-bit: the exponents of the input's column maxima first; the
    // vectors of the chain are then held scaled (SplitScale).
    int* cexp = nullptr;
    if (is_split16(prec) && aux) {
        const int S = col_exp_slices(h->N);
        float* part = (float*)aux;
        cexp = (int*)(part + (size_t)nrhs * S);
        LaunchDesc D{};
        D.a.ce = ColExpArgs{in_ext, ld, h->N, nrhs, S, part, cexp};
        D.which = LevelKernel::ColExp;
        D.bytes = (double)h->N * nrhs * cs;
        D.level = 0;
        out.push_back(D);
    }
    // The scale exponents of the chain's vectors: hU for the input copy and
    // every up level, hD for every down level and the output.  Both sides
    // copy rows between levels, so each side keeps one scale, set by its
    // vectors with the most points behind an entry (the top up step's y, the
    // leaves' z); the middle moves from one to the other while staging.
    auto hbound = [&](long long pts) {
        int lg = 0;
        while ((1LL << lg) < pts) ++lg;
        return SPLIT16_HEADROOM - lg;
    };
    const int hU = hbound(h->N / ipow(h->P, h->L - h->b + 1)), hD = hbound(h->N / h->P);
    const SplitScale sc_in{cexp, hU}, sc_out{cexp, hD};
    auto pow2 = [](int e) { return std::ldexp(1.0f, e); };
    // The top up step may hand the middle its vectors already split (UpArgs::presplit); whether it
    // does is settled at launch from the two kernels' variants (launch_checked)
    const char* xenv = std::getenv("MIDBF_SPLIT_EXCHANGE");
    const bool exch = mfma && is_split16(prec) && !adjoint && h->b >= 2 && !(xenv && xenv[0] == '0');
    int o = 0;   // buffer holding the current level's vectors
    for (int s = 0; s < h->b; ++s) {
        const LevelSide& lv = up[s];
        LaunchDesc D{};
        if (lat_in && s == 0) {
            D.a.tr = TransposeArgs{in_ext, lat, ld, h->N, nrhs, sc_in};
            D.which = LevelKernel::TransposeIn;
            D.bytes = 2.0 * h->N * nrhs * cs;
            D.level = 0;
            out.push_back(D);
            o ^= 1;
            continue;
        }
        UpArgs& a = D.a.up;
        a.G = G;
        a.lev = level_args(h, lv, prec);
        a.s = s;
        a.Ps = ipow(h->P, s);
        a.ext = in_ext;
        a.ld = ld;
        a.in = buf[o ^ 1];
        a.k_prev = s ? up[s - 1].d_k : nullptr;
        a.yoff_prev = s ? up[s - 1].d_y_off : nullptr;
        a.out = buf[o];
        a.nrhs = nrhs;
        a.sc = sc_in;
        if (lat_in && s == 1) {
            a.in = lat;
            a.lev.src = lv.d_src_lat;
            a.lattice_in = 1;
        }
        const int ncand = s == 0 ? h->n0 : lv.nmax;
        a.ncand_max = ncand;
        a.nred_max = ncand - lv.kmin;
        a.presplit = exch && s == h->b - 1 ? (cexp ? pow2(hD - hU) : 1.f) : 0.f;
        // forward VALU up kernel: candidate vector plus one redundant-input strip per wave
        const size_t up_lds = (size_t)ncand * cs * (adjoint || rt > 1 ? rt : 1 + 4);
        const double vin = (s == 0 ? (double)h->N : (double)lv.total_n / h->P) * nrhs * cs;
        const double vout = (double)lv.total_k * nrhs * cs;
        const double fac = (double)lv.entries * cs + (double)lv.total_n * 4 + (double)lv.nid * 32;
        D.which = adjoint ? LevelKernel::AdjUp : LevelKernel::Up;
        D.grid = dim3((unsigned)groups, tiles);
        D.smem = mfma ? 0 : up_lds;
        D.bytes = fac + vin + vout;
        D.flops = fl * lv.entries * nrhs;
        D.mfma_count = mfma ? lv.nid : 0;
        D.level = s;
        if (mfma && s == 0 && lv.entries == 0 && h->n0 <= 64 && !adjoint && prec != PREC_FP64 && !h->points) {
            // every leaf keeps all its points: a staged copy per leaf (vin read once)
            D.which = LevelKernel::UpLeafCopy;
            D.mfma_count = groups;
            D.flops = 0;
        } else if (s == 0 && cexp) {
            // split 16-bit leaves with a product: the scaled row-major copy of the
            // input first, which the leaf kernels then read in place of the input
            MIDBF_CHECK(lat != nullptr, MIDBF_ERR_ARG, "split 16-bit applies need the lattice copy");
            LaunchDesc T{};
            T.a.tr = TransposeArgs{in_ext, lat, ld, h->N, nrhs, sc_in};
            T.which = LevelKernel::TransposeIn;
            T.bytes = 2.0 * h->N * nrhs * cs;
            T.level = 0;
            out.push_back(T);
            a.ext = nullptr;
            a.in = lat;
        }
        out.push_back(D);
        o ^= 1;
    }
    {
        const Middle& M = h->mid;
        MidArgs a{};
        a.nr = M.d_nr;
        a.nc = M.d_nc;
        a.off = M.d_off;
        a.S = M.S[prec];
        a.pieces = M.pieces;
        a.in_off = M.d_in_off;
        a.in_len = M.d_in_len;
        a.out_off = M.d_out_off;
        a.out_len = M.d_out_len;
        a.in = buf[o ^ 1];
        a.out = buf[o];
        a.nrhs = nrhs;
        a.in_max = M.nc_max;
        a.out_max = M.nr_max;
        a.ang = (is_split16(prec) && !adjoint) ? (const int*)M.ang : nullptr;
        a.bscale = cexp ? pow2(hD - hU) : 1.f;
        a.presplit = exch ? 1 : 0;
        if (adjoint && mfma) {
            // x = S^H z on the matrix cores: the blocks seen transposed (rows = columns of S),
            // inputs from the row pieces, outputs to the column pieces
            std::swap(a.nr, a.nc);
            std::swap(a.in_off, a.out_off);
            std::swap(a.in_len, a.out_len);
            a.in_max = M.nr_max;
            a.out_max = M.nc_max;
        }
        // FP32 matrix cores: split the rows of few large blocks over several workgroups
        const int rows_max = adjoint ? M.nc_max : M.nr_max;
        a.mchunks = (mfma && prec == PREC_FP32)
                        ? (int)std::max<long long>(1, std::min<long long>((2048 + M.nblk - 1) / std::max<long long>(M.nblk, 1),
                                                                          (rows_max + 127) / 128))
                        : 1;
        const int width = adjoint ? M.nr_max : M.nc_max;
        // VALU path: entries of the staged vector per LDS pass
        a.chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)std::max(width, 1), LDS_LIMIT / (rt * cs)));
        const long long chunk = chunk_middle ? 65535 : std::max<long long>(M.nblk, 1);
        for (long long b0 = 0; b0 < M.nblk; b0 += chunk) {
            const long long cnt = std::min<long long>(chunk, M.nblk - b0);
            LaunchDesc D{};
            MidArgs& ab = D.a.mid;
            ab = a;
            ab.nr += b0; ab.nc += b0; ab.off += b0;
            ab.in_off += b0 * M.pieces; ab.in_len += b0 * M.pieces;
            ab.out_off += b0 * M.pieces; ab.out_len += b0 * M.pieces;
            const double frac = (double)cnt / M.nblk;
            const double vec = (double)(h->rows.back().total_k + h->cols.back().total_k) * nrhs * cs;
            D.which = adjoint ? LevelKernel::AdjMiddle : LevelKernel::Middle;
            D.grid = dim3((unsigned)cnt, tiles);
            D.smem = (size_t)std::min(width, ab.chunk) * rt * cs;
            // split applies read the blocks' phase tiles: 4 B per entry (the
            // padding of partial tiles is counted as stored bytes only)
            const double fac_bytes = ab.ang ? 4.0 * M.total : (double)M.total * cs;
            D.bytes = frac * (fac_bytes + (double)M.nblk * 40 + vec);
            if (ab.ang) D.stored = frac * ((double)M.ang_bytes + (double)M.nblk * 40 + vec);
            D.flops = frac * fl * M.total * nrhs;
            D.mfma_count = mfma ? cnt : 0;
            D.level = -1;
            out.push_back(D);
        }
        o ^= 1;
    }
    for (int s = h->b - 1; s >= 0; --s) {
        const LevelSide& lv = down[s];
        LaunchDesc D{};
        DownArgs& a = D.a.down;
        a.G = G;
        a.lev = level_args(h, lv, prec);
        a.s = s;
        a.Ps = ipow(h->P, s);
        a.in = buf[o ^ 1];
        a.ext = lat && s == 0 ? nullptr : out_ext;
        a.ld = ld;
        a.out = lat && s == 0 ? lat : buf[o];
        a.k_prev = s ? down[s - 1].d_k : nullptr;
        a.yoff_prev = s ? down[s - 1].d_y_off : nullptr;
        a.nrhs = nrhs;
        a.ncand_max = lv.nmax;
        a.kmax = lv.kmax;
        const double vin = (double)lv.total_k * nrhs * cs;
        const double vout = (s == 0 ? (double)h->N : (double)lv.total_n / h->P) * nrhs * cs;
        const double fac = (double)lv.entries * cs + (double)lv.total_n * 4 + (double)lv.nid * 32;
        D.level = s;
        const int dvar = (prec == PREC_FP16 ? h->fp16_variant : h->bf16_variant)[1][std::min(s, midbf_plan::VMAXLEV - 1)];
        if (mfma && is_split16(prec) && lv.groups > 0 && !adjoint) {
            // split 16-bit, s >= 1: one dense block per group, run by the middle kernels
            MidArgs m{};
            m.nr = lv.d_g_nr;
            m.nc = lv.d_g_nc;
            m.off = lv.d_g_tile_off;
            m.S = lv.g_T[prec];
            m.pieces = h->P;
            m.in_off = lv.d_g_in_off;
            m.in_len = lv.d_g_in_len;
            m.out_off = lv.d_g_out_off;
            m.out_len = lv.d_g_out_len;
            m.in = buf[o ^ 1];
            m.out = buf[o];
            m.nrhs = nrhs;
            m.in_max = lv.g_nc_max;
            m.out_max = lv.g_nr_max;
            m.mchunks = 1;
            m.bscale = 1.f;          // z keeps its scale going down
            D.a.mid = m;
            D.which = LevelKernel::DownDense;
            D.grid = dim3();
            D.smem = 0;
            // algorithmic: the T entries (8 B as hi / lo pairs); the group tiles
            // also hold the skeleton rows' identity entries and tile padding
            D.bytes = (double)lv.entries * cs + (double)lv.groups * 48 + vin + vout;
            D.stored = (double)lv.g_tiles * BF16_TILE_BYTES + (double)lv.groups * 48 + vin + vout;
            D.flops = fl * lv.g_entries * nrhs;
            D.mfma_count = lv.groups;
            out.push_back(D);
        } else if (mfma && is_split16(prec) && s == 0 && h->n0 <= 64 && !adjoint && (nrhs == 1 || lat)) {
            // split 16-bit leaves: the P siblings summed in LDS, each point's row written once
            D.which = LevelKernel::DownLeaf;
            D.grid = dim3();
            D.smem = 0;
            D.bytes = fac + vin + vout;
            D.flops = fl * lv.entries * nrhs;
            D.mfma_count = groups;
            out.push_back(D);
        } else if (mfma && is_split16(prec) && dvar >= 5 && lv.kmax <= SPLIT16_RESIDENT_K && (nrhs == 1 || lat || s > 0)) {
            // split 16-bit with z resident: the siblings of each group add into its candidate rows
            D.which = LevelKernel::DownGroup;
            D.grid = dim3();
            D.smem = 0;
            D.bytes = fac + vin + vout;
            D.flops = fl * lv.entries * nrhs;
            D.mfma_count = groups;
            out.push_back(D);
        } else if (mfma) {
            // per-ID contributions to the scratch block, then the ordered group sums
            const double scr = (double)lv.total_n * nrhs * cs;
            D.which = adjoint ? LevelKernel::AdjDown : LevelKernel::Down;
            D.grid = dim3();
            D.smem = 0;
            D.bytes = fac + vin + scr;
            D.flops = fl * lv.entries * nrhs;
            D.mfma_count = lv.nid;
            out.push_back(D);
            D.which = LevelKernel::DownSum;
            D.bytes = scr + vout;
            D.flops = 2.0 * (lv.total_n - lv.total_n / h->P) * nrhs;
            D.mfma_count = groups;
            out.push_back(D);
        } else {
            D.which = adjoint ? LevelKernel::AdjDown : LevelKernel::Down;
            D.grid = dim3((unsigned)groups, tiles);
            D.smem = (size_t)(lv.nmax + lv.kmax) * rt * cs;
            D.bytes = fac + vin + vout;
            D.flops = 8.0 * lv.entries * nrhs;
            D.mfma_count = 0;
            out.push_back(D);
        }
        o ^= 1;
    }
    if (lat) {
        LaunchDesc D{};
        D.a.tr = TransposeArgs{lat, out_ext, ld, h->N, nrhs, sc_out};
        D.which = LevelKernel::Transpose;
        D.bytes = 2.0 * h->N * nrhs * cs;
        D.level = 1;
        out.push_back(D);
    }
    return out;
}

void check_apply_args(midbf_plan* h, const void* in_ext, void* out_ext, int nrhs, long long ld, int prec) {
    MIDBF_CHECK(nrhs >= 1, MIDBF_ERR_ARG, "nrhs must be >= 1");
    MIDBF_CHECK(ld >= h->N, MIDBF_ERR_ARG, "ld must be >= N");
    MIDBF_CHECK(in_ext && out_ext, MIDBF_ERR_ARG, "null vector pointer");
    MIDBF_CHECK(h->keep & (1u << prec), MIDBF_ERR_ARG, "this precision's factors were not kept by the build");
}

// Which kernels an apply runs: matrix cores (split 16-bit always; FP32 and
// FP64 for many right-hand sides) and, on matrix cores with several
// right-hand sides, the row-major lattice copy around the leaf levels.
struct ApplyMode {
    bool mfma, lat;
    int rt;
};

ApplyMode apply_mode(const midbf_plan* h, int nrhs, int prec, bool adjoint) {
    const bool fits = h->max_n <= MFMA_CROW_MAX && h->mid.nr_max + h->mid.nc_max <= 2 * MFMA_CROW_MAX;
    const bool fits_bf16 =
        h->max_n <= BF16_CROW_MAX && h->mid.nr_max <= BF16_CROW_MAX && h->mid.nc_max <= BF16_CROW_MAX;
    MIDBF_CHECK(!is_split16(prec) || (!adjoint && fits_bf16), MIDBF_ERR_UNIMPLEMENTED,
                "the split 16-bit applies exist for the forward transform with candidate sets up to 2048");
    MIDBF_CHECK(!is_split16(prec) || !h->points, MIDBF_ERR_UNIMPLEMENTED,
                "scattered points are applied in FP64 and FP32");
    ApplyMode m;
    m.mfma = is_split16(prec) || ((prec == PREC_FP32 || prec == PREC_FP64) && nrhs >= MFMA_MIN_NRHS && fits);
    m.lat = m.mfma && (nrhs > 1 || is_split16(prec));
    m.rt = nrhs == 1 ? 1 : (prec == PREC_FP64 ? APPLY_RT64 : APPLY_RT);
    return m;
}

// Whether a launch sequence uses the matrix-core down pass's per-ID
// contribution block (Workspace::scratch).
bool needs_scratch(const std::vector<LaunchDesc>& launches) {
    for (const LaunchDesc& D : launches)
        if (D.mfma_count > 0 && (D.which == LevelKernel::Down || D.which == LevelKernel::AdjDown ||
                                 D.which == LevelKernel::DownSum))
            return true;
    return false;
}

std::vector<LaunchDesc> plan_for(midbf_plan* h, const Workspace& ws, const ApplyMode& m, const void* in_ext,
                                 void* out_ext, int nrhs, long long ld, int prec, bool adjoint) {
    return plan_apply(h, in_ext, out_ext, nrhs, ld, prec, adjoint, m.mfma, ws.buf, true, m.rt,
                      m.lat ? ws.lat : nullptr, ws.aux);
}

// Launch a planned apply; the contribution block is read from ws at launch.
// profile = false: no events are taken, even with the handle's profiler on.
void launch_planned(midbf_plan* h, const Workspace& ws, const ApplyMode& m, const std::vector<LaunchDesc>& launches,
                    int nrhs, int prec, hipStream_t st, bool profile) {
    for (const LaunchDesc& D : launches)
        launch_checked(h, ws, D.which, prec, m.rt, &D.a, D.grid, D.smem, st, D.bytes, D.flops, D.mfma_count, nrhs,
                       D.level, profile, D.stored > 0.0 ? D.stored : -1.0);
}

void run_apply(midbf_plan* h, const void* in_ext, void* out_ext, int nrhs, long long ld, int prec,
               hipStream_t st, bool adjoint) {
    check_apply_args(h, in_ext, out_ext, nrhs, ld, prec);
    const ApplyMode m = apply_mode(h, nrhs, prec, adjoint);
    ensure_workspace(h, prec, nrhs, false, m.lat);
    const auto launches = plan_for(h, h->ws[prec], m, in_ext, out_ext, nrhs, ld, prec, adjoint);
    if (needs_scratch(launches)) ensure_workspace(h, prec, nrhs, true, m.lat);
    launch_planned(h, h->ws[prec], m, launches, nrhs, prec, st, true);
}

// Device address of the no-allocation scratch on the current device, looked
// up once per device with that device current.
void* noalloc_scratch() {
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static void* addr[MAX_DEVICES] = {};
    int dev = -1;
    MIDBF_HIP(hipGetDevice(&dev));
    MIDBF_CHECK(dev >= 0 && dev < MAX_DEVICES, MIDBF_ERR_HIP, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        MIDBF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        MIDBF_CHECK(p != nullptr, MIDBF_ERR_HIP, "no device address for the no-allocation scratch");
        addr[dev] = p;
    }
    return addr[dev];
}

// midbf_apply with every workspace part carved out of the static scratch
// (256-byte aligned pieces: both level buffers, the lattice copy, then the
// contribution block if the launches use it); no device or profiler
// allocation.
void run_apply_noalloc(midbf_plan* h, const void* in_ext, void* out_ext, int nrhs, long long ld, int prec,
                       hipStream_t st) {
    check_apply_args(h, in_ext, out_ext, nrhs, ld, prec);
    const ApplyMode m = apply_mode(h, nrhs, prec, false);
    const WorkspaceNeed need = workspace_need(h, prec, nrhs, true, m.lat);
    auto round_up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t b = round_up(need.buf), la = round_up(need.lat), ax = round_up(need.aux),
                 sc = round_up(need.scratch);
    unsigned char* base = (unsigned char*)noalloc_scratch();
    Workspace ws;
    ws.buf[0] = base;
    ws.buf[1] = base + b;
    ws.bytes = need.buf;
    ws.lat = m.lat ? base + 2 * b : nullptr;
    ws.lat_bytes = need.lat;
    ws.aux = need.aux ? base + 2 * b + la : nullptr;
    ws.aux_bytes = need.aux;
    const auto launches = plan_for(h, ws, m, in_ext, out_ext, nrhs, ld, prec, false);
    const bool scr = needs_scratch(launches);
    if (scr) {
        ws.scratch = base + 2 * b + la + ax;
        ws.scratch_bytes = need.scratch;
    }
    const size_t total = 2 * b + la + ax + (scr ? sc : 0);
    MIDBF_CHECK(total <= (size_t)MIDBF_NOALLOC_SCRATCH_BYTES, MIDBF_ERR_SHAPE,
                "this apply needs " + std::to_string(total) + " bytes of workspace; the no-allocation scratch holds " +
                    std::to_string((size_t)MIDBF_NOALLOC_SCRATCH_BYTES) +
                    " (use midbf_apply, or fewer right-hand sides per call)");
    launch_planned(h, ws, m, launches, nrhs, prec, st, false);
}

}  // namespace

}  // namespace midbf

// One apply's launch sequence captured in a hipGraph (midbf_apply_graph_*).
struct midbf_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace midbf {
namespace {

void free_graph(midbf_graph_s* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

// Capture the launches of midbf_apply(h, in, out, ...) on a private stream.
// The handle's workspace for nrhs is reserved (allocated) before the capture,
// so the graph holds no allocation; profiling events are not captured.
midbf_graph_s* capture_apply(midbf_plan* h, const void* in_ext, void* out_ext, int nrhs, long long ld, int prec,
                             hipStream_t st) {
    check_apply_args(h, in_ext, out_ext, nrhs, ld, prec);
    const ApplyMode m = apply_mode(h, nrhs, prec, false);
    ensure_workspace(h, prec, nrhs, false, m.lat);
    const auto launches = plan_for(h, h->ws[prec], m, in_ext, out_ext, nrhs, ld, prec, false);
    if (needs_scratch(launches)) ensure_workspace(h, prec, nrhs, true, m.lat);
    MIDBF_HIP(hipStreamSynchronize(st));
    std::unique_ptr<midbf_graph_s, void (*)(midbf_graph_s*)> g(new midbf_graph_s, free_graph);
    hipStream_t cap;
    MIDBF_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    try {
        MIDBF_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        launch_planned(h, h->ws[prec], m, launches, nrhs, prec, cap, false);
        MIDBF_HIP(hipStreamEndCapture(cap, &g->graph));
        MIDBF_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    } catch (...) {
        hipGraph_t dangling = nullptr;
        (void)hipStreamEndCapture(cap, &dangling);
        if (dangling) (void)hipGraphDestroy(dangling);
        (void)hipStreamDestroy(cap);
        throw;
    }
    MIDBF_HIP(hipStreamDestroy(cap));
    return g.release();
}

}  // namespace
}  // namespace midbf

// A batch of forward transforms (midbf_batch_*): the stage table on the
// device, one pair of level buffers per transform, and one persistent launch
// per run (optionally replayed from a captured hipGraph).
struct midbf_batch_s {
    int prec = 0, rt = 1, nst = 0, rounds = 0, grid = 0;
    size_t smem = 0;
    long long items = 0;
    std::vector<void*> bufs;
    midbf::BatchStage* d_st = nullptr;
    midbf::BatchSegment* d_seg = nullptr;
    unsigned* d_ctl = nullptr;          // control block of the persistent runs (BATCH_CTL_HEAD + nst words)
    midbf::PersistArgs args{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double bytes = 0, flops = 0;
};

namespace midbf {

// The queue of a batch.  Stage (j, r) is level launch r of transform j, with
// items[j][r] tasks; dep = stage (j, r - 1) or -1.  Segments of at most
// `chunk` consecutive items are handed out level by level (every transform's
// level r before any level r + 1); within a level, transforms of one sharing
// group (share[j]: the same factorization) go item block by item block, so
// the segments of all members that read the same factor blocks are adjacent
// in the queue and run at about the same time (the later reads hit the
// caches).  Segments only ever depend on earlier segments.
struct Schedule {
    std::vector<int> dep;
    std::vector<long long> items;
    std::vector<BatchSegment> seg;
};

Schedule build_schedule(const std::vector<std::vector<long long>>& items, const std::vector<int>& share, int chunk) {
    MIDBF_CHECK(chunk >= 1 && share.size() == items.size(), MIDBF_ERR_ARG, "bad batch schedule arguments");
    Schedule S;
    const int T = (int)items.size();
    size_t rounds = 0;
    for (const auto& v : items) rounds = std::max(rounds, v.size());
    std::vector<std::vector<int>> stage_of(T);
    for (size_t r = 0; r < rounds; ++r)           // stages numbered level by level
        for (int j = 0; j < T; ++j) {
            if (r >= items[j].size()) continue;
            MIDBF_CHECK(items[j][r] >= 1, MIDBF_ERR_SHAPE, "a level launch without workgroups");
            S.dep.push_back(r ? stage_of[j][r - 1] : -1);
            S.items.push_back(items[j][r]);
            stage_of[j].push_back((int)S.items.size() - 1);
        }
    std::vector<int> groups;                      // sharing groups in order of first appearance
    for (int j = 0; j < T; ++j)
        if (std::find(groups.begin(), groups.end(), share[j]) == groups.end()) groups.push_back(share[j]);
    for (size_t r = 0; r < rounds; ++r)
        for (int gid : groups) {
            long long most = 0;
            for (int j = 0; j < T; ++j)
                if (share[j] == gid && r < items[j].size()) most = std::max(most, items[j][r]);
            for (long long i0 = 0; i0 < most; i0 += chunk)
                for (int j = 0; j < T; ++j) {
                    if (share[j] != gid || r >= items[j].size() || i0 >= items[j][r]) continue;
                    S.seg.push_back(BatchSegment{stage_of[j][r], (int)std::min<long long>(chunk, items[j][r] - i0), i0});
                }
        }
    return S;
}

// The persistent kernel's queue protocol run by host threads in place of
// workgroups (any number, also far fewer than segments): take one segment per
// atomic step, wait for its dependency stage to complete, "run" its items (a
// short random pause), count them complete.  A wait longer than limit_ms
// counts as a stall.  Returns the items completed and the stalls.
void simulate_schedule(const Schedule& S, int workers, int limit_ms, unsigned seed, long long& completed,
                       long long& stalls) {
    std::atomic<long long> next{0}, comp{0}, stall{0};
    std::vector<std::atomic<long long>> done(S.items.size());
    for (auto& d : done) d.store(0);
    const long long nseg = (long long)S.seg.size();
    auto worker = [&](int w) {
        unsigned x = seed * 2654435761u + (unsigned)w * 40503u + 1u;
        for (;;) {
            const long long si = next.fetch_add(1);
            if (si >= nseg) return;
            const BatchSegment& sg = S.seg[si];
            const int dep = S.dep[sg.stage];
            if (dep >= 0) {
                const auto start = std::chrono::steady_clock::now();
                while (done[dep].load(std::memory_order_acquire) < S.items[dep]) {
                    if (std::chrono::steady_clock::now() - start > std::chrono::milliseconds(limit_ms)) {
                        stall.fetch_add(1);
                        break;
                    }
                    std::this_thread::yield();
                }
            }
            x = x * 1664525u + 1013904223u;
            if ((x >> 28) == 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
            done[sg.stage].fetch_add(sg.count, std::memory_order_release);
            comp.fetch_add(sg.count);
        }
    };
    std::vector<std::thread> th;
    for (int w = 0; w < workers; ++w) th.emplace_back(worker, w);
    for (auto& t : th) t.join();
    completed = comp.load();
    stalls = stall.load();
}

namespace {

void free_batch(midbf_batch_s* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (void* p : b->bufs) (void)hipFree(p);
    if (b->d_st) (void)hipFree(b->d_st);
    if (b->d_seg) (void)hipFree(b->d_seg);
    if (b->d_ctl) (void)hipFree(b->d_ctl);
    delete b;
}

constexpr int BATCH_CHUNK = 8;                    // items per segment of the queue
constexpr long long BATCH_SPIN_LIMIT = 1LL << 20; // polls (~1-2 us each) before a wait is abandoned

void launch_batch(const midbf_batch_s* b, hipStream_t st) {
    launch_persistent(b->prec, b->rt, b->args, b->grid, b->smem, st);
}

midbf_batch_s* create_batch(int count, const midbf_handle* hs, const void* const* f, void* const* g, const int* nrhs,
                            int prec, bool use_graph, hipStream_t st) {
    MIDBF_CHECK(count >= 1, MIDBF_ERR_ARG, "empty batch");
    MIDBF_CHECK(prec == PREC_FP64 || prec == PREC_FP32, MIDBF_ERR_UNIMPLEMENTED,
                "the batched apply runs in FP64 or FP32");
    for (int j = 0; j < count; ++j) {
        MIDBF_CHECK(hs[j], MIDBF_ERR_ARG, "null handle in batch");
        check_apply_args(hs[j], f[j], g[j], nrhs[j], hs[j]->N, prec);
    }
    std::unique_ptr<midbf_batch_s, void (*)(midbf_batch_s*)> b(new midbf_batch_s, free_batch);
    b->prec = prec;
    const size_t cs = csize(prec);
    bool single = true;
    for (int j = 0; j < count; ++j) single = single && nrhs[j] == 1;
    b->rt = single ? 1 : (prec == PREC_FP64 ? APPLY_RT64 : APPLY_RT);
    std::vector<std::vector<LaunchDesc>> seq(count);
    std::vector<std::vector<long long>> items(count);
    std::vector<int> share(count);
    for (int j = 0; j < count; ++j) {
        midbf_plan* h = hs[j];
        void* buf[2] = {nullptr, nullptr};
        const size_t need = (size_t)std::max<long long>(h->max_total_k, 1) * nrhs[j] * cs;
        for (int i = 0; i < 2; ++i) {
            MIDBF_HIP(hipMalloc(&buf[i], need));
            b->bufs.push_back(buf[i]);
        }
        seq[j] = plan_apply(h, f[j], g[j], nrhs[j], h->N, prec, false, false, buf, false, b->rt);
        for (const LaunchDesc& D : seq[j]) items[j].push_back((long long)D.grid.x * D.grid.y);
        b->rounds = std::max(b->rounds, (int)seq[j].size());
        share[j] = j;                                    // transforms with one handle share its factors
        for (int i = 0; i < j; ++i)
            if (hs[i] == h) {
                share[j] = share[i];
                break;
            }
    }
    const Schedule S = build_schedule(items, share, BATCH_CHUNK);
    MIDBF_CHECK(S.seg.size() < 0x7fffffffULL - 65536, MIDBF_ERR_SHAPE, "batch too large");
    std::vector<BatchStage> stages(S.items.size());
    {
        size_t q = 0;
        for (int r = 0; r < b->rounds; ++r)              // the schedule's stage numbering
            for (int j = 0; j < count; ++j) {
                if (r >= (int)seq[j].size()) continue;
                const LaunchDesc& D = seq[j][r];
                MIDBF_CHECK(D.smem <= LDS_LIMIT, MIDBF_ERR_UNIMPLEMENTED,
                            "candidate vectors of this factorization exceed the apply kernels' LDS budget");
                BatchStage& B = stages[q];
                B = BatchStage{};
                B.kind = D.which == LevelKernel::Up ? 0 : (D.which == LevelKernel::Middle ? 1 : 2);
                B.tiles = (int)D.grid.y;
                B.items = S.items[q];
                B.dep = S.dep[q];
                std::memcpy(&B.a, &D.a, sizeof(B.a));
                b->smem = std::max(b->smem, D.smem);
                b->bytes += D.bytes;
                b->flops += D.flops;
                b->items += S.items[q];
                ++q;
            }
    }
    b->nst = (int)stages.size();
    MIDBF_HIP(hipMalloc(&b->d_st, stages.size() * sizeof(BatchStage)));
    MIDBF_HIP(hipMemcpyAsync(b->d_st, stages.data(), stages.size() * sizeof(BatchStage), hipMemcpyHostToDevice, st));
    MIDBF_HIP(hipMalloc(&b->d_seg, S.seg.size() * sizeof(BatchSegment)));
    MIDBF_HIP(hipMemcpyAsync(b->d_seg, S.seg.data(), S.seg.size() * sizeof(BatchSegment), hipMemcpyHostToDevice, st));
    const size_t ctl_bytes = (BATCH_CTL_HEAD + stages.size()) * sizeof(unsigned);
    MIDBF_HIP(hipMalloc(&b->d_ctl, ctl_bytes));
    MIDBF_HIP(hipMemsetAsync(b->d_ctl, 0, ctl_bytes, st));      // (once, outside any captured graph)
    MIDBF_HIP(hipStreamSynchronize(st));
    b->grid = (int)std::min<long long>(persistent_capacity(prec, b->rt, b->smem), (long long)S.seg.size());
    b->args = PersistArgs{b->d_st, b->d_seg, (int)S.seg.size(), b->d_ctl, b->nst, BATCH_SPIN_LIMIT};
    if (use_graph) {
        hipStream_t cap;
        MIDBF_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        try {
            MIDBF_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            launch_batch(b.get(), cap);
            MIDBF_HIP(hipStreamEndCapture(cap, &b->graph));
            MIDBF_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        } catch (...) {
            hipGraph_t dangling = nullptr;
            (void)hipStreamEndCapture(cap, &dangling);
            if (dangling) (void)hipGraphDestroy(dangling);
            (void)hipStreamDestroy(cap);
            throw;
        }
        MIDBF_HIP(hipStreamDestroy(cap));
    }
    return b.release();
}

void run_batch(midbf_batch_s* b, hipStream_t st) {
    if (b->exec) MIDBF_HIP(hipGraphLaunch(b->exec, st));
    else launch_batch(b, st);
}

}  // namespace
}  // namespace midbf

using namespace midbf;

extern "C" {

midbf_status midbf_build(const midbf_params* p, void* stream, midbf_handle* out) {
    if (!p || !out) return fail(MIDBF_ERR_ARG, "null argument");
    *out = nullptr;
    return guarded([&] { *out = build_plan(*p, (hipStream_t)stream); });
}

midbf_status midbf_save(midbf_handle h, const char* path, void* stream) {
    if (!h || !path) return fail(MIDBF_ERR_ARG, "null argument");
    return guarded([&] { save_plan(h, path, (hipStream_t)stream); });
}

midbf_status midbf_load(const char* path, unsigned precisions, void* stream, midbf_params* params_out,
                        midbf_handle* out) {
    if (!path || !out) return fail(MIDBF_ERR_ARG, "null argument");
    *out = nullptr;
    return guarded([&] { *out = load_plan(path, precisions, (hipStream_t)stream, params_out); });
}

midbf_status midbf_apply(midbf_handle h, const void* f, void* g, int nrhs, long long ld, midbf_precision prec,
                         void* stream) {
    if (!h) return fail(MIDBF_ERR_ARG, "null handle");
    return guarded([&] { run_apply(h, f, g, nrhs, ld, prec_index(prec), (hipStream_t)stream, false); });
}

midbf_status midbf_apply_noalloc(midbf_handle h, const void* f, void* g, int nrhs, long long ld,
                                 midbf_precision prec, void* stream) {
    if (!h) return fail(MIDBF_ERR_ARG, "null handle");
    return guarded([&] { run_apply_noalloc(h, f, g, nrhs, ld, prec_index(prec), (hipStream_t)stream); });
}

midbf_status midbf_apply_graph_create(midbf_handle h, const void* f, void* g, int nrhs, long long ld,
                                      midbf_precision prec, void* stream, midbf_graph* out) {
    if (!out) return fail(MIDBF_ERR_ARG, "null argument");
    *out = nullptr;
    if (!h) return fail(MIDBF_ERR_ARG, "null handle");
    return guarded([&] { *out = capture_apply(h, f, g, nrhs, ld, prec_index(prec), (hipStream_t)stream); });
}

midbf_status midbf_graph_launch(midbf_graph g, void* stream) {
    if (!g) return fail(MIDBF_ERR_ARG, "null graph");
    return guarded([&] { MIDBF_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream)); });
}

void midbf_graph_destroy(midbf_graph g) { free_graph(g); }

midbf_status midbf_apply_adjoint(midbf_handle h, const void* g, void* f, int nrhs, long long ld,
                                 midbf_precision prec, void* stream) {
    if (!h) return fail(MIDBF_ERR_ARG, "null handle");
    return guarded([&] { run_apply(h, g, f, nrhs, ld, prec_index(prec), (hipStream_t)stream, true); });
}

midbf_status midbf_apply_batched(int count, const midbf_handle* hs, const void* const* f, void* const* g,
                                 const int* nrhs, midbf_precision prec, void* stream) {
    if (count < 0 || (count > 0 && (!hs || !f || !g || !nrhs))) return fail(MIDBF_ERR_ARG, "null argument");
    if (count == 0) return MIDBF_OK;
    return guarded([&] {
        hipStream_t st = (hipStream_t)stream;
        std::unique_ptr<midbf_batch_s, void (*)(midbf_batch_s*)> b(
            create_batch(count, hs, f, g, nrhs, prec_index(prec), false, st), free_batch);
        run_batch(b.get(), st);
        MIDBF_HIP(hipStreamSynchronize(st));    // the batch's buffers are freed on return
    });
}

midbf_status midbf_batch_create(int count, const midbf_handle* hs, const void* const* f, void* const* g,
                                const int* nrhs, midbf_precision prec, int use_graph, void* stream, midbf_batch* out) {
    if (!out) return fail(MIDBF_ERR_ARG, "null argument");
    *out = nullptr;
    if (count < 1 || !hs || !f || !g || !nrhs) return fail(MIDBF_ERR_ARG, "empty batch or null argument");
    return guarded([&] { *out = create_batch(count, hs, f, g, nrhs, prec_index(prec), use_graph != 0,
                                             (hipStream_t)stream); });
}

midbf_status midbf_batch_run(midbf_batch b, void* stream) {
    if (!b) return fail(MIDBF_ERR_ARG, "null batch");
    return guarded([&] { run_batch(b, (hipStream_t)stream); });
}

midbf_status midbf_batch_get_stats(midbf_batch b, midbf_batch_stats* out) {
    if (!b || !out) return fail(MIDBF_ERR_ARG, "null argument");
    return guarded([&] {
        unsigned timeouts = 0;
        MIDBF_HIP(hipDeviceSynchronize());
        MIDBF_HIP(hipMemcpy(&timeouts, b->d_ctl + 2, sizeof(unsigned), hipMemcpyDeviceToHost));
        out->stages = b->nst;
        out->rounds = b->rounds;
        out->items = b->items;
        out->graph = b->exec != nullptr;
        out->lds_bytes = (long long)b->smem;
        out->bytes = b->bytes;
        out->flops = b->flops;
        out->launches = 1;
        out->workgroups = b->grid;
        out->timeouts = (long long)timeouts;
    });
}

midbf_status midbf_schedule_simulate(int count, const int* levels, const long long* items, const int* share,
                                     int workers, int chunk, int limit_ms, unsigned seed, long long* completed,
                                     long long* stalls) {
    if (count < 1 || !levels || !items || !completed || !stalls || workers < 1 || chunk < 1 || limit_ms < 1)
        return fail(MIDBF_ERR_ARG, "bad schedule simulation arguments");
    return guarded([&] {
        std::vector<std::vector<long long>> it(count);
        std::vector<int> sh(count);
        long long o = 0;
        for (int j = 0; j < count; ++j) {
            MIDBF_CHECK(levels[j] >= 0, MIDBF_ERR_ARG, "negative level count");
            it[j].assign(items + o, items + o + levels[j]);
            o += levels[j];
            sh[j] = share ? share[j] : j;
        }
        const Schedule S = build_schedule(it, sh, chunk);
        simulate_schedule(S, workers, limit_ms, seed, *completed, *stalls);
    });
}

void midbf_batch_destroy(midbf_batch b) { free_batch(b); }

midbf_status midbf_factor_stats(midbf_handle h, midbf_stats* out) {
    if (!h || !out) return fail(MIDBF_ERR_ARG, "null argument");
    *out = h->stats;
    return MIDBF_OK;
}

midbf_status midbf_ranks(midbf_handle h, int side, int step, int* out, long long count) {
    if (!h || !out) return fail(MIDBF_ERR_ARG, "null argument");
    if (side < 0 || side > 1 || step < 0 || step >= h->b) return fail(MIDBF_ERR_ARG, "bad side or step");
    const auto& lv = side == 0 ? h->rows[step] : h->cols[step];
    if (count < 0 || count > (long long)lv.k.size())
        return fail(MIDBF_ERR_ARG, "count must lie in [0, number of IDs]");
    std::memcpy(out, lv.k.data(), count * sizeof(int));
    return MIDBF_OK;
}

midbf_status midbf_kernel_entries(const midbf_params* p, const int* rows, int nrows, const int* cols, int ncols,
                                  void* out, void* stream) {
    if (!p || (nrows > 0 && !rows) || (ncols > 0 && !cols) || !out) return fail(MIDBF_ERR_ARG, "null argument");
    return guarded([&] {
        kernel_entries(*p, rows, nrows, cols, ncols, out, (hipStream_t)stream);
    });
}

midbf_status midbf_id_batch(void* X, int batch, int m, int n, double tol, int k_cap, int* k_dev, int* perm_dev,
                            void* T_dev, void* stream) {
    if (!X || !k_dev || !perm_dev || !T_dev) return fail(MIDBF_ERR_ARG, "null argument");
    return guarded([&] { id_batch(X, batch, m, n, tol, k_cap, k_dev, perm_dev, T_dev, (hipStream_t)stream); });
}

// name of a profiled launch -> (kind, step): up / down(+sum) / middle, "_s<step>" suffix
static void kind_level(const std::string& name, int& q, int& lv) {
    q = name.rfind("up", 0) == 0 ? 0 : (name.rfind("down", 0) == 0 ? 1 : 2);
    lv = 0;
    const size_t p = name.rfind("_s");
    if (p != std::string::npos && p + 2 < name.size() && isdigit((unsigned char)name[p + 2])) lv = std::atoi(name.c_str() + p + 2);
    lv = std::min(lv, midbf_plan::VMAXLEV - 1);
}

midbf_status midbf_tune(midbf_handle h, int nrhs, midbf_precision prec, void* stream, int* variants) {
    if (!h) return fail(MIDBF_ERR_ARG, "null handle");
    return guarded([&] {
        const int pi = prec_index(prec);
        hipStream_t st = (hipStream_t)stream;
        const bool bf = is_split16(pi) && (h->keep & (1u << pi));
        auto& var = pi == PREC_FP16   ? h->fp16_variant
                    : pi == PREC_BF16 ? h->bf16_variant
                    : pi == PREC_FP64 ? h->mfma64_variant
                                      : h->mfma_variant;
        const int nvar = bf ? BF16_VARIANTS : (pi == PREC_FP64 ? MFMA64_VARIANTS : MFMA_VARIANTS);
        constexpr int NL = midbf_plan::VMAXLEV;
        const bool cores = (pi == PREC_FP32 || pi == PREC_FP64) && nrhs >= MFMA_MIN_NRHS && (h->keep & (1u << pi));
        if (bf || cores) {
            void* f = nullptr;
            void* g = nullptr;
            const size_t bytes = (size_t)h->N * nrhs * csize(pi);
            MIDBF_HIP(hipMalloc(&f, bytes));
            if (hipMalloc(&g, bytes) != hipSuccess) {
                (void)hipFree(f);
                throw Error(MIDBF_ERR_OOM, "tuning buffers");
            }
            const bool was_on = h->prof.on, was_lv = h->prof.by_level;
            const std::vector<ProfRecord> saved = h->prof.recs;
            h->prof.recs.clear();
            std::vector<double> best(3 * NL, 1e300);
            std::vector<int> pick(3 * NL, 0);
            try {
                MIDBF_HIP(hipMemsetAsync(f, 0, bytes, st));
                for (int v = 0; v < nvar; ++v) {
                    for (int q = 0; q < 3; ++q)
                        for (int l = 0; l < NL; ++l) var[q][l] = v;
                    h->prof.on = false;
                    run_apply(h, f, g, nrhs, h->N, pi, st, false);          // warm-up
                    // each kernel's time: the faster of two timed applies
                    std::vector<double> t(3 * NL, 1e300);
                    for (int rep = 0; rep < 2; ++rep) {
                        h->prof.on = true;
                        h->prof.by_level = true;
                        run_apply(h, f, g, nrhs, h->N, pi, st, false);
                        h->prof.on = false;
                        std::vector<double> tr(3 * NL, 0.0);
                        for (auto& r : h->prof.recs) {
                            MIDBF_HIP(hipEventSynchronize(r.b));
                            float ms = 0.f;
                            MIDBF_HIP(hipEventElapsedTime(&ms, r.a, r.b));
                            int q, lv;
                            kind_level(r.name, q, lv);
                            if (r.name.rfind("transpose", 0) != 0) tr[q * NL + lv] += ms;
                            h->prof.pool.push_back(r.a);
                            h->prof.pool.push_back(r.b);
                        }
                        h->prof.recs.clear();
                        for (int i = 0; i < 3 * NL; ++i)
                            if (tr[i] > 0.0) t[i] = std::min(t[i], tr[i]);
                    }
                    for (int i = 0; i < 3 * NL; ++i)
                        if (t[i] < 1e300 && t[i] < best[i]) { best[i] = t[i]; pick[i] = v; }
                }
            } catch (...) {
                h->prof.on = was_on;
                h->prof.by_level = was_lv;
                h->prof.recs = saved;
                (void)hipFree(f);
                (void)hipFree(g);
                throw;
            }
            h->prof.on = was_on;
            h->prof.by_level = was_lv;
            h->prof.recs = saved;
            MIDBF_HIP(hipStreamSynchronize(st));
            (void)hipFree(f);
            (void)hipFree(g);
            for (int q = 0; q < 3; ++q)
                for (int l = 0; l < NL; ++l) var[q][l] = pick[q * NL + l];
        }
        // reported: the choice for the largest step of each kind (up, down) and the middle
        if (variants) {
            const int top = std::max(0, std::min(h->b - 1, NL - 1));
            variants[0] = var[0][top];
            variants[1] = var[1][top];
            variants[2] = var[2][0];
        }
    });
}

midbf_status midbf_set_variants(midbf_handle h, midbf_precision prec, const int* variants) {
    if (!h || !variants) return fail(MIDBF_ERR_ARG, "null argument");
    const bool bf = prec == MIDBF_SPLIT_BF16 || prec == MIDBF_SPLIT_FP16;
    const bool f64 = prec == MIDBF_FP64;
    if (!bf && !f64 && prec != MIDBF_FP32) return fail(MIDBF_ERR_ARG, "unknown precision");
    const int nvar = bf ? BF16_VARIANTS : (f64 ? MFMA64_VARIANTS : MFMA_VARIANTS);
    for (int q = 0; q < 3; ++q)
        if (variants[q] < 0 || variants[q] >= nvar) return fail(MIDBF_ERR_ARG, "unknown variant");
    auto& var = prec == MIDBF_SPLIT_FP16   ? h->fp16_variant
                : prec == MIDBF_SPLIT_BF16 ? h->bf16_variant
                : f64                      ? h->mfma64_variant
                                           : h->mfma_variant;
    for (int q = 0; q < 3; ++q)
        for (int l = 0; l < midbf_plan::VMAXLEV; ++l) var[q][l] = variants[q];
    return MIDBF_OK;
}

midbf_status midbf_profile_enable(midbf_handle h, int on) {
    if (!h) return fail(MIDBF_ERR_ARG, "null handle");
    h->prof.on = on != 0;
    h->prof.by_level = on == 2;
    return MIDBF_OK;
}

midbf_status midbf_profile_read(midbf_handle h, midbf_kernel_time* out, int max_entries, int* count) {
    if (!h || !count || (max_entries > 0 && !out)) return fail(MIDBF_ERR_ARG, "null argument");
    return guarded([&] {
        Profiler& P = h->prof;
        std::vector<midbf_kernel_time> agg;
        for (auto& r : P.recs) {
            MIDBF_HIP(hipEventSynchronize(r.b));
            float ms = 0.f;
            MIDBF_HIP(hipEventElapsedTime(&ms, r.a, r.b));
            auto it = std::find_if(agg.begin(), agg.end(),
                                   [&](const midbf_kernel_time& t) { return r.name == t.name; });
            if (it == agg.end()) {
                midbf_kernel_time t{};
                std::strncpy(t.name, r.name.c_str(), sizeof(t.name) - 1);
                agg.push_back(t);
                it = agg.end() - 1;
            }
            it->launches += 1;
            it->total_ms += ms;
            it->bytes += r.bytes;
            it->stored_bytes += r.stored;
            it->flops += r.flops;
            P.pool.push_back(r.a);
            P.pool.push_back(r.b);
        }
        P.recs.clear();
        *count = (int)agg.size();
        for (int i = 0; i < (int)agg.size() && i < max_entries; ++i) out[i] = agg[i];
    });
}

void midbf_destroy(midbf_handle h) {
    if (h) {
        for (auto& r : h->prof.recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        for (auto e : h->prof.pool) (void)hipEventDestroy(e);
    }
    destroy_plan(h);
}

midbf_status phase_recover(int d, int n, const double* X1, const double* X2, midbf_sample_cb cb, void* user, int r,
                           int q, double tau, uint64_t seed, void* stream, double* U_dev, double* V_dev,
                           phase_recover_info* info) {
    return guarded([&] {
        phase_recover_run(d, n, X1, X2, cb, user, r, q, tau, seed, (hipStream_t)stream, U_dev, V_dev, info);
    });
}

midbf_status phase_recover_points(int d, long long N, const double* X1, const double* X2, midbf_sample_cb cb,
                                  void* user, int r, int q, double tau, uint64_t seed, void* stream, double* U_dev,
                                  double* V_dev, phase_recover_info* info) {
    if (N < 2) return fail(MIDBF_ERR_ARG, "need at least two points");
    return guarded([&] {
        phase_recover_run(d, 0, X1, X2, cb, user, r, q, tau, seed, (hipStream_t)stream, U_dev, V_dev, info, N);
    });
}

midbf_status midbf_recovery_path(const double* pts, long long N, int d, long long root, int* P_out, void* stream) {
    if (!pts || !P_out) return fail(MIDBF_ERR_ARG, "null argument");
    return guarded([&] { recovery_path_points(pts, N, d, root, P_out, (hipStream_t)stream); });
}

const char* midbf_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
