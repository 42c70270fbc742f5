// Many-right-hand-side apply on the matrix cores, FP32 (v_mfma_f32_16x16x4f32)
// or FP64 (v_mfma_f64_16x16x4f64), accumulating in the same precision.
//
// With 64 right-hand sides every factor block becomes a dense complex GEMM,
// C (rows x 64) = A (rows x K) B (K x 64), computed as three real products
// per complex product (Gauss's form):
//     Cr = Ar Br - Ai Bi,   Ci = (Ar + Ai)(Br + Bi) - Ar Br - Ai Bi.
// Lane l of a wave supplies A[l%16][l/16] and B[l/16][l%16] and receives
// D[4(l/16)+v][l%16] (FP32) or D[l/16+4v][l%16] (FP64), v < 4 (both checked
// on the device).  A (the factor) streams
// from HBM exactly once per launch; B (the level vectors, gathered through
// the candidate permutation) is staged through LDS in chunks of KC rows and
// shared by the four waves; each wave owns up to MTW 16-row tiles x 64
// columns of C.  (MTW, KC, pipelining) come in a few variants that the
// autotuner (midbf_tune) times on the factorization at hand.
//   up     (column side, going up):  C = y[id] (k rows), A = T (k x (n-k), column-major),
//          B = candidate rows perm[k..n), plus the skeleton rows perm[0..k).
//   down   (row side, going down):   C = candidate rows perm[k..n), A = T^T (T
//          row-major k x (n-k)), B = z[id]; each ID writes its contribution to
//          a scratch block, then the 2^d contributions of a group are summed in
//          a fixed order (no atomics, bitwise reproducible).
//   middle: C = z rows, A = S (column-major), B = y rows.
#include <type_traits>

#include "apply.h"
#include "mfma.h"

namespace midbf {

namespace {

// The real type of a path: its complex element, 4-wide accumulator and MFMA.
template <class T> struct Real;
template <> struct Real<float> {
    typedef float2 C2;
    typedef float acc4 __attribute__((ext_vector_type(4)));
    static __device__ acc4 mfma(float a, float b, acc4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    // row of the 16 x 16 result held in register v of a lane in row group lk = l/16
    static __device__ int out_row(int lk, int v) { return 4 * lk + v; }
};
template <> struct Real<double> {
    typedef double2 C2;
    typedef double acc4 __attribute__((ext_vector_type(4)));
    static __device__ acc4 mfma(double a, double b, acc4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // the FP64 instruction interleaves the row groups instead
    static __device__ int out_row(int lk, int v) { return lk + 4 * v; }
};
template <class T> __device__ inline typename Real<T>::C2 c2(T x, T y) {
    typename Real<T>::C2 v;
    v.x = x;
    v.y = y;
    return v;
}

constexpr int MT = 256;          // threads per workgroup (up, down)
constexpr int MW = MT / 64;      // waves
constexpr int NRHS = MFMA_NRHS;  // columns per workgroup (4 tiles of 16)

// One k-step of 4 for every (row tile, column tile) of a wave, with three real
// products per complex product (Gauss): p1 += Ar Br, p2 += Ai Bi,
// p3 += (Ar + Ai)(Br + Bi); then Cr = p1 - p2 and Ci = p3 - p1 - p2
// (finish_gauss).  Each sweep issues independent MFMAs back to back.
template <class T, int MTW, int NTC, class Acc = typename Real<T>::acc4, class C2 = typename Real<T>::C2>
__device__ inline void kstep(Acc (&p1)[MTW][4], Acc (&p2)[MTW][4], Acc (&p3)[MTW][4], const C2 (&a)[MTW],
                             const C2 (&b)[4], int ntiles) {
    T as[MTW], bs[4];
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) as[mt] = a[mt].x + a[mt].y;
#pragma unroll
    for (int nt = 0; nt < NTC; ++nt) bs[nt] = b[nt].x + b[nt].y;
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) {
        if (mt < ntiles) {
#pragma unroll
            for (int nt = 0; nt < NTC; ++nt) {
                p1[mt][nt] = Real<T>::mfma(a[mt].x, b[nt].x, p1[mt][nt]);
                p2[mt][nt] = Real<T>::mfma(a[mt].y, b[nt].y, p2[mt][nt]);
                p3[mt][nt] = Real<T>::mfma(as[mt], bs[nt], p3[mt][nt]);
            }
        }
    }
}

template <class Acc, int MTW, int NTC>
__device__ inline void finish_gauss(Acc (&cr)[MTW][4], Acc (&ci)[MTW][4], const Acc (&p3)[MTW][4]) {
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
        for (int nt = 0; nt < NTC; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const auto r = cr[mt][nt][v] - ci[mt][nt][v];
                ci[mt][nt][v] = p3[mt][nt][v] - cr[mt][nt][v] - ci[mt][nt][v];
                cr[mt][nt][v] = r;
            }
}


template <int MTW_, int KC_, bool PIPE_, int NT_ = MT, int NTC_ = 4, class T_ = float>
struct Cfg {
    typedef T_ T;                         // real type (float or double)
    typedef typename Real<T_>::C2 C2;
    typedef typename Real<T_>::acc4 Acc;
    static constexpr int MTW = MTW_;      // 16-row tiles per wave
    static constexpr int KC = KC_;        // K rows per LDS chunk
    static constexpr bool PIPE = PIPE_;   // chunk-deep register prefetch + double-buffered LDS
    static constexpr int NT = NT_;        // threads per workgroup
    static constexpr int NTC = NTC_;      // 16-column tiles per workgroup (4: 64 right-hand sides)
    static constexpr int W = NTC * 16;    // right-hand sides per workgroup
    static constexpr int ROUND = NT / 64 * MTW * 16;
};

// The same tiling with one 16-column tile (few right-hand sides).
template <class C> using Narrow = Cfg<C::MTW, C::KC, C::PIPE, C::NT, 1, typename C::T>;

// Rows [base, base + 16 MTW) of C (+)= A B for one wave.  A is column-major
// with leading dimension M, or with ADJ the conjugate of a row-major block with
// leading dimension K (A[row][col] = conj(F[row K + col]): the adjoint passes
// read the forward factors this way); brow(j, r) returns B[j][r] (j < K, r < nr).
// Every thread of the workgroup must call this (it synchronizes).
//   PIPE: the wave's A fragments of chunk c+1 and this thread's B elements of
//   chunk c+1 are loaded into registers while chunk c is multiplied from the
//   other register set and the other LDS buffer; one barrier per chunk.
//   otherwise: one LDS buffer, A prefetched one k-step ahead.
template <class C, int NT, bool ADJ = false, class BRow>
__device__ void gemm_rows(typename C::Acc (&cr)[C::MTW][4], typename C::Acc (&ci)[C::MTW][4],
                          const typename C::C2* __restrict__ A, int M, int K, int base, BRow brow, int nr,
                          typename C::C2* sB) {
    using T = typename C::T;
    using C2 = typename C::C2;
    using Acc = typename C::Acc;
    constexpr int MTW = C::MTW, KC = C::KC, W = C::W, NTC = C::NTC;
    constexpr int BPT = (KC * W + NT - 1) / NT;   // B elements staged per thread and chunk
    const int tid = threadIdx.x, l = tid & 63, lr = l & 15, lk = l >> 4;
    const int ntl = base < M ? min(MTW, (M - base + 15) / 16) : 0;
    const int nch = (K + KC - 1) / KC;
    if (nch == 0) return;
    // cr, ci enter as zero and collect Ar Br and Ai Bi; p3 the sum product
    Acc p3[MTW][4];
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) p3[mt][nt] = Acc{0, 0, 0, 0};
    auto loadA1 = [&](int col, C2 (&dst)[MTW]) {
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
            const int row = base + mt * 16 + lr;
            if constexpr (ADJ) {
                const C2 v = (mt < ntl && col < K && row < M) ? A[(long long)row * K + col] : c2<T>(0, 0);
                dst[mt] = c2<T>(v.x, -v.y);
            } else {
                dst[mt] = (mt < ntl && col < K && row < M) ? A[(long long)col * M + row] : c2<T>(0, 0);
            }
        }
    };
    C2 bt[BPT];
    auto loadB = [&](int c0) {
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            const int e = tid + q * NT, jj = e / W, r = e - jj * W, j = c0 + jj;
            bt[q] = (e < KC * W && j < K && r < nr) ? brow(j, r) : c2<T>(0, 0);
        }
    };
    auto storeB = [&](int buf) {
#pragma unroll
        for (int q = 0; q < BPT; ++q)
            if (tid + q * NT < KC * W) sB[buf * KC * W + tid + q * NT] = bt[q];
    };
    if constexpr (C::PIPE) {
        C2 acur[KC / 4][MTW], anext[KC / 4][MTW];
#pragma unroll
        for (int ks = 0; ks < KC / 4; ++ks) loadA1(ks * 4 + lk, acur[ks]);
        loadB(0);
        __syncthreads();          // the previous user of sB is done
        storeB(0);
        __syncthreads();
        for (int c = 0; c < nch; ++c) {
            const bool more = c + 1 < nch;
            if (more) {
#pragma unroll
                for (int ks = 0; ks < KC / 4; ++ks) loadA1((c + 1) * KC + ks * 4 + lk, anext[ks]);
                loadB((c + 1) * KC);
            }
            const C2* sb = sB + (c & 1) * KC * W;
            if (ntl > 0) {
#pragma unroll
                for (int ks = 0; ks < KC / 4; ++ks) {
                    C2 bv[4];
#pragma unroll
                    for (int nt = 0; nt < NTC; ++nt) bv[nt] = sb[(ks * 4 + lk) * W + nt * 16 + lr];
                    kstep<T, MTW, NTC>(cr, ci, p3, acur[ks], bv, ntl);
                }
            }
            if (more) {
                storeB((c + 1) & 1);
#pragma unroll
                for (int ks = 0; ks < KC / 4; ++ks)
#pragma unroll
                    for (int mt = 0; mt < MTW; ++mt) acur[ks][mt] = anext[ks][mt];
            }
            __syncthreads();
        }
        finish_gauss<Acc, MTW, NTC>(cr, ci, p3);
    } else {
        for (int c = 0; c < nch; ++c) {
            loadB(c * KC);
            __syncthreads();
            storeB(0);
            __syncthreads();
            if (ntl > 0) {
                C2 an[MTW];
                loadA1(c * KC + lk, an);
#pragma unroll 2
                for (int ks = 0; ks < KC / 4; ++ks) {
                    C2 a[MTW];
#pragma unroll
                    for (int mt = 0; mt < MTW; ++mt) a[mt] = an[mt];
                    if (ks + 1 < KC / 4) loadA1(c * KC + (ks + 1) * 4 + lk, an);
                    C2 bv[4];
#pragma unroll
                    for (int nt = 0; nt < NTC; ++nt) bv[nt] = sB[(ks * 4 + lk) * W + nt * 16 + lr];
                    kstep<T, MTW, NTC>(cr, ci, p3, a, bv, ntl);
                }
            }
        }
        __syncthreads();
        finish_gauss<Acc, MTW, NTC>(cr, ci, p3);
    }
}

template <class Acc, int MTW>
__device__ inline void zero_acc(Acc (&cr)[MTW][4], Acc (&ci)[MTW][4]) {
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) { cr[mt][nt] = Acc{0, 0, 0, 0}; ci[mt][nt] = Acc{0, 0, 0, 0}; }
}

// Row numbers of a group's candidate vector in the previous level buffer
// (or points of the leaf when s == 0: the lattice box's, or with a slot table
// the leaf's first nleaf slots).
template <int NT>
__device__ int candidate_rows(int* crow, const ApplyGeom& G, int s, long long a, long long partner, long long Ps,
                              const int* k_prev, const long long* yoff_prev, const int* slot = nullptr,
                              int nleaf = 0) {
    if (s == 0) {
        if (slot) {
            for (int c = threadIdx.x; c < nleaf; c += NT) crow[c] = slot[a * G.n0 + c];
            return nleaf;
        }
        int origin[3];
        node_origin(a, G.L, G.d, G.n, origin);
        for (int c = threadIdx.x; c < G.n0; c += NT) crow[c] = (int)box_point(origin, G.leaf, c, G.d, G.n);
        return G.n0;
    }
    int len[MAX_P];
    long long off[MAX_P];
    child_pieces(len, off, G.P, a, partner, Ps, k_prev, yoff_prev);
    int start = 0;
#pragma unroll
    for (int t = 0; t < MAX_P; ++t) {
        if (t < G.P) {
            for (int c = threadIdx.x; c < len[t]; c += NT) crow[start + c] = (int)(off[t] + c);
            start += len[t];
        }
    }
    return start;
}

// element (row, rhs) of a level buffer (row-major, nrhs wide) or of an
// external column-major block (s == 0)
template <class C2> __device__ inline C2 load_vec(bool ext, const C2* p, long long ld, int nrhs, int row, int r) {
    return ext ? p[(long long)r * ld + row] : p[(long long)row * nrhs + r];
}
template <class C2> __device__ inline C2* vec_ptr(bool ext, C2* p, long long ld, int nrhs, int row, int r) {
    return ext ? p + (long long)r * ld + row : p + (long long)row * nrhs + r;
}

// Blocks of 32 consecutive IDs spread over the eight XCDs so that the four
// IDs of one group run on the same XCD (shared L2 for their candidate vector).
__device__ inline long long xcd_group_order(long long b, long long nid, int P) {
    if (P != 4 || (nid & 31) != 0) return b;
    const long long x = b & 7, t = (b >> 3) & 3, q = b >> 5;
    return ((q << 3) + x) * 4 + t;
}

// ADJ: the adjoint going up (row side, A = conj(T) with T row-major k x (n-k)).
template <class C, bool ADJ = false>
__global__ __launch_bounds__(C::NT) void up_mfma(UpArgs A, long long nid) {
    constexpr int MTW = C::MTW;
    using T = typename C::T;
    using C2 = typename C::C2;
    using Acc = typename C::Acc;
    extern __shared__ int dyn_rows[];          // ncand_max candidate rows, then as many source rows
    int* crow = dyn_rows;
    int* srcrow = dyn_rows + A.ncand_max;
    __shared__ C2 sB[(C::PIPE ? 2 : 1) * C::KC * C::W];
    const long long id = xcd_group_order(blockIdx.x, nid, A.G.P);
    const long long g = id / A.G.P;
    const long long a = g / A.Ps, ap = g - (g / A.Ps) * A.Ps;
    const int r0 = blockIdx.y * C::W;
    const int nr = min(C::W, A.nrhs - r0);
    candidate_rows<C::NT>(crow, A.G, A.s, a, ap, A.Ps, A.k_prev, A.yoff_prev, A.lev.slot, A.lev.n[g * A.G.P]);
    // the leaves read the caller's block, or its row-major copy (A.ext null)
    const bool ext = A.s == 0 && A.ext;
    const C2* xin = ext ? (const C2*)A.ext : (const C2*)A.in;
    C2* out = (C2*)A.out;
    const int k = A.lev.k[id], nred = A.lev.n[id] - k;
    const int* perm = A.lev.perm + A.lev.perm_off[id];
    const C2* Tb = (const C2*)A.lev.T[id];
    const long long yo = A.lev.y_off[id];
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
    __syncthreads();
    for (int j = tid; j < nred; j += C::NT) srcrow[j] = crow[perm[k + j]];
    __syncthreads();
    auto brow = [&](int j, int r) { return load_vec(ext, xin, A.ld, A.nrhs, srcrow[j], r0 + r); };
    for (int m0 = 0; m0 < k; m0 += C::ROUND) {
        const int base = m0 + wave * MTW * 16;
        Acc cr[MTW][4], ci[MTW][4];
        zero_acc<Acc, MTW>(cr, ci);
        gemm_rows<C, C::NT, ADJ>(cr, ci, Tb, k, nred, base, brow, nr, sB);
        // C + skeleton rows of the candidate vector.  Per 16-row tile the
        // skeleton inputs are loaded at in-range addresses (row 0 / column 0
        // outside the block) so that a lane's loads issue together.
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
            C2 sv[4][C::NTC];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = base + mt * 16 + Real<T>::out_row(lk, v);
                const int src = crow[perm[row < k ? row : 0]];
#pragma unroll
                for (int nt = 0; nt < C::NTC; ++nt) {
                    const int r = nt * 16 + lr;
                    sv[v][nt] = load_vec(ext, xin, A.ld, A.nrhs, src, r0 + (r < nr ? r : 0));
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = base + mt * 16 + Real<T>::out_row(lk, v);
                if (row < k) {
#pragma unroll
                    for (int nt = 0; nt < C::NTC; ++nt) {
                        const int r = nt * 16 + lr;
                        if (r < nr)
                            out[(yo + row) * A.nrhs + r0 + r] =
                                c2<T>(cr[mt][nt][v] + sv[v][nt].x, ci[mt][nt][v] + sv[v][nt].y);
                    }
                }
            }
        }
    }
}

// Going down, one workgroup per decomposition: its contribution to every
// candidate row of its group -- z on the skeleton rows, T^T z on the
// redundant rows -- goes to the scratch block scr[perm_off[id] + position].
// ADJ: the adjoint going down (column side, A = T^H with T column-major k x (n-k)).
template <class C, bool ADJ = false>
__global__ __launch_bounds__(C::NT) void down_mfma(DownArgs A, long long nid, typename C::C2* scr) {
    constexpr int MTW = C::MTW;
    using T = typename C::T;
    using C2 = typename C::C2;
    using Acc = typename C::Acc;
    __shared__ C2 sB[(C::PIPE ? 2 : 1) * C::KC * C::W];
    const long long id = xcd_group_order(blockIdx.x, nid, A.G.P);
    const int r0 = blockIdx.y * C::W;
    const int nr = min(C::W, A.nrhs - r0);
    const C2* zin = (const C2*)A.in;
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
    const int k = A.lev.k[id], nred = A.lev.n[id] - k;
    const int* perm = A.lev.perm + A.lev.perm_off[id];
    const C2* Tb = (const C2*)A.lev.T[id];
    const long long yo = A.lev.y_off[id];
    C2* w = scr + A.lev.perm_off[id] * A.nrhs;
    for (int e = tid; e < k * C::W; e += C::NT) {
        const int i = e / C::W, r = e - i * C::W;
        if (r < nr) w[(long long)perm[i] * A.nrhs + r0 + r] = zin[(yo + i) * A.nrhs + r0 + r];
    }
    const C2* z = zin + yo * A.nrhs + r0;
    auto brow = [&](int i, int r) { return z[(long long)i * A.nrhs + r]; };
    for (int m0 = 0; m0 < nred; m0 += C::ROUND) {
        const int base = m0 + wave * MTW * 16;
        Acc cr[MTW][4], ci[MTW][4];
        zero_acc<Acc, MTW>(cr, ci);
        gemm_rows<C, C::NT, ADJ>(cr, ci, Tb, nred, k, base, brow, nr, sB);
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = base + mt * 16 + Real<T>::out_row(lk, v);
                if (row < nred) {
                    C2* d = w + (long long)perm[k + row] * A.nrhs + r0;
#pragma unroll
                    for (int nt = 0; nt < C::NTC; ++nt) {
                        const int r = nt * 16 + lr;
                        if (r < nr) d[r] = c2<T>(cr[mt][nt][v], ci[mt][nt][v]);
                    }
                }
            }
        }
    }
}

// The 2^d contributions of a group summed in a fixed order and written to
// the candidate rows (previous level buffer, or the leaf's lattice points).
template <class C2>
__global__ __launch_bounds__(MT) void down_sum(DownArgs A, const C2* scr) {
    extern __shared__ int crow[];               // ncand_max candidate rows
    __shared__ long long base[8];
    const long long g = blockIdx.x;
    const long long a = g / A.Ps, bp = g - (g / A.Ps) * A.Ps;
    const int r0 = blockIdx.y * NRHS;
    const int nr = min(NRHS, A.nrhs - r0);
    const int ncand = candidate_rows<MT>(crow, A.G, A.s, a, bp, A.Ps, A.k_prev, A.yoff_prev, A.lev.slot,
                                         A.lev.n[g * A.G.P]);
    if (threadIdx.x < A.G.P) base[threadIdx.x] = A.lev.perm_off[g * A.G.P + threadIdx.x] * A.nrhs + r0;
    __syncthreads();
    const bool ext = A.s == 0 && A.ext;
    C2* outp = ext ? (C2*)A.ext : (C2*)A.out;
    // complex64: two right-hand sides per thread (16-byte loads) when the row stride allows it
    const bool pairs = sizeof(C2) == 8 && (A.nrhs % 2 == 0) && (nr % 2 == 0) && !ext;
    if constexpr (sizeof(C2) == 8) if (pairs) {
        const int half = nr / 2;
        for (int e = threadIdx.x; e < ncand * half; e += MT) {
            const int p = e / half, r = 2 * (e - p * half);
            float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
            float4 v[8];
#pragma unroll
            for (int t = 0; t < 8; ++t)       // P <= 8; the P loads issue together
                if (t < A.G.P) v[t] = *reinterpret_cast<const float4*>(scr + base[t] + (long long)p * A.nrhs + r);
#pragma unroll
            for (int t = 0; t < 8; ++t)
                if (t < A.G.P) { acc.x += v[t].x; acc.y += v[t].y; acc.z += v[t].z; acc.w += v[t].w; }
            *reinterpret_cast<float4*>(outp + (long long)crow[p] * A.nrhs + r0 + r) = acc;
        }
        return;
    }
    for (int e = threadIdx.x; e < ncand * NRHS; e += MT) {
        const int p = e / NRHS, r = e - p * NRHS;
        if (r >= nr) continue;
        decltype(C2::x) sx = 0, sy = 0;
        C2 v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t)           // P <= 8; the P loads issue together
            if (t < A.G.P) v[t] = scr[base[t] + (long long)p * A.nrhs + r];
#pragma unroll
        for (int t = 0; t < 8; ++t)
            if (t < A.G.P) {
                sx += v[t].x;
                sy += v[t].y;
            }
        C2 o;
        o.x = sx;
        o.y = sy;
        *vec_ptr(ext, outp, A.ld, A.nrhs, crow[p], r0 + r) = o;
    }
}

// ADJ: x = S^H z; the caller swaps the block shapes (nr <-> nc) and the input and
// output piece tables, so M = columns of S and K = its rows.
template <class C, bool ADJ = false>
__global__ __launch_bounds__(C::NT) void middle_mfma(MidArgs A) {
    constexpr int MTW = C::MTW;
    using T = typename C::T;
    using C2 = typename C::C2;
    using Acc = typename C::Acc;
    extern __shared__ int dyn_rows[];          // in_max input rows, then out_max output rows
    int* crow_in = dyn_rows;
    int* crow_out = dyn_rows + A.in_max;
    __shared__ C2 sB[(C::PIPE ? 2 : 1) * C::KC * C::W];
    const long long bi = blockIdx.x / A.mchunks;
    const int chunk = (int)(blockIdx.x - bi * A.mchunks);
    const int r0 = blockIdx.y * C::W;
    const int nr = min(C::W, A.nrhs - r0);
    const int M = A.nr[bi], K = A.nc[bi];
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
    middle_rows<C::NT>(crow_in, crow_out, A, bi);
    const C2* xin = (const C2*)A.in;
    C2* zout = (C2*)A.out;
    const C2* S = (const C2*)A.S + A.off[bi];
    __syncthreads();
    auto brow = [&](int j, int r) { return xin[(long long)crow_in[j] * A.nrhs + r0 + r]; };
    // rows of this workgroup: a run of whole rounds
    const int per = ((M + A.mchunks - 1) / A.mchunks + C::ROUND - 1) / C::ROUND * C::ROUND;
    const int mlo = chunk * per, mhi = min(M, mlo + per);
    for (int m0 = mlo; m0 < mhi; m0 += C::ROUND) {
        const int base = m0 + wave * MTW * 16;
        Acc cr[MTW][4], ci[MTW][4];
        zero_acc<Acc, MTW>(cr, ci);
        gemm_rows<C, C::NT, ADJ>(cr, ci, S, M, K, base, brow, nr, sB);
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = base + mt * 16 + Real<T>::out_row(lk, v);
                if (row < M) {
                    const long long dst = crow_out[row];
#pragma unroll
                    for (int nt = 0; nt < C::NTC; ++nt) {
                        const int r = nt * 16 + lr;
                        if (r < nr) zout[dst * A.nrhs + r0 + r] = c2<T>(cr[mt][nt][v], ci[mt][nt][v]);
                    }
                }
            }
        }
    }
}

using V0 = Cfg<3, 32, false>;
using V1 = Cfg<2, 32, false>;
using V2 = Cfg<3, 16, true>;
using V3 = Cfg<2, 16, true>;
using V4 = Cfg<4, 32, false>;
using V5 = Cfg<2, 16, true, 512>;
using V6 = Cfg<1, 16, true, 512>;
using V7 = Cfg<2, 32, false, 512>;
using V8 = Cfg<1, 16, true, 1024>;
using V9 = Cfg<1, 32, true, 512>;

template <class C>
void launch_variant(LevelKernel which, const void* args, long long count, int nrhs, void* scratch, hipStream_t s) {
    const dim3 grid((unsigned)count, (nrhs + C::W - 1) / C::W);
    switch (which) {
        case LevelKernel::Up:
        case LevelKernel::AdjUp: {
            const UpArgs& a = *(const UpArgs*)args;
            if (which == LevelKernel::AdjUp)
                hipLaunchKernelGGL((up_mfma<C, true>), grid, dim3(C::NT), 2 * sizeof(int) * a.ncand_max, s, a, count);
            else
                hipLaunchKernelGGL(up_mfma<C>, grid, dim3(C::NT), 2 * sizeof(int) * a.ncand_max, s, a, count);
            break;
        }
        case LevelKernel::Down:
            hipLaunchKernelGGL(down_mfma<C>, grid, dim3(C::NT), 0, s, *(const DownArgs*)args, count,
                               (typename C::C2*)scratch);
            break;
        case LevelKernel::AdjDown:
            hipLaunchKernelGGL((down_mfma<C, true>), grid, dim3(C::NT), 0, s, *(const DownArgs*)args, count,
                               (typename C::C2*)scratch);
            break;
        case LevelKernel::DownSum: {
            const DownArgs& a = *(const DownArgs*)args;
            const dim3 sgrid((unsigned)count, (nrhs + NRHS - 1) / NRHS);     // its own 64-column tiling
            hipLaunchKernelGGL(down_sum<typename C::C2>, sgrid, dim3(MT), sizeof(int) * a.ncand_max, s, a,
                               (const typename C::C2*)scratch);
            break;
        }
        case LevelKernel::Middle:
        case LevelKernel::AdjMiddle: {
            const MidArgs& a = *(const MidArgs*)args;
            MIDBF_CHECK(a.mchunks >= 1, MIDBF_ERR_ARG, "middle row split must be >= 1");
            const dim3 mgrid((unsigned)(count * a.mchunks), grid.y);
            if (which == LevelKernel::AdjMiddle)
                hipLaunchKernelGGL((middle_mfma<C, true>), mgrid, dim3(C::NT), sizeof(int) * (a.in_max + a.out_max),
                                   s, a);
            else
                hipLaunchKernelGGL(middle_mfma<C>, mgrid, dim3(C::NT), sizeof(int) * (a.in_max + a.out_max), s, a);
            break;
        }
        default:
            throw Error(MIDBF_ERR_UNIMPLEMENTED, "no matrix-core kernel for this level kind");
    }
    MIDBF_HIP(hipGetLastError());
}

// Row-major N x nrhs -> external column-major block, in 64 x 64 tiles through
// LDS (rows padded to 65 entries: the column reads of each half-wave touch
// distinct banks); both global sides are coalesced.
// TO_EXT: row-major copy -> external column-major block; otherwise the reverse.
template <class C2, bool TO_EXT = true>
__global__ __launch_bounds__(256) void transpose_kernel(TransposeArgs A) {
    __shared__ C2 t[64][65];
    const long long p0 = (long long)blockIdx.x * 64;
    const int r0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const C2* src = (const C2*)A.src;
    C2* dst = (C2*)A.dst;
    // loads at in-range addresses (clamped row and column), so that a thread's
    // sixteen loads issue together; only the stores are guarded
    // split 16-bit applies: the copy of the input is scaled, the output
    // unscaled, per right-hand side (SplitScale; complex64 only)
    constexpr bool SC = std::is_same_v<C2, float2>;
    if constexpr (TO_EXT) {
#pragma unroll
        for (int pp = ty; pp < 64; pp += 4) {
            const long long p = min(p0 + pp, A.N - 1);
            const int r = min(r0 + tx, A.nrhs - 1);
            t[pp][tx] = src[p * A.nrhs + r];
        }
        __syncthreads();
        for (int rr = ty; rr < 64; rr += 4) {
            const long long p = p0 + tx;
            const int r = r0 + rr;
            if (p < A.N && r < A.nrhs) {
                C2 v = t[tx][rr];
                if constexpr (SC) {
                    const float f = split_scale_of(A.sc, r, -1);
                    v = make_float2(v.x * f, v.y * f);
                }
                dst[(long long)r * A.ld + p] = v;
            }
        }
    } else {
#pragma unroll
        for (int rr = ty; rr < 64; rr += 4) {
            const long long p = min(p0 + tx, A.N - 1);
            const int r = min(r0 + rr, A.nrhs - 1);
            t[tx][rr] = src[(long long)r * A.ld + p];
        }
        __syncthreads();
        float f = 1.f;
        if constexpr (SC) f = split_scale_of(A.sc, min(r0 + tx, A.nrhs - 1), 1);
        for (int pp = ty; pp < 64; pp += 4) {
            const long long p = p0 + pp;
            const int r = r0 + tx;
            if (p < A.N && r < A.nrhs) {
                C2 v = t[pp][tx];
                if constexpr (SC) v = make_float2(v.x * f, v.y * f);
                dst[p * A.nrhs + r] = v;
            }
        }
    }
}

// The first up step when no leaf decomposition has redundant points: y rows of
// partner t are x at the leaf points perm_t[i].  The leaf's 64-column block of
// x is read once (runs of consecutive lattice points, coalesced per column)
// into LDS and written as whole rows for each of the P partners.
__global__ __launch_bounds__(256) void up_leaf_copy(UpArgs A) {
    extern __shared__ __align__(16) float2 xs[];      // n0 x (NRHS + 1)
    __shared__ int crow[64];                          // n0 <= 64 (checked at launch)
    const long long g = blockIdx.x;
    const int r0 = blockIdx.y * NRHS;
    const int nr = min(NRHS, A.nrhs - r0);
    const int n0 = candidate_rows<256>(crow, A.G, 0, g, 0, 1, nullptr, nullptr);
    __syncthreads();
    const float2* x = (const float2*)A.ext;
    for (int e = threadIdx.x; e < n0 * NRHS; e += 256) {
        const int r = e / n0, c = e - r * n0;
        float2 v = make_float2(0.f, 0.f);
        if (r < nr) {
            v = x[(long long)(r0 + r) * A.ld + crow[c]];
            const float f = split_scale_of(A.sc, r0 + r, 1);      // split 16-bit: the scaled input copy
            v = make_float2(v.x * f, v.y * f);
        }
        xs[c * (NRHS + 1) + r] = v;
    }
    __syncthreads();
    float2* out = (float2*)A.out;
    for (int t = 0; t < A.G.P; ++t) {
        const long long id = g * A.G.P + t;
        const int k = A.lev.k[id];
        const int* perm = A.lev.perm + A.lev.perm_off[id];
        const long long yo = A.lev.y_off[id];
        for (int e = threadIdx.x; e < k * NRHS; e += 256) {
            const int i = e / NRHS, r = e - i * NRHS;
            if (r < nr) out[(yo + i) * A.nrhs + r0 + r] = xs[perm[i] * (NRHS + 1) + r];
        }
    }
}

}  // namespace

void launch_up_leaf_copy(const UpArgs& A, long long groups, int nrhs, hipStream_t s) {
    MIDBF_CHECK(A.G.n0 <= 64 && A.ext, MIDBF_ERR_ARG, "leaf copy needs the external block and n0 <= 64");
    const size_t smem = (size_t)A.G.n0 * (NRHS + 1) * sizeof(float2);
    MIDBF_CHECK(smem <= 64 * 1024, MIDBF_ERR_UNIMPLEMENTED, "leaf block exceeds the copy kernel's LDS");
    const dim3 grid((unsigned)groups, (nrhs + NRHS - 1) / NRHS);
    hipLaunchKernelGGL(up_leaf_copy, grid, dim3(256), smem, s, A);
    MIDBF_HIP(hipGetLastError());
}

void launch_transpose(const TransposeArgs& A, bool fp64, hipStream_t s) {
    const dim3 grid((unsigned)((A.N + 63) / 64), (unsigned)((A.nrhs + 63) / 64));
    if (fp64) hipLaunchKernelGGL(transpose_kernel<double2>, grid, dim3(256), 0, s, A);
    else hipLaunchKernelGGL(transpose_kernel<float2>, grid, dim3(256), 0, s, A);
    MIDBF_HIP(hipGetLastError());
}

void launch_transpose_in(const TransposeArgs& A, hipStream_t s) {
    const dim3 grid((unsigned)((A.N + 63) / 64), (unsigned)((A.nrhs + 63) / 64));
    hipLaunchKernelGGL((transpose_kernel<float2, false>), grid, dim3(256), 0, s, A);
    MIDBF_HIP(hipGetLastError());
}

namespace {
// FP64: one 16-row tile per wave (three 4-wide FP64 accumulators per column tile).
using D0 = Cfg<1, 16, true, 512, 4, double>;
using D1 = Cfg<1, 16, false, 512, 4, double>;
using D2 = Cfg<1, 16, true, 256, 4, double>;
using D3 = Cfg<1, 32, false, 256, 4, double>;
using D4 = Cfg<1, 32, true, 256, 4, double>;

// 64 right-hand sides per workgroup, or one 16-column tile when there are at
// most 16 (no matrix-core work on empty columns).
template <class C>
void launch_width(LevelKernel which, const void* args, long long count, int nrhs, void* scratch, hipStream_t s) {
    if (nrhs <= 16) launch_variant<Narrow<C>>(which, args, count, nrhs, scratch, s);
    else launch_variant<C>(which, args, count, nrhs, scratch, s);
}
}  // namespace

void launch_mfma_kernel(LevelKernel which, int variant, const void* args, long long count, int nrhs, void* scratch,
                        hipStream_t s, bool fp64) {
    if (fp64) {
        switch (variant) {
            case 0: launch_width<D0>(which, args, count, nrhs, scratch, s); break;
            case 1: launch_width<D1>(which, args, count, nrhs, scratch, s); break;
            case 2: launch_width<D2>(which, args, count, nrhs, scratch, s); break;
            case 3: launch_width<D3>(which, args, count, nrhs, scratch, s); break;
            case 4: launch_width<D4>(which, args, count, nrhs, scratch, s); break;
            default: throw Error(MIDBF_ERR_ARG, "unknown FP64 matrix-core variant");
        }
        return;
    }
    switch (variant) {
        case 0: launch_width<V0>(which, args, count, nrhs, scratch, s); break;
        case 1: launch_width<V1>(which, args, count, nrhs, scratch, s); break;
        case 2: launch_width<V2>(which, args, count, nrhs, scratch, s); break;
        case 3: launch_width<V3>(which, args, count, nrhs, scratch, s); break;
        case 4: launch_width<V4>(which, args, count, nrhs, scratch, s); break;
        case 5: launch_width<V5>(which, args, count, nrhs, scratch, s); break;
        case 6: launch_width<V6>(which, args, count, nrhs, scratch, s); break;
        case 7: launch_width<V7>(which, args, count, nrhs, scratch, s); break;
        case 8: launch_width<V8>(which, args, count, nrhs, scratch, s); break;
        case 9: launch_width<V9>(which, args, count, nrhs, scratch, s); break;
        default: throw Error(MIDBF_ERR_ARG, "unknown matrix-core variant");
    }
}

}  // namespace midbf
