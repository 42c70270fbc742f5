// Split 16-bit matrix-core apply (complex64 vectors, FP32 accumulation), with
// E = bf16 or fp16.
//
// Every factor entry and every vector entry x is split into two 16-bit values,
// hi = E(x) and lo = E(x - hi), and each real product uses three products
// hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_{bf16,f16} (lane l supplies
// A[l%16][8(l/16)+i] and B[8(l/16)+i][l%16], i < 8; checked on the device).
// bf16 keeps FP32's range with ~2^-16 relative error per split value; fp16
// keeps ~2^-22 but needs |x| < 65504 (and loses digits below ~6e-5 in lo).
// A complex product costs 12 MFMAs:
//     Cr += Ar Br - Ai Bi,  Ci += Ar Bi + Ai Br,  each real product split three ways.
//
// Factors are stored as MFMA fragments: a 16-row x 32-column tile of A is
// 64 lanes x (re_hi[8], im_hi[8], re_lo[8], im_lo[8]) bf16 = 4 KB, so one wave
// loads a whole tile with four fully coalesced 16-byte loads per lane.  Tiles of
// one block are stored row-tile major (all K tiles of row tile 0, then row tile 1...).
// B (the level vectors) is split on the fly while it is staged through LDS in
// the same fragment order.
#include <algorithm>
#include <type_traits>

#include "apply.h"
#include "mfma.h"

namespace midbf {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef int intx4 __attribute__((ext_vector_type(4)));

// The two 16-bit element types of the split (bf16: 8-bit mantissa, wide
// range; fp16: 11-bit mantissa, |x| < 65504) and their 8-wide MFMA operands.
template <class E> struct Split16;
template <> struct Split16<__bf16> {
    typedef __bf16 v8 __attribute__((ext_vector_type(8)));
};
template <> struct Split16<_Float16> {
    typedef _Float16 v8 __attribute__((ext_vector_type(8)));
};
template <class E> using V8 = typename Split16<E>::v8;

__device__ inline floatx4 mfma16(V8<__bf16> a, V8<__bf16> b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ inline floatx4 mfma16(V8<_Float16> a, V8<_Float16> b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

constexpr int NRHS = MFMA_NRHS;
constexpr int KT = 32;                       // K per tile / per chunk
constexpr int CROW_MAX = BF16_CROW_MAX;

template <class E> struct Frag {
    V8<E> rh, ih, rl, il;
};

// One fragment tile staged in LDS, plane-major: the 64 lanes' 16-byte pieces
// of each plane are contiguous, so a wave's ds_read_b128 / ds_write_b128 of
// one plane touches consecutive banks (the lane-major Frag order would put
// the lanes 64 bytes apart, a four-way bank conflict).
template <class E> struct LFrag {
    V8<E> rh[64], ih[64], rl[64], il[64];
};

template <class E> __device__ inline Frag<E> lds_frag(const LFrag<E>* t, int lane) {
    Frag<E> f;
    f.rh = t->rh[lane];
    f.ih = t->ih[lane];
    f.rl = t->rl[lane];
    f.il = t->il[lane];
    return f;
}

typedef unsigned uintx4 __attribute__((ext_vector_type(4)));

// fp16 hi and lo parts of two FP32 values a, b, each packed as a pair (a in
// the low half): hi = fp16(x) (one v_cvt_pk_f16_f32), lo = fp16(x - hi) by one
// mixed-precision FMA per value (v_fma_mixlo / mixhi_f16: -hi as fp16 source
// times 1 plus x as FP32 source, rounded once to fp16).  x - hi is exact in
// FP32, so lo is bit for bit the two-conversion result, in three
// instructions per pair instead of eight.
__device__ inline void split_pair_f16(float a, float b, unsigned& hi, unsigned& lo) {
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    hi = __builtin_bit_cast(unsigned, h2{(_Float16)a, (_Float16)b});
    unsigned r;
    asm("v_fma_mixlo_f16 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]\n\t"
        "v_fma_mixhi_f16 %0, -%1, 1.0, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
        : "=&v"(r)
        : "v"(hi), "v"(a), "v"(b));
    lo = r;
}

// The hi / lo planes of eight complex values (re[i], im[i]) as one fragment
// lane of E.
template <class E> __device__ inline void split8(const float (&re)[8], const float (&im)[8], V8<E>& rh, V8<E>& ih,
                                                 V8<E>& rl, V8<E>& il) {
    if constexpr (std::is_same_v<E, _Float16>) {
        uintx4 h0, h1, l0, l1;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            unsigned a, b, c, d;
            split_pair_f16(re[2 * p], re[2 * p + 1], a, b);
            split_pair_f16(im[2 * p], im[2 * p + 1], c, d);
            h0[p] = a;
            l0[p] = b;
            h1[p] = c;
            l1[p] = d;
        }
        rh = __builtin_bit_cast(V8<E>, h0);
        ih = __builtin_bit_cast(V8<E>, h1);
        rl = __builtin_bit_cast(V8<E>, l0);
        il = __builtin_bit_cast(V8<E>, l1);
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const E xh = (E)re[i], yh = (E)im[i];
            rh[i] = xh;
            ih[i] = yh;
            rl[i] = (E)(re[i] - (float)xh);
            il[i] = (E)(im[i] - (float)yh);
        }
    }
}

// Split eight complex values (one fragment lane: 8 K rows of one column),
// times sc (a power of two, see SplitScale), into hi/lo planes and store them
// at lane `lane` of tile t.
template <class E> __device__ inline void lds_split_store(LFrag<E>* t, int lane, const float2 (&v)[8], float sc) {
    float re[8], im[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        re[i] = v[i].x * sc;
        im[i] = v[i].y * sc;
    }
    V8<E> rh, ih, rl, il;
    split8<E>(re, im, rh, ih, rl, il);
    t->rh[lane] = rh;
    t->ih[lane] = ih;
    t->rl[lane] = rl;
    t->il[lane] = il;
}

// One complex value split into hi / lo halves of E, in the exchange form of
// the top up step's output: x = hi(re) | hi(im) << 16, y = lo(re) | lo(im) << 16
// (the same conversions as split8, so the planes built from it are the same).
template <class E> __device__ inline uint2 split_one(float re, float im) {
    unsigned hw, lw;
    if constexpr (std::is_same_v<E, _Float16>) {
        split_pair_f16(re, im, hw, lw);
    } else {
        const E xh = (E)re, yh = (E)im;
        const E xl = (E)(re - (float)xh), yl = (E)(im - (float)yh);
        hw = (unsigned)__builtin_bit_cast(unsigned short, xh) | ((unsigned)__builtin_bit_cast(unsigned short, yh) << 16);
        lw = (unsigned)__builtin_bit_cast(unsigned short, xl) | ((unsigned)__builtin_bit_cast(unsigned short, yl) << 16);
    }
    return make_uint2(hw, lw);
}

// Eight values of one fragment lane (8 K rows of one column) already in the
// exchange form (carried in float2 registers, bits untouched) moved into the
// four planes of tile t: only 16-bit halves are regrouped.
template <class E> __device__ inline void lds_presplit_store(LFrag<E>* t, int lane, const float2 (&v)[8]) {
    uintx4 rh, ih, rl, il;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const unsigned h0 = __builtin_bit_cast(unsigned, v[2 * p].x), h1 = __builtin_bit_cast(unsigned, v[2 * p + 1].x);
        const unsigned l0 = __builtin_bit_cast(unsigned, v[2 * p].y), l1 = __builtin_bit_cast(unsigned, v[2 * p + 1].y);
        // v_perm_b32 picks bytes of {src0 : src1} (src1 = bytes 0-3): low halves, then high halves
        rh[p] = __builtin_amdgcn_perm(h1, h0, 0x05040100u);
        ih[p] = __builtin_amdgcn_perm(h1, h0, 0x07060302u);
        rl[p] = __builtin_amdgcn_perm(l1, l0, 0x05040100u);
        il[p] = __builtin_amdgcn_perm(l1, l0, 0x07060302u);
    }
    t->rh[lane] = __builtin_bit_cast(V8<E>, rh);
    t->ih[lane] = __builtin_bit_cast(V8<E>, ih);
    t->rl[lane] = __builtin_bit_cast(V8<E>, rl);
    t->il[lane] = __builtin_bit_cast(V8<E>, il);
}

template <class V> __device__ inline V neg8(V v) {     // sign flip of eight 16-bit values
    intx4 x = __builtin_bit_cast(intx4, v);
    x ^= (int)0x80008000;
    return __builtin_bit_cast(V, x);
}

// One lane's eight entries exp(2 pi i t) of a phase tile (t in units of 2^-32
// turns, |t| <= 1/2), split into hi / lo planes.  v_sin_f32 / v_cos_f32 take
// their argument in turns.
struct AngRaw {
    intx4 a0, a1;
};

template <class E> __device__ inline Frag<E> angle_frag(const AngRaw& r) {
    const intx4 a0 = r.a0, a1 = r.a1;
    float c[8], s[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float t = (float)(i < 4 ? a0[i] : a1[i - 4]) * 0x1p-32f;
        c[i] = __builtin_amdgcn_cosf(t);
        s[i] = __builtin_amdgcn_sinf(t);
    }
    Frag<E> f;
    split8<E>(c, s, f.rh, f.ih, f.rl, f.il);
    return f;
}

template <class E, int MTW>
__device__ inline void kstep_bf16(floatx4 (&cr)[MTW][4], floatx4 (&ci)[MTW][4], const Frag<E> (&a)[MTW],
                                  const Frag<E> (&b)[4], int ntl) {
#define MF(acc, x, y) acc = mfma16(x, y, acc)
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) {
        if (mt >= ntl) continue;
        const V8<E> nih = neg8(a[mt].ih), nil = neg8(a[mt].il);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            MF(cr[mt][nt], a[mt].rh, b[nt].rh);
            MF(ci[mt][nt], a[mt].rh, b[nt].ih);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            MF(cr[mt][nt], nih, b[nt].ih);
            MF(ci[mt][nt], a[mt].ih, b[nt].rh);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            MF(cr[mt][nt], a[mt].rh, b[nt].rl);
            MF(ci[mt][nt], a[mt].rh, b[nt].il);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            MF(cr[mt][nt], a[mt].rl, b[nt].rh);
            MF(ci[mt][nt], a[mt].rl, b[nt].ih);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            MF(cr[mt][nt], nih, b[nt].il);
            MF(ci[mt][nt], a[mt].ih, b[nt].rl);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            MF(cr[mt][nt], nil, b[nt].ih);
            MF(ci[mt][nt], a[mt].il, b[nt].rh);
        }
    }
#undef MF
}

// The same twelve products for a single column tile nt.
template <class E, int MTW>
__device__ inline void kstep1_bf16(floatx4 (&cr)[MTW][4], floatx4 (&ci)[MTW][4], const Frag<E> (&a)[MTW],
                                   const Frag<E>& b, int nt, int ntl) {
#define MF(acc, x, y) acc = mfma16(x, y, acc)
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) {
        if (mt >= ntl) continue;
        const V8<E> nih = neg8(a[mt].ih), nil = neg8(a[mt].il);
        MF(cr[mt][nt], a[mt].rh, b.rh);
        MF(ci[mt][nt], a[mt].rh, b.ih);
        MF(cr[mt][nt], nih, b.ih);
        MF(ci[mt][nt], a[mt].ih, b.rh);
        MF(cr[mt][nt], a[mt].rh, b.rl);
        MF(ci[mt][nt], a[mt].rh, b.il);
        MF(cr[mt][nt], a[mt].rl, b.rh);
        MF(ci[mt][nt], a[mt].rl, b.ih);
        MF(cr[mt][nt], nih, b.il);
        MF(ci[mt][nt], a[mt].ih, b.rl);
        MF(cr[mt][nt], nil, b.ih);
        MF(ci[mt][nt], a[mt].il, b.rh);
    }
#undef MF
}

template <int MTW_, int NT_, int CT_>
struct BCfg {
    static constexpr int MTW = MTW_;     // 16-row tiles per wave
    static constexpr int NT = NT_;       // threads per workgroup
    static constexpr int CT = CT_;       // K tiles (of 32) per pipeline stage
    static constexpr int ROUND = NT / 64 * MTW * 16;
    static_assert(NT >= 256 * CT, "at most one 8-row B block per thread and stage");
};

// Rows [base, base + 16 MTW) of C (+)= A B for one wave, where A's tiles of
// row tile t start at Atiles + t * ktiles tiles.  B[j][r] = src[boff(j, r)].
// One stage = CT K tiles: every thread loads 8 consecutive K rows of one B
// column (coalesced across the wave), splits them into hi/lo planes and writes
// them as four 16-byte pieces of one MFMA fragment; A fragments and B rows of
// stage c+1 are in flight while stage c is multiplied; double-buffered LDS,
// one barrier per stage.  Every thread of the workgroup must call this.
template <class C, class E, class BOff>
__device__ void gemm_rows_bf16(floatx4 (&cr)[C::MTW][4], floatx4 (&ci)[C::MTW][4], const Frag<E>* __restrict__ Atiles,
                               int M, int K, int base, const float2* __restrict__ src, BOff boff, int nr,
                               LFrag<E>* sB, float bsc) {
    constexpr int MTW = C::MTW, CT = C::CT;
    constexpr int KS = CT * KT;                     // K rows per stage
    const int tid = threadIdx.x, l = tid & 63;
    const int ntl = base < M ? min(MTW, (M - base + 15) / 16) : 0;
    const int ktiles = (K + KT - 1) / KT;
    if (ktiles == 0) return;
    const int nst = (ktiles + CT - 1) / CT;
    const int mt0 = base / 16;
    // this thread's B column and 8-row block within a stage (threads beyond
    // 256 CT stage nothing)
    const bool stager = tid < 256 * CT;
    const int br = tid & 63, bj = (tid >> 6) * 8;
    auto loadA = [&](int st, Frag<E> (&dst)[CT][MTW]) {
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int kt = st * CT + c;
#pragma unroll
            for (int mt = 0; mt < MTW; ++mt)
                if (mt < ntl && kt < ktiles) dst[c][mt] = Atiles[((long long)(mt0 + mt) * ktiles + kt) * 64 + l];
        }
    };
    float2 bt[8];
    auto loadB = [&](int st) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int j = st * KS + bj + i;
            bt[i] = (stager && j < K && br < nr) ? src[boff(j, br)] : make_float2(0.f, 0.f);
        }
    };
    auto storeB = [&](int buf) {
        if (!stager) return;
        const int kt = bj / KT, kk = bj % KT;
        lds_split_store(sB + (buf * CT + kt) * 4 + (br >> 4), (kk >> 3) * 16 + (br & 15), bt, bsc);
    };
    Frag<E> acur[CT][MTW], anext[CT][MTW];
    loadA(0, acur);
    loadB(0);
    __syncthreads();
    storeB(0);
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
        const bool more = st + 1 < nst;
        if (more) {
            loadA(st + 1, anext);
            loadB(st + 1);
        }
        if (ntl > 0) {
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                if (st * CT + c < ktiles) {
                    const LFrag<E>* sb = sB + ((st & 1) * CT + c) * 4;
                    if constexpr (C::NT >= 1024) {
                        // one B fragment at a time (register budget of 16 waves)
#pragma unroll
                        for (int nt = 0; nt < 4; ++nt) {
                            const Frag<E> b = lds_frag(sb + nt, l);
                            kstep1_bf16<E, MTW>(cr, ci, acur[c], b, nt, ntl);
                        }
                    } else {
                        Frag<E> b[4];
#pragma unroll
                        for (int nt = 0; nt < 4; ++nt) b[nt] = lds_frag(sb + nt, l);
                        kstep_bf16<E, MTW>(cr, ci, acur[c], b, ntl);
                    }
                }
            }
        }
        if (more) {
            storeB((st + 1) & 1);
#pragma unroll
            for (int c = 0; c < CT; ++c)
#pragma unroll
                for (int mt = 0; mt < MTW; ++mt) acur[c][mt] = anext[c][mt];
        }
        __syncthreads();
    }
}

template <int MTW>
__device__ inline void zero_acc(floatx4 (&cr)[MTW][4], floatx4 (&ci)[MTW][4]) {
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) { cr[mt][nt] = floatx4{0, 0, 0, 0}; ci[mt][nt] = floatx4{0, 0, 0, 0}; }
}

template <int NT>
__device__ int candidate_rows(int* crow, const ApplyGeom& G, int s, long long a, long long partner, long long Ps,
                              const int* k_prev, const long long* yoff_prev) {
    if (s == 0) {
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

__device__ inline float2 load_vec(bool ext, const float2* p, long long ld, int nrhs, int row, int r) {
    return ext ? p[(long long)r * ld + row] : p[(long long)row * nrhs + r];
}

__device__ inline long long xcd_group_order(long long b, long long nid, int P) {
    if (P != 4 || (nid & 31) != 0) return b;
    const long long x = b & 7, t = (b >> 3) & 3, q = b >> 5;
    return ((q << 3) + x) * 4 + t;
}

template <class C, class E>
__global__ __launch_bounds__(C::NT) void up_bf16(UpArgs A, long long nid) {
    constexpr int MTW = C::MTW;
    __shared__ int crow[CROW_MAX];
    __shared__ int srcrow[CROW_MAX];
    __shared__ LFrag<E> sB[2 * C::CT * 4];
    const long long id = xcd_group_order(blockIdx.x, nid, A.G.P);
    const long long g = id / A.G.P;
    const long long a = g / A.Ps, ap = g - (g / A.Ps) * A.Ps;
    const int r0 = blockIdx.y * NRHS;
    const int nr = min(NRHS, A.nrhs - r0);
    candidate_rows<C::NT>(crow, A.G, A.s, a, ap, A.Ps, A.k_prev, A.yoff_prev);
    const bool ext = A.s == 0 && A.ext;   // else the leaves read the row-major copy in A.in
    const float2* xin = ext ? (const float2*)A.ext : (const float2*)A.in;
    float2* out = (float2*)A.out;
    const int k = A.lev.k[id], nred = A.lev.n[id] - k;
    const int* perm = A.lev.perm + A.lev.perm_off[id];
    const Frag<E>* Tt = (const Frag<E>*)A.lev.T[id];
    const long long yo = A.lev.y_off[id];
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
    __syncthreads();
    for (int j = tid; j < nred; j += C::NT) srcrow[j] = crow[perm[k + j]];
    __syncthreads();
    auto run = [&](const float2* xb, auto boff) {
        for (int m0 = 0; m0 < k; m0 += C::ROUND) {
            const int base = m0 + wave * MTW * 16;
            floatx4 cr[MTW][4], ci[MTW][4];
            zero_acc<MTW>(cr, ci);
            gemm_rows_bf16<C, E>(cr, ci, Tt, k, nred, base, xb, boff, nr, sB, 1.f);
#pragma unroll
            for (int mt = 0; mt < MTW; ++mt) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = base + mt * 16 + 4 * lk + v;
                    if (row < k) {
                        const int src = crow[perm[row]];
#pragma unroll
                        for (int nt = 0; nt < 4; ++nt) {
                            const int r = nt * 16 + lr;
                            if (r < nr) {
                                const float2 sv = load_vec(ext, xin, A.ld, A.nrhs, src, r0 + r);
                                out[(yo + row) * A.nrhs + r0 + r] = make_float2(
                                    cr[mt][nt][v] + sv.x, ci[mt][nt][v] + sv.y);
                            }
                        }
                    }
                }
            }
        }
    };
    // B rows are input rows: at the leaves the caller's column-major input
    // (ld apart per right-hand side), above them a level buffer (nrhs wide)
    if (ext)
        run(xin + (long long)r0 * A.ld, [&](int j, int c) { return (long long)c * A.ld + srcrow[j]; });
    else
        run(xin + r0, [&](int j, int c) { return (long long)srcrow[j] * A.nrhs + c; });
}

template <class C, class E>
__global__ __launch_bounds__(C::NT) void down_bf16(DownArgs A, long long nid, float2* scr) {
    constexpr int MTW = C::MTW;
    __shared__ LFrag<E> sB[2 * C::CT * 4];
    const long long id = xcd_group_order(blockIdx.x, nid, A.G.P);
    const int r0 = blockIdx.y * NRHS;
    const int nr = min(NRHS, A.nrhs - r0);
    const float2* zin = (const float2*)A.in;
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
    const int k = A.lev.k[id], nred = A.lev.n[id] - k;
    const int* perm = A.lev.perm + A.lev.perm_off[id];
    const Frag<E>* Tt = (const Frag<E>*)A.lev.T[id];
    const long long yo = A.lev.y_off[id];
    float2* w = scr + A.lev.perm_off[id] * A.nrhs;
    for (int e = tid; e < k * NRHS; e += C::NT) {
        const int i = e / NRHS, r = e - i * NRHS;
        if (r < nr) w[(long long)perm[i] * A.nrhs + r0 + r] = zin[(yo + i) * A.nrhs + r0 + r];
    }
    const float2* z = zin + yo * A.nrhs + r0;
    auto boff = [&](int i, int c) { return (long long)i * A.nrhs + c; };
    for (int m0 = 0; m0 < nred; m0 += C::ROUND) {
        const int base = m0 + wave * MTW * 16;
        floatx4 cr[MTW][4], ci[MTW][4];
        zero_acc<MTW>(cr, ci);
        gemm_rows_bf16<C, E>(cr, ci, Tt, nred, k, base, z, boff, nr, sB, 1.f);
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = base + mt * 16 + 4 * lk + v;
                if (row < nred) {
                    float2* d = w + (long long)perm[k + row] * A.nrhs + r0;
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        const int r = nt * 16 + lr;
                        if (r < nr) d[r] = make_float2(cr[mt][nt][v], ci[mt][nt][v]);
                    }
                }
            }
        }
    }
}

template <class C, class E>
__global__ __launch_bounds__(C::NT) void middle_bf16(MidArgs A, const long long* tile_off) {
    constexpr int MTW = C::MTW;
    __shared__ int crow_in[CROW_MAX];
    __shared__ int crow_out[CROW_MAX];
    __shared__ LFrag<E> sB[2 * C::CT * 4];
    const long long bi = blockIdx.x;
    const int r0 = blockIdx.y * NRHS;
    const int nr = min(NRHS, A.nrhs - r0);
    const int M = A.nr[bi], K = A.nc[bi];
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
    middle_rows<C::NT>(crow_in, crow_out, A, bi);
    const float2* xin = (const float2*)A.in;
    float2* zout = (float2*)A.out;
    const Frag<E>* St = (const Frag<E>*)A.S + tile_off[bi] * 64;
    __syncthreads();
    auto boff = [&](int j, int c) { return (long long)crow_in[j] * A.nrhs + c; };
    for (int m0 = 0; m0 < M; m0 += C::ROUND) {
        const int base = m0 + wave * MTW * 16;
        floatx4 cr[MTW][4], ci[MTW][4];
        zero_acc<MTW>(cr, ci);
        gemm_rows_bf16<C, E>(cr, ci, St, M, K, base, xin + r0, boff, nr, sB, A.bscale);
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = base + mt * 16 + 4 * lk + v;
                if (row < M) {
                    const long long dst = crow_out[row];
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        const int r = nt * 16 + lr;
                        if (r < nr)
                            zout[dst * A.nrhs + r0 + r] = make_float2(cr[mt][nt][v], ci[mt][nt][v]);
                    }
                }
            }
        }
    }
}

// Going down with the whole z block resident in LDS (k <= 32 RES_KT): one
// workgroup per decomposition stages z once, split into fragments; then each
// wave streams the fragment tiles of A = T^T row tile by row tile, two tiles
// ahead, with no barrier in the loop.  The down GEMMs are short in K (k) and
// long in M (n - k), so the shared B never needs restaging.
// Eight consecutive K rows j0 .. j0 + 7 of column col of B, B[j][c] =
// src[boff(j, c)], zero beyond K rows or nr columns (K, nr >= 1).  Every
// address is formed in range first (row and column clamped), so the eight
// index reads and the eight loads issue back to back, with no branch around
// each load; the values outside B are zeroed afterwards.
template <class BOff>
__device__ inline void load_b8(float2 (&v)[8], const float2* __restrict__ src, BOff boff, int j0, int col, int K,
                               int nr) {
    const int c = col < nr ? col : 0;
    long long o[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) o[i] = boff(min(j0 + i, K - 1), c);
    float2 x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = src[o[i]];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = (j0 + i < K && col < nr) ? x[i] : make_float2(0.f, 0.f);
}

constexpr int RES_KT = 8;
static_assert(RES_KT * KT == SPLIT16_RESIDENT_K, "resident rank limit");

// C = A B for every row tile of an M x K block, B (K <= RES_KT * KT rows,
// B[j][c] = src[boff(j, c)]) resident in LDS: B is staged once, split into
// fragments; then wave w takes row tiles w, w + NW, ... and streams their A
// tiles two ahead with no barrier in the loop (the first two are requested
// before B is staged).  epi(base, cr, ci) stores the finished row tile of
// rows [base, base + 16) (also for K = 0, with zeros).  ONE_B: read one B
// fragment at a time (fewer registers).  Every thread of the workgroup must
// call this.
template <class E, int NT, bool ONE_B, class BOff, class Epi>
__device__ void gemm_resident(const Frag<E>* __restrict__ Atiles, int M, int K, const float2* __restrict__ src,
                              BOff boff, int nr, LFrag<E>* sB, float bsc, Epi epi) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
    const int ktiles = (K + KT - 1) / KT;
    const int mtiles = (M + 15) / 16;
    const int mine = mtiles > wave ? (mtiles - wave + NW - 1) / NW : 0;   // row tiles of this wave
    floatx4 cr[1][4], ci[1][4];
    if (ktiles == 0) {
        zero_acc<1>(cr, ci);
        for (int t = 0; t < mine; ++t) epi((wave + t * NW) * 16, cr, ci);
        return;
    }
    const int total = mine * ktiles;
    auto tile_at = [&](int q) {
        const int mt = wave + (q / ktiles) * NW, kt = q - (q / ktiles) * ktiles;
        return Atiles[((long long)mt * ktiles + kt) * 64 + l];
    };
    Frag<E> f0[1], f1, f2;
    if (total > 0) f0[0] = tile_at(0);
    if (total > 1) f1 = tile_at(1);
    for (int f = tid; f < ktiles * 256; f += NT) {
        const int kt = f >> 8, rem = f & 255, kb = rem >> 6, col = rem & 63;
        float2 v[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int j = kt * KT + kb * 8 + i;
            v[i] = (j < K && col < nr) ? src[boff(j, col)] : make_float2(0.f, 0.f);
        }
        lds_split_store(sB + kt * 4 + (col >> 4), kb * 16 + (col & 15), v, bsc);
    }
    __syncthreads();
    for (int q = 0; q < total; ++q) {
        if (q + 2 < total) f2 = tile_at(q + 2);
        const int kt = q - (q / ktiles) * ktiles;
        if (kt == 0) zero_acc<1>(cr, ci);
        if constexpr (ONE_B) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const Frag<E> b = lds_frag(sB + kt * 4 + nt, l);
                kstep1_bf16<E, 1>(cr, ci, f0, b, nt, 1);
            }
        } else {
            Frag<E> b[4];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) b[nt] = lds_frag(sB + kt * 4 + nt, l);
            kstep_bf16<E, 1>(cr, ci, f0, b, 1);
        }
        if (kt == ktiles - 1) epi((wave + (q / ktiles) * NW) * 16, cr, ci);
        f0[0] = f1;
        f1 = f2;
    }
}

template <class E, int NT>
__global__ __launch_bounds__(NT) void down_res16(DownArgs A, long long nid, float2* scr) {
    __shared__ LFrag<E> sB[RES_KT * 4];
    const long long id = xcd_group_order(blockIdx.x, nid, A.G.P);
    const int r0 = blockIdx.y * NRHS;
    const int nr = min(NRHS, A.nrhs - r0);
    const float2* zin = (const float2*)A.in;
    const int tid = threadIdx.x, l = tid & 63, lr = l & 15, lk = l >> 4;
    const int k = A.lev.k[id], nred = A.lev.n[id] - k;
    const int* perm = A.lev.perm + A.lev.perm_off[id];
    const Frag<E>* Tt = (const Frag<E>*)A.lev.T[id];
    const long long yo = A.lev.y_off[id];
    float2* w = scr + A.lev.perm_off[id] * A.nrhs;
    for (int e = tid; e < k * NRHS; e += NT) {
        const int i = e / NRHS, r = e - i * NRHS;
        if (r < nr) w[(long long)perm[i] * A.nrhs + r0 + r] = zin[(yo + i) * A.nrhs + r0 + r];
    }
    if (nred == 0) return;
    // z (k x 64) resident (k <= RES_KT * KT, checked at launch); rows of T^T z scattered by perm
    auto epi = [&](int base, const floatx4 (&cr)[1][4], const floatx4 (&ci)[1][4]) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = base + 4 * lk + v;
            if (row < nred) {
                float2* d = w + (long long)perm[k + row] * A.nrhs + r0;
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const int r = nt * 16 + lr;
                    if (r < nr) d[r] = make_float2(cr[0][nt][v], ci[0][nt][v]);
                }
            }
        }
    };
    gemm_resident<E, NT, (NT >= 1024)>(Tt, nred, k, zin + yo * A.nrhs + r0,
                                       [&](int j, int c) { return (long long)j * A.nrhs + c; }, nr, sB, 1.f, epi);
}

// Going down, one workgroup per group of 2^d sibling decompositions (same
// candidate set): sibling t's contribution -- z_t on its skeleton rows, T_t^T
// z_t on its redundant rows -- is added to the group's candidate rows in the
// order t = 0, 1, ... (t = 0 writes, the others read-add-write; a barrier
// separates the siblings), so no per-ID scratch and no separate sum pass are
// needed.  The candidate rows are rows of the previous level buffer, or of the
// row-major lattice copy at the leaves (both nrhs wide; with one right-hand
// side the caller's block itself).  z_t resident (k <= RES_KT * KT).
template <class E, int NT>
__global__ __launch_bounds__(NT) void down_group16(DownArgs A) {
    extern __shared__ __align__(16) int crow[];            // ncand_max candidate rows
    __shared__ LFrag<E> sB[RES_KT * 4];
    const long long g = blockIdx.x;
    const long long a = g / A.Ps, bp = g - (g / A.Ps) * A.Ps;
    const int r0 = blockIdx.y * NRHS;
    const int nr = min(NRHS, A.nrhs - r0);
    candidate_rows<NT>(crow, A.G, A.s, a, bp, A.Ps, A.k_prev, A.yoff_prev);
    float2* outp = (A.s == 0 && A.ext) ? (float2*)A.ext : (float2*)A.out;
    const float2* zin = (const float2*)A.in;
    const int tid = threadIdx.x, l = tid & 63, lr = l & 15, lk = l >> 4;
    for (int t = 0; t < A.G.P; ++t) {
        __syncthreads();          // crow ready; the previous sibling's rows written and sB free
        const long long id = g * A.G.P + t;
        const int k = A.lev.k[id], nred = A.lev.n[id] - k;
        const int* perm = A.lev.perm + A.lev.perm_off[id];
        const Frag<E>* Tt = (const Frag<E>*)A.lev.T[id];
        const long long yo = A.lev.y_off[id];
        const bool first = t == 0;
        for (int e = tid; e < k * NRHS; e += NT) {
            const int i = e / NRHS, r = e - i * NRHS;
            if (r < nr) {
                float2* d = outp + (long long)crow[perm[i]] * A.nrhs + r0 + r;
                const float2 v = zin[(yo + i) * A.nrhs + r0 + r];
                if (first) {
                    *d = v;
                } else {
                    const float2 o = *d;
                    *d = make_float2(o.x + v.x, o.y + v.y);
                }
            }
        }
        auto dst_row = [&](int row) { return outp + (long long)crow[perm[k + row]] * A.nrhs + r0; };
        auto epi = [&](int base, const floatx4 (&cr)[1][4], const floatx4 (&ci)[1][4]) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = base + 4 * lk + v;
                if (row < nred) {
                    float2* d = dst_row(row);
                    if (first) {
#pragma unroll
                        for (int nt = 0; nt < 4; ++nt) {
                            const int r = nt * 16 + lr;
                            if (r < nr) d[r] = make_float2(cr[0][nt][v], ci[0][nt][v]);
                        }
                    } else {
                        float2 o[4];
#pragma unroll
                        for (int nt = 0; nt < 4; ++nt) {
                            const int r = nt * 16 + lr;
                            if (r < nr) o[nt] = d[r];
                        }
#pragma unroll
                        for (int nt = 0; nt < 4; ++nt) {
                            const int r = nt * 16 + lr;
                            if (r < nr)
                                d[r] = make_float2(o[nt].x + cr[0][nt][v], o[nt].y + ci[0][nt][v]);
                        }
                    }
                }
            }
        };
        gemm_resident<E, NT, (NT >= 768)>(Tt, nred, k, zin + yo * A.nrhs + r0,
                                          [&](int j, int c) { return (long long)j * A.nrhs + c; }, nr, sB, 1.f, epi);
    }
}

// The last down step (the leaves, n0 <= 64 points): one workgroup per leaf
// sums its P siblings' contributions in LDS and writes each point's row once
// (row-major, nrhs wide: the lattice copy, or with one right-hand side the
// caller's block).  Every point first gets the z_t rows of the siblings that
// keep it as a skeleton, in sibling order (one thread per point and column, so
// the P loads are in flight together); then T_t^T z_t is added on the other
// points, sibling by sibling.  z_t resident (k <= n0 <= 64).
constexpr int LEAF_MAX = 64;

template <class E>
__global__ __launch_bounds__(256) void down_leaf16(DownArgs A) {
    __shared__ float2 acc[LEAF_MAX][NRHS + 1];
    __shared__ int crow[LEAF_MAX];
    __shared__ int inv[MAX_P][LEAF_MAX];
    __shared__ int ks[MAX_P];
    __shared__ long long yos[MAX_P];
    __shared__ LFrag<E> sB[2 * 4];
    const long long g = blockIdx.x;
    const int r0 = blockIdx.y * NRHS;
    const int nr = min(NRHS, A.nrhs - r0);
    const int n0 = A.G.n0, P = A.G.P;
    const int tid = threadIdx.x, l = tid & 63, lr = l & 15, lk = l >> 4;
    candidate_rows<256>(crow, A.G, 0, g, 0, 1, nullptr, nullptr);
    if (tid < P) {
        ks[tid] = A.lev.k[g * P + tid];
        yos[tid] = A.lev.y_off[g * P + tid];
    }
    for (int e = tid; e < P * n0; e += 256) {
        const int t = e / n0, p = e - t * n0;
        inv[t][A.lev.perm[A.lev.perm_off[g * P + t] + p]] = p;
    }
    __syncthreads();
    const float2* zin = (const float2*)A.in;
    // Each thread's (point, column) elements in batches of GB.  Every load's
    // address is formed in range (row 0 of the buffer where a sibling does not
    // keep the point), so a batch's P * GB loads issue together; the absent
    // terms are selected away, and the sum keeps sibling order.
    constexpr int GB = 4;
    for (int e0 = tid; e0 < n0 * NRHS; e0 += 256 * GB) {
        float2 v[GB][MAX_P];
        bool use[GB][MAX_P];
#pragma unroll
        for (int b = 0; b < GB; ++b) {
            const int e = e0 + b * 256;
            const bool in = e < n0 * NRHS;
            const int p = in ? e / NRHS : 0, r = in ? e - p * NRHS : 0;
#pragma unroll
            for (int t = 0; t < MAX_P; ++t) {
                if (t < P) {
                    const int i = inv[t][p];
                    use[b][t] = in && r < nr && i < ks[t];
                    const long long row = use[b][t] ? yos[t] + i : 0;
                    v[b][t] = zin[row * A.nrhs + (use[b][t] ? r0 + r : 0)];
                }
            }
        }
#pragma unroll
        for (int b = 0; b < GB; ++b) {
            const int e = e0 + b * 256;
            if (e < n0 * NRHS) {
                const int p = e / NRHS, r = e - p * NRHS;
                float2 sum = make_float2(0.f, 0.f);
#pragma unroll
                for (int t = 0; t < MAX_P; ++t)
                    if (t < P && use[b][t]) sum = make_float2(sum.x + v[b][t].x, sum.y + v[b][t].y);
                acc[p][r] = sum;
            }
        }
    }
    for (int t = 0; t < P; ++t) {
        const long long id = g * P + t;
        const int k = ks[t], nred = n0 - k;
        if (nred == 0) continue;      // (uniform over the workgroup)
        __syncthreads();          // acc holds the earlier contributions; sB free
        const int* perm = A.lev.perm + A.lev.perm_off[id];
        const Frag<E>* Tt = (const Frag<E>*)A.lev.T[id];
        const long long yo = yos[t];
        auto epi = [&](int base, const floatx4 (&cr)[1][4], const floatx4 (&ci)[1][4]) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = base + 4 * lk + v;
                if (row < nred) {
                    float2* d = acc[perm[k + row]];
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        const int r = nt * 16 + lr;
                        d[r] = make_float2(d[r].x + cr[0][nt][v], d[r].y + ci[0][nt][v]);
                    }
                }
            }
        };
        gemm_resident<E, 256, false>(Tt, nred, k, zin + yo * A.nrhs + r0,
                                     [&](int j, int c) { return (long long)j * A.nrhs + c; }, nr, sB, 1.f, epi);
    }
    __syncthreads();
    float2* outp = A.ext ? (float2*)A.ext : (float2*)A.out;
    for (int e = tid; e < n0 * NRHS; e += 256) {
        const int p = e / NRHS, r = e - p * NRHS;
        if (r < nr) outp[(long long)crow[p] * A.nrhs + r0 + r] = acc[p][r];
    }
}

// Rows [base, base + 16) of C = A B for one wave (one row tile), over K in
// stages of RCT K-tiles: B stages double-buffered in LDS (all threads split and
// store them), A fragments streamed per wave AD tiles ahead across stage
// boundaries.  Every thread of the workgroup must call this.  RCT * 256
// fragment lanes per stage split evenly over NT threads.
template <int NT> constexpr int rct_for() { return NT == 768 ? 3 : 4; }

// A tiles in flight stay raw (phase tiles are expanded only when used).
template <class E, bool ANG> using ARaw = std::conditional_t<ANG, AngRaw, Frag<E>>;

template <class E, bool ANG>
__device__ inline ARaw<E, ANG> a_tile(const Frag<E>* __restrict__ Atiles, const int* __restrict__ Aang, int mt,
                                      int ktiles, int kt) {
    const long long idx = ((long long)mt * ktiles + kt) * 64 + (threadIdx.x & 63);
    if constexpr (ANG) {
        AngRaw r;
        r.a0 = *(const intx4*)(Aang + idx * 8);
        r.a1 = *(const intx4*)(Aang + idx * 8 + 4);
        return r;
    } else {
        return Atiles[idx];
    }
}

// The A tiles of one wave of gemm_res16: the one in use and AD requested
// ahead.  a_prefetch issues the first AD; a kernel with table loads and
// barriers ahead of the GEMM calls it first and passes preloaded = true.
template <class E, int AD, bool ANG>
struct APipe {
    ARaw<E, ANG> fa[AD + 1];
};

template <class E, int AD, bool ANG>
__device__ inline void a_prefetch(APipe<E, AD, ANG>& p, const Frag<E>* __restrict__ Atiles,
                                  const int* __restrict__ Aang, int M, int K, int base) {
    const int ktiles = (K + KT - 1) / KT;
    if (base < M) {
#pragma unroll
        for (int i = 0; i < AD; ++i)
            if (i < ktiles) p.fa[i] = a_tile<E, ANG>(Atiles, Aang, base / 16, ktiles, i);
    }
}

// BATCH: B stages gathered with load_b8 (measured faster for the up steps,
// slower for the phase-tile middle).  RCT_ > 0: K tiles per B stage (else
// rct_for<NT>), with one B fragment in registers at a time.  PRE: B arrives
// in the exchange form (split_one; bsc is then already applied).
template <class E, int NT, int AD, bool ANG = false, bool BATCH = false, int RCT_ = 0, bool PRE = false,
          class BOff>
__device__ void gemm_res16(floatx4 (&cr)[1][4], floatx4 (&ci)[1][4], const Frag<E>* __restrict__ Atiles, int M,
                           int K, int base, const float2* __restrict__ src, BOff boff, int nr, LFrag<E>* sB,
                           float bsc, const int* __restrict__ Aang, APipe<E, AD, ANG>& pipe, bool preloaded) {
    constexpr int RCT = RCT_ > 0 ? RCT_ : rct_for<NT>();
    constexpr int FPT = RCT * 256 / NT;            // B fragments staged per thread and stage
    static_assert(FPT >= 1 && FPT * NT == RCT * 256, "stage must split evenly over the threads");
    const int tid = threadIdx.x, l = tid & 63;
    const int ktiles = (K + KT - 1) / KT;
    if (ktiles == 0) return;
    const int nst = (ktiles + RCT - 1) / RCT;
    const bool active = base < M;
    const int mt = base / 16;
    float2 bt[FPT][8];
    auto loadB = [&](int st) {
#pragma unroll
        for (int q = 0; q < FPT; ++q) {
            const int f = tid + q * NT, kt = f >> 8, kb = (f & 255) >> 6, col = f & 63;
            if constexpr (BATCH) {
                load_b8(bt[q], src, boff, (st * RCT + kt) * KT + kb * 8, col, K, nr);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int j = (st * RCT + kt) * KT + kb * 8 + i;
                    bt[q][i] = (j < K && col < nr) ? src[boff(j, col)] : make_float2(0.f, 0.f);
                }
            }
        }
    };
    auto storeB = [&](int buf) {
#pragma unroll
        for (int q = 0; q < FPT; ++q) {
            const int f = tid + q * NT, kt = f >> 8, kb = (f & 255) >> 6, col = f & 63;
            if constexpr (PRE) lds_presplit_store(sB + (buf * RCT + kt) * 4 + (col >> 4), kb * 16 + (col & 15), bt[q]);
            else lds_split_store(sB + (buf * RCT + kt) * 4 + (col >> 4), kb * 16 + (col & 15), bt[q], bsc);
        }
    };
    auto tile_at = [&](int kt) { return a_tile<E, ANG>(Atiles, Aang, mt, ktiles, kt); };
    auto& fa = pipe.fa;
    if (!preloaded) a_prefetch<E, AD, ANG>(pipe, Atiles, Aang, M, K, base);
    loadB(0);
    __syncthreads();          // the previous user of sB is done
    storeB(0);
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
        const bool more = st + 1 < nst;
        if (more) loadB(st + 1);
        const LFrag<E>* sb = sB + (st & 1) * RCT * 4;
        if (active) {
#pragma unroll
            for (int c = 0; c < RCT; ++c) {
                const int kt = st * RCT + c;
                if (kt < ktiles) {
                    if (kt + AD < ktiles) fa[AD] = tile_at(kt + AD);
                    Frag<E> a0[1];
                    if constexpr (ANG) a0[0] = angle_frag<E>(fa[0]);
                    else a0[0] = fa[0];
                    if constexpr (NT >= 768 || RCT_ > 0) {
                        // one B fragment at a time (register budget of 12 or 16 waves per CU)
#pragma unroll
                        for (int nt = 0; nt < 4; ++nt) {
                            const Frag<E> b = lds_frag(sb + c * 4 + nt, l);
                            kstep1_bf16<E, 1>(cr, ci, a0, b, nt, 1);
                        }
                    } else {
                        Frag<E> b[4];
#pragma unroll
                        for (int nt = 0; nt < 4; ++nt) b[nt] = lds_frag(sb + c * 4 + nt, l);
                        kstep_bf16<E, 1>(cr, ci, a0, b, 1);
                    }
#pragma unroll
                    for (int i = 0; i < AD; ++i) fa[i] = fa[i + 1];
                }
            }
        }
        if (more) storeB((st + 1) & 1);
        __syncthreads();
    }
}

// Going up, one workgroup per decomposition.  Input rows come from the level's
// source-row table (LevelArgs::src, built once per plan): one coalesced copy
// of the ID's n entries into LDS and one barrier, in place of the child-piece
// tables, the permutation lookups and their two barriers.  RES_ONLY: every
// decomposition of the level has n - k <= RES_KT * KT, so only the resident
// path is built.
// PRE: the top up step writes its output in the exchange form for the middle
// (UpArgs::presplit).
template <class E, int NT, bool RES_ONLY, bool PRE = false>
__global__ __launch_bounds__(NT) void up_res16(UpArgs A, long long nid) {
    constexpr int NW = NT / 64;
    __shared__ int srow[CROW_MAX];
    __shared__ LFrag<E> sB[std::max(2 * rct_for<NT>(), RES_KT) * 4];
    const long long id = xcd_group_order(blockIdx.x, nid, A.G.P);
    const int r0 = blockIdx.y * NRHS;
    const int nr = min(NRHS, A.nrhs - r0);
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
    const int k = A.lev.k[id], nred = A.lev.n[id] - k;
    const Frag<E>* Tt = (const Frag<E>*)A.lev.T[id];
    const long long yo = A.lev.y_off[id];
    const bool ext = A.s == 0 && A.ext;   // else the leaves read the row-major copy in A.in
    const float2* xin = ext ? (const float2*)A.ext : (const float2*)A.in;
    float2* out = (float2*)A.out;
    // input row of each candidate position p (n <= CROW_MAX, checked at build)
    const int* src = A.lev.src + A.lev.perm_off[id];
    for (int p = tid; p < k + nred; p += NT) srow[p] = src[p];
    __syncthreads();
    // The skeleton inputs of a row tile are loaded at in-range addresses (row
    // 0 / column 0 outside the tile) so that all sixteen loads of a lane issue
    // together; only the rows and columns inside are stored.
    auto epi = [&](int base, const floatx4 (&cr)[1][4], const floatx4 (&ci)[1][4]) {
        float2 sv[4][4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = base + 4 * lk + v;
            const int src = srow[row < k ? row : 0];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int r = nt * 16 + lr;
                sv[v][nt] = load_vec(ext, xin, A.ld, A.nrhs, src, r0 + (r < nr ? r : 0));
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = base + 4 * lk + v;
            if (row < k) {
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const int r = nt * 16 + lr;
                    if (r < nr) {
                        const float xr = cr[0][nt][v] + sv[v][nt].x, xi = ci[0][nt][v] + sv[v][nt].y;
                        if constexpr (PRE)
                            ((uint2*)out)[(yo + row) * A.nrhs + r0 + r] =
                                split_one<E>(xr * A.presplit, xi * A.presplit);
                        else out[(yo + row) * A.nrhs + r0 + r] = make_float2(xr, xi);
                    }
                }
            }
        }
    };
    auto run = [&](const float2* xb, auto boff) {
        if (RES_ONLY || nred <= RES_KT * KT) {       // the redundant inputs fit in LDS: staged once
            gemm_resident<E, NT, (NT >= 768)>(Tt, k, nred, xb, boff, nr, sB, 1.f, epi);
            return;
        }
        if constexpr (!RES_ONLY) {
            constexpr int UAD = NT >= 1024 ? 1 : 2;   // factor tiles requested ahead (16 waves: register budget)
            APipe<E, UAD, false> pipe;
            for (int m0 = 0; m0 < k; m0 += NW * 16) {
                const int base = m0 + wave * 16;
                floatx4 cr[1][4], ci[1][4];
                zero_acc<1>(cr, ci);
                gemm_res16<E, NT, UAD, false, true>(cr, ci, Tt, k, nred, base, xb, boff, nr, sB, 1.f, nullptr, pipe,
                                                    false);
                epi(base, cr, ci);
            }
        }
    };
    // B rows are input rows: at the leaves the caller's column-major input
    // (ld apart per right-hand side), above them a level buffer (nrhs wide)
    if (ext)
        run(xin + (long long)r0 * A.ld, [&](int j, int c) { return (long long)c * A.ld + srow[k + j]; });
    else
        run(xin + r0, [&](int j, int c) { return (long long)srow[k + j] * A.nrhs + c; });
}

// The source-row table of one up level: one workgroup per ID.
struct SrcRowsArgs {
    ApplyGeom G;
    int s;
    long long Ps;
    const int* n;
    const long long* perm_off;
    const int* perm;
    const int* k_prev;
    const long long* yoff_prev;
    int* out;
    long long id0;
};

__global__ __launch_bounds__(256) void src_lattice_kernel(const int* skel, const int* src, long long count,
                                                         int* out) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < count) out[i] = skel[src[i]];
}

__global__ __launch_bounds__(256) void src_rows_kernel(SrcRowsArgs A) {
    __shared__ int crow[CROW_MAX];
    const long long id = A.id0 + blockIdx.x;
    const long long g = id / A.G.P;
    const long long a = g / A.Ps, ap = g - (g / A.Ps) * A.Ps;
    candidate_rows<256>(crow, A.G, A.s, a, ap, A.Ps, A.k_prev, A.yoff_prev);
    __syncthreads();
    const long long po = A.perm_off[id];
    const int n = A.n[id];
    for (int p = threadIdx.x; p < n; p += 256) A.out[po + p] = crow[A.perm[po + p]];
}

// TWO: two-tile B stages and at most 128 registers, so that two workgroups
// share a CU (LDS 80 KB each at 512 threads) and one's table loads, first
// gather and barriers overlap the other's products.
template <class E, int NT, bool ANG, bool TWO = false, bool PRE = false>
__global__ __launch_bounds__(NT, TWO ? NT / 128 : 1) void middle_res16(MidArgs A, const long long* tile_off) {
    constexpr int NW = NT / 64;
    constexpr int RCT = TWO ? 2 : rct_for<NT>();
    __shared__ int crow_in[CROW_MAX];
    __shared__ int crow_out[CROW_MAX];
    __shared__ LFrag<E> sB[2 * RCT * 4];
    // workgroup -> (block, chunk of NW row tiles).  Workgroups are dealt to the
    // eight XCDs in turn, so the chunks of a block are numbered eight apart:
    // they run on one XCD at about the same time and share its input rows in L2.
    const int mc = A.mchunks;
    const long long b = blockIdx.x, cnt = gridDim.x / mc;
    long long bi;
    int chunk;
    if (cnt % 8 == 0) {
        const long long q = b >> 3;
        bi = (q / mc) * 8 + (b & 7);
        chunk = (int)(q % mc);
    } else {
        bi = b / mc;
        chunk = (int)(b % mc);
    }
    const int M = A.nr[bi], K = A.nc[bi];
    if (chunk * NW * 16 >= M) return;        // (uniform over the workgroup)
    const int r0 = blockIdx.y * NRHS;
    const int nr = min(NRHS, A.nrhs - r0);
    const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
    const Frag<E>* St = (const Frag<E>*)A.S + tile_off[bi] * 64;
    const int* Sang = ANG ? A.ang + tile_off[bi] * 512 : nullptr;
    // the first factor tiles are requested ahead of the row tables and the barrier
    constexpr int MAD = (NT >= 1024 || TWO) ? 1 : 2;  // factor tiles requested ahead (16 waves: register budget)
    APipe<E, MAD, ANG> pipe;
    const int m_first = chunk * NW * 16;
    a_prefetch<E, MAD, ANG>(pipe, St, Sang, M, K, m_first + wave * 16);
    middle_rows<NT>(crow_in, crow_out, A, bi);
    const float2* xin = (const float2*)A.in;
    float2* zout = (float2*)A.out;
    __syncthreads();
    auto boff = [&](int j, int c) { return (long long)crow_in[j] * A.nrhs + c; };
    for (int m0 = m_first; m0 < M; m0 += mc * NW * 16) {
        const int base = m0 + wave * 16;
        floatx4 cr[1][4], ci[1][4];
        zero_acc<1>(cr, ci);
        // (only the middle itself, with phase tiles, changes the vectors' scale)
        gemm_res16<E, NT, MAD, ANG, false, TWO ? RCT : 0, PRE>(cr, ci, St, M, K, base, xin + r0, boff, nr, sB,
                                                              ANG ? A.bscale : 1.f, Sang, pipe, m0 == m_first);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = base + 4 * lk + v;
            if (row < M) {
                const long long dst = crow_out[row];
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const int r = nt * 16 + lr;
                    if (r < nr)
                        zout[dst * A.nrhs + r0 + r] = make_float2(cr[0][nt][v], ci[0][nt][v]);
                }
            }
        }
    }
}

// Largest |re| or |im| of slice blockIdx.x of column blockIdx.y (ColExpArgs).
__global__ __launch_bounds__(256) void colmax_kernel(ColExpArgs A) {
    __shared__ float red[4];
    const int r = blockIdx.y, b = blockIdx.x;
    const long long chunk = (A.N + A.S - 1) / A.S;
    const long long p0 = (long long)b * chunk, p1 = min(A.N, p0 + chunk);
    const float2* x = (const float2*)A.src + (long long)r * A.ld;
    float m = 0.f;
    for (long long p = p0 + threadIdx.x; p < p1; p += 256) {
        const float2 v = x[p];
        m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) A.part[(long long)r * A.S + b] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

__global__ __launch_bounds__(256) void colexp_kernel(ColExpArgs A) {
    for (int r = threadIdx.x; r < A.nrhs; r += 256) {
        float m = 0.f;
        for (int b = 0; b < A.S; ++b) m = fmaxf(m, A.part[(long long)r * A.S + b]);
        int e = 0;
        if (m > 0.f && m <= 3.4e38f) (void)frexpf(m, &e);
        A.cexp[r] = e;
    }
}

using W0 = BCfg<1, 512, 2>;
using W1 = BCfg<1, 256, 1>;
using W2 = BCfg<2, 256, 1>;
using W3 = BCfg<1, 1024, 1>;
using W4 = BCfg<1, 1024, 2>;

template <class C, class E>
void launch_bvariant(LevelKernel which, const void* args, long long count, int nrhs, void* scratch,
                     const long long* tile_off, hipStream_t s) {
    const dim3 grid((unsigned)count, (nrhs + NRHS - 1) / NRHS);
    switch (which) {
        case LevelKernel::Up:
            MIDBF_CHECK(!((const UpArgs*)args)->lattice_in, MIDBF_ERR_ARG,
                        "this up kernel does not read the lattice source-row table");
            hipLaunchKernelGGL((up_bf16<C, E>), grid, dim3(C::NT), 0, s, *(const UpArgs*)args, count);
            break;
        case LevelKernel::Down:
            hipLaunchKernelGGL((down_bf16<C, E>), grid, dim3(C::NT), 0, s, *(const DownArgs*)args, count,
                               (float2*)scratch);
            break;
        case LevelKernel::Middle:
            hipLaunchKernelGGL((middle_bf16<C, E>), grid, dim3(C::NT), 0, s, *(const MidArgs*)args, tile_off);
            break;
        default:
            throw Error(MIDBF_ERR_UNIMPLEMENTED, "no split-bf16 kernel for this level kind");
    }
    MIDBF_HIP(hipGetLastError());
}

// ---- packing of factor blocks into fragment tiles (build time) --------------

// A(row, col) of a block given by a column-major FP32 matrix (lda = M) or by T
// inside an FP64 sample slab; tiles row-tile major, zero padded.
struct PackTilesArgs {
    int mode;                 // 0: FP64 slab, A(i, j) = T[i][j] (T at X[i*n + k + j]); 1: transposed T
                              // 2: FP32 column-major block (lda = M)
    const double2* X;         // mode 0/1: slab base
    long long x_stride;
    const int* k_w;
    const int* n_w;
    const float2* S;          // mode 2
    const long long* s_off;   // mode 2: element offset per block
    const int* nr;
    const int* nc;
    void* out;
    const long long* tile_off;  // per block / ID: first tile
    unsigned* tmax;             // mode 0/1, or null: atomic max of |re|, |im| of the entries (FP32 bits)
};

template <class E>
__global__ void pack_tiles_kernel(PackTilesArgs P) {
    const int b = blockIdx.x;
    int M, K;
    const double2* X = nullptr;
    const float2* S = nullptr;
    int k = 0, n = 0;
    if (P.mode == 2) {
        M = P.nr[b];
        K = P.nc[b];
        S = P.S + P.s_off[b];
    } else {
        k = P.k_w[b];
        n = P.n_w[b];
        X = P.X + (long long)b * P.x_stride;
        M = P.mode == 0 ? k : n - k;
        K = P.mode == 0 ? n - k : k;
    }
    const int mtiles = (M + 15) / 16, ktiles = (K + KT - 1) / KT;
    Frag<E>* out = (Frag<E>*)P.out + P.tile_off[b] * 64;
    const long long nfr = (long long)mtiles * ktiles * 64;
    float amax = 0.f;
    for (long long e = threadIdx.x; e < nfr; e += blockDim.x) {
        const int lane = (int)(e & 63);
        const long long tile = e >> 6;
        const int mt = (int)(tile / ktiles), kt = (int)(tile - (long long)mt * ktiles);
        const int row = mt * 16 + (lane & 15);
        const int c0 = kt * KT + (lane >> 4) * 8;
        Frag<E> f;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int col = c0 + i;
            float x = 0.f, y = 0.f;
            if (row < M && col < K) {
                if (P.mode == 2) {
                    const float2 v = S[(long long)col * M + row];
                    x = v.x;
                    y = v.y;
                } else {
                    const int ti = P.mode == 0 ? row : col, tj = P.mode == 0 ? col : row;
                    const double2 v = X[(long long)ti * n + k + tj];
                    amax = fmaxf(amax, (float)fmax(fabs(v.x), fabs(v.y)));
                    const float xh = (float)(E)v.x, yh = (float)(E)v.y;
                    f.rh[i] = (E)v.x;
                    f.ih[i] = (E)v.y;
                    f.rl[i] = (E)(v.x - (double)xh);
                    f.il[i] = (E)(v.y - (double)yh);
                    continue;
                }
            }
            const E xh = (E)x, yh = (E)y;
            f.rh[i] = xh;
            f.ih[i] = yh;
            f.rl[i] = (E)(x - (float)xh);
            f.il[i] = (E)(y - (float)yh);
        }
        out[e] = f;
    }
    if (P.tmax) {
        __shared__ float red[4];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = amax;
        __syncthreads();
        if (threadIdx.x == 0)
            atomicMax(P.tmax, __float_as_uint(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]))));
    }
}

// The dense block of a group of P sibling row decompositions (one step):
// U_g(r, off_t + i) = entry (r, i) of Pi_t [I; T_t^T], r a candidate position
// (0 <= r < n, shared by the siblings), i < k_t, off_t = k_0 + ... + k_{t-1}.
// Built from the siblings' own split tiles (A_t = T_t^T, (n - k_t) x k_t), so
// the hi / lo values are the same ones; the identity entries are exact.
struct PackGroupArgs {
    int P;
    const int* k;                 // per ID
    const long long* perm_off;
    const int* perm;
    void* const* T;               // per ID: its split tiles
    const int* nr;                // per group: n
    const int* nc;                // per group: sum of k
    const long long* tile_off;    // per group: first tile
    void* out;
    long long g0;                 // first group of this launch
};

__global__ __launch_bounds__(256) void pack_angle_kernel(PhaseDesc ph, const int* nr_, const int* nc_,
                                                         const long long* pts_off, const int* pts,
                                                         const long long* tile_off, int* out, long long b0) {
    const long long b = b0 + blockIdx.x;
    const int nr = nr_[b], nc = nc_[b];
    const int* rp = pts + pts_off[b];
    const int* cp = rp + nr;
    const int mtiles = (nr + 15) / 16, ktiles = (nc + KT - 1) / KT;
    int* o = out + tile_off[b] * 512;
    const long long n = (long long)mtiles * ktiles * 512;
    for (long long e = threadIdx.x; e < n; e += blockDim.x) {
        const int i = (int)(e & 7);
        const long long lt = e >> 3;
        const int lane = (int)(lt & 63);
        const long long tile = lt >> 6;
        const int mt = (int)(tile / ktiles), kt = (int)(tile - (long long)mt * ktiles);
        const int row = mt * 16 + (lane & 15), col = kt * KT + (lane >> 4) * 8 + i;
        int v = 0;
        if (row < nr && col < nc) {
            double f = phase_frac(ph, rp[row], cp[col]);      // [0, 1)
            if (f >= 0.5) f -= 1.0;
            v = (int)fmax(-2147483648.0, fmin(2147483647.0, rint(f * 4294967296.0)));
        }
        o[e] = v;
    }
}

constexpr int GROUP_NMAX = BF16_CROW_MAX;

template <class E>
__global__ __launch_bounds__(256) void pack_group_kernel(PackGroupArgs A) {
    __shared__ int inv[MAX_P][GROUP_NMAX];       // candidate position -> place in sibling t's permutation
    __shared__ int kt_[MAX_P], off_[MAX_P + 1];
    const long long g = A.g0 + blockIdx.x;
    const int n = A.nr[g], nc = A.nc[g], P = A.P;
    if (threadIdx.x == 0) {
        off_[0] = 0;
        for (int t = 0; t < P; ++t) {
            kt_[t] = A.k[g * P + t];
            off_[t + 1] = off_[t] + kt_[t];
        }
    }
    for (int t = 0; t < P; ++t) {
        const int* perm = A.perm + A.perm_off[g * P + t];
        for (int p = threadIdx.x; p < n; p += blockDim.x) inv[t][perm[p]] = p;
    }
    __syncthreads();
    const int mtiles = (n + 15) / 16, ktiles = (nc + KT - 1) / KT;
    Frag<E>* out = (Frag<E>*)A.out + A.tile_off[g] * 64;
    const long long nfr = (long long)mtiles * ktiles * 64;
    for (long long e = threadIdx.x; e < nfr; e += blockDim.x) {
        const int lane = (int)(e & 63);
        const long long tile = e >> 6;
        const int mt = (int)(tile / ktiles), kt = (int)(tile - (long long)mt * ktiles);
        const int row = mt * 16 + (lane & 15);
        const int c0 = kt * KT + (lane >> 4) * 8;
        Frag<E> f;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int col = c0 + i;
            E rh = (E)0.f, ih = (E)0.f, rl = (E)0.f, il = (E)0.f;
            if (row < n && col < nc) {
                int t = 0;
                while (col >= off_[t + 1]) ++t;
                const int ii = col - off_[t], k = kt_[t], pos = inv[t][row];
                if (pos < k) {
                    if (pos == ii) rh = (E)1.f;
                } else {
                    // element (j, ii) of A_t = T_t^T in its own tiles
                    const int j = pos - k, ktl = (k + KT - 1) / KT;
                    const long long stile = (long long)(j >> 4) * ktl + (ii >> 5);
                    const int sl = (j & 15) + 16 * ((ii & 31) >> 3), si = ii & 7;
                    const E* src = (const E*)((const Frag<E>*)A.T[g * P + t] + stile * 64 + sl);
                    rh = src[si];
                    ih = src[8 + si];
                    rl = src[16 + si];
                    il = src[24 + si];
                }
            }
            f.rh[i] = rh;
            f.ih[i] = ih;
            f.rl[i] = rl;
            f.il[i] = il;
        }
        out[e] = f;
    }
}

}  // namespace

void pack_angle_tiles(const PhaseDesc& ph, const int* nr, const int* nc, const long long* pts_off, const int* pts,
                      const long long* tile_off, long long count, void* out, hipStream_t s) {
    for (long long b0 = 0; b0 < count; b0 += 65535) {
        const unsigned cnt = (unsigned)std::min<long long>(65535, count - b0);
        hipLaunchKernelGGL(pack_angle_kernel, dim3(cnt), dim3(256), 0, s, ph, nr, nc, pts_off, pts, tile_off,
                           (int*)out, b0);
        MIDBF_HIP(hipGetLastError());
    }
}

void launch_col_exponents(const ColExpArgs& A, hipStream_t s) {
    MIDBF_CHECK(A.S >= 1 && A.S <= 65535 && A.nrhs >= 1 && A.nrhs <= 65535, MIDBF_ERR_ARG,
                "column exponent pass: bad slice or column count");
    hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)A.S, (unsigned)A.nrhs), dim3(256), 0, s, A);
    MIDBF_HIP(hipGetLastError());
    hipLaunchKernelGGL(colexp_kernel, dim3(1), dim3(256), 0, s, A);
    MIDBF_HIP(hipGetLastError());
}

void pack_src_lattice(const int* skel, const int* src, long long count, int* out, hipStream_t st) {
    if (count <= 0) return;
    const long long blocks = (count + 255) / 256;
    hipLaunchKernelGGL(src_lattice_kernel, dim3((unsigned)blocks), dim3(256), 0, st, skel, src, count, out);
    MIDBF_HIP(hipGetLastError());
}

void pack_src_rows(const ApplyGeom& G, int s, long long Ps, const int* n, const long long* perm_off, const int* perm,
                   const int* k_prev, const long long* yoff_prev, long long nid, int* out, hipStream_t st) {
    for (long long i0 = 0; i0 < nid; i0 += 65535) {
        const unsigned cnt = (unsigned)std::min<long long>(65535, nid - i0);
        SrcRowsArgs A{G, s, Ps, n, perm_off, perm, k_prev, yoff_prev, out, i0};
        hipLaunchKernelGGL(src_rows_kernel, dim3(cnt), dim3(256), 0, st, A);
        MIDBF_HIP(hipGetLastError());
    }
}

void pack_group_tiles(int elem, int P, const int* k, const long long* perm_off, const int* perm, void* const* T,
                      const int* nr, const int* nc, const long long* tile_off, long long groups, void* out,
                      hipStream_t s) {
    for (long long g0 = 0; g0 < groups; g0 += 65535) {
        const unsigned cnt = (unsigned)std::min<long long>(65535, groups - g0);
        PackGroupArgs A{P, k, perm_off, perm, T, nr, nc, tile_off, out, g0};
        if (elem == SPLIT16_FP16) hipLaunchKernelGGL(pack_group_kernel<_Float16>, dim3(cnt), dim3(256), 0, s, A);
        else hipLaunchKernelGGL(pack_group_kernel<__bf16>, dim3(cnt), dim3(256), 0, s, A);
        MIDBF_HIP(hipGetLastError());
    }
}

namespace {
// Up and middle with multi-tile B stages and streamed A; down with z resident
// (ranks beyond the resident capacity run W0).  NT = 512, 768 or 1024 threads.
// TWO: the middle kinds (phase-tile middle, dense group down) in the form
// that puts two workgroups on a CU.
template <class E, int NT, bool TWO = false>
void launch_res16(LevelKernel which, const void* args, long long count, int nrhs, void* scratch,
                  const long long* tile_off, hipStream_t s) {
    const dim3 grid((unsigned)count, (nrhs + NRHS - 1) / NRHS);
    if (which == LevelKernel::Up) {
        const UpArgs& a = *(const UpArgs*)args;
        MIDBF_CHECK(a.lev.src != nullptr, MIDBF_ERR_ARG, "the split up kernels need the level's source-row table");
        const bool res = a.nred_max <= RES_KT * KT;
        if (a.presplit > 0.f) {
            if (res) hipLaunchKernelGGL((up_res16<E, NT, true, true>), grid, dim3(NT), 0, s, a, count);
            else hipLaunchKernelGGL((up_res16<E, NT, false, true>), grid, dim3(NT), 0, s, a, count);
        } else {
            if (res) hipLaunchKernelGGL((up_res16<E, NT, true>), grid, dim3(NT), 0, s, a, count);
            else hipLaunchKernelGGL((up_res16<E, NT, false>), grid, dim3(NT), 0, s, a, count);
        }
    }
    else if (which == LevelKernel::Middle) {
        // one workgroup per chunk of NT / 64 row tiles of a block
        MidArgs a = *(const MidArgs*)args;
        MIDBF_CHECK(a.ang || a.bscale == 1.f, MIDBF_ERR_ARG, "a scale change needs the middle's phase tiles");
        a.mchunks = std::max(1, (a.out_max + NT / 4 - 1) / (NT / 4));
        const dim3 mgrid((unsigned)(count * a.mchunks), grid.y);
        MIDBF_CHECK(!a.presplit || a.ang, MIDBF_ERR_ARG, "split vectors go to the phase-tile middle only");
        if (a.ang && a.presplit)
            hipLaunchKernelGGL((middle_res16<E, NT, true, TWO, true>), mgrid, dim3(NT), 0, s, a, tile_off);
        else if (a.ang) hipLaunchKernelGGL((middle_res16<E, NT, true, TWO>), mgrid, dim3(NT), 0, s, a, tile_off);
        else hipLaunchKernelGGL((middle_res16<E, NT, false, TWO>), mgrid, dim3(NT), 0, s, a, tile_off);
    }
    else if (which == LevelKernel::Down && ((const DownArgs*)args)->kmax <= RES_KT * KT)
        hipLaunchKernelGGL((down_res16<E, NT>), grid, dim3(NT), 0, s, *(const DownArgs*)args, count,
                           (float2*)scratch);
    else if (which == LevelKernel::DownGroup) {
        const DownArgs& a = *(const DownArgs*)args;
        MIDBF_CHECK(a.kmax <= RES_KT * KT, MIDBF_ERR_ARG, "grouped down pass needs ranks <= 256");
        constexpr int GNT = NT == 1024 ? 768 : NT;     // the 16-wave build would spill
        hipLaunchKernelGGL((down_group16<E, GNT>), grid, dim3(GNT), sizeof(int) * a.ncand_max, s, a);
    }
    else
        launch_bvariant<W0, E>(which, args, count, nrhs, scratch, tile_off, s);
    MIDBF_HIP(hipGetLastError());
}

template <class E>
void launch_split16(LevelKernel which, int variant, const void* args, long long count, int nrhs, void* scratch,
                    const long long* tile_off, hipStream_t s) {
    switch (variant) {
        case 0: launch_bvariant<W0, E>(which, args, count, nrhs, scratch, tile_off, s); break;
        case 1: launch_bvariant<W1, E>(which, args, count, nrhs, scratch, tile_off, s); break;
        case 2: launch_bvariant<W2, E>(which, args, count, nrhs, scratch, tile_off, s); break;
        case 3: launch_bvariant<W3, E>(which, args, count, nrhs, scratch, tile_off, s); break;
        case 4: launch_bvariant<W4, E>(which, args, count, nrhs, scratch, tile_off, s); break;
        case 7: launch_res16<E, 512>(which, args, count, nrhs, scratch, tile_off, s); break;
        case 8: launch_res16<E, 1024>(which, args, count, nrhs, scratch, tile_off, s); break;
        case 9: launch_res16<E, 768>(which, args, count, nrhs, scratch, tile_off, s); break;
        case 10:
            // the middle kinds with two workgroups per CU; the other kinds as variant 9
            if (which == LevelKernel::Middle) launch_res16<E, 512, true>(which, args, count, nrhs, scratch, tile_off, s);
            else launch_res16<E, 768>(which, args, count, nrhs, scratch, tile_off, s);
            break;
        case 5:
        case 6: {
            // down with z resident in LDS (variant 5: 512 threads, 6: 1024); other kinds, or ranks
            // beyond the resident capacity, run W0 / W3
            if (which == LevelKernel::DownGroup) {
                if (variant == 5) launch_res16<E, 512>(which, args, count, nrhs, scratch, tile_off, s);
                else launch_res16<E, 1024>(which, args, count, nrhs, scratch, tile_off, s);
                break;
            }
            const bool res = which == LevelKernel::Down && ((const DownArgs*)args)->kmax <= RES_KT * KT;
            if (!res) {
                if (variant == 5) launch_bvariant<W0, E>(which, args, count, nrhs, scratch, tile_off, s);
                else launch_bvariant<W3, E>(which, args, count, nrhs, scratch, tile_off, s);
                break;
            }
            const dim3 grid((unsigned)count, (nrhs + NRHS - 1) / NRHS);
            if (variant == 5)
                hipLaunchKernelGGL((down_res16<E, 512>), grid, dim3(512), 0, s, *(const DownArgs*)args, count,
                                   (float2*)scratch);
            else
                hipLaunchKernelGGL((down_res16<E, 1024>), grid, dim3(1024), 0, s, *(const DownArgs*)args, count,
                                   (float2*)scratch);
            MIDBF_HIP(hipGetLastError());
            break;
        }
        default: throw Error(MIDBF_ERR_ARG, "unknown split-16-bit variant");
    }
}

void launch_pack(const PackTilesArgs& P, int elem, unsigned count, hipStream_t s) {
    if (elem == SPLIT16_FP16) hipLaunchKernelGGL(pack_tiles_kernel<_Float16>, dim3(count), dim3(256), 0, s, P);
    else hipLaunchKernelGGL(pack_tiles_kernel<__bf16>, dim3(count), dim3(256), 0, s, P);
    MIDBF_HIP(hipGetLastError());
}
}  // namespace

void launch_bf16_kernel(int elem, LevelKernel which, int variant, const void* args, long long count, int nrhs,
                        void* scratch, const long long* tile_off, hipStream_t s) {
    if (which == LevelKernel::DownDense) which = LevelKernel::Middle;     // same kernels, group blocks
    if (which == LevelKernel::DownLeaf) {
        const DownArgs& a = *(const DownArgs*)args;
        MIDBF_CHECK(a.G.n0 <= LEAF_MAX && a.s == 0, MIDBF_ERR_ARG, "leaf down pass needs n0 <= 64 at the leaves");
        const dim3 grid((unsigned)count, (nrhs + NRHS - 1) / NRHS);
        if (elem == SPLIT16_FP16) hipLaunchKernelGGL(down_leaf16<_Float16>, grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL(down_leaf16<__bf16>, grid, dim3(256), 0, s, a);
        MIDBF_HIP(hipGetLastError());
        return;
    }
    if (elem == SPLIT16_FP16) launch_split16<_Float16>(which, variant, args, count, nrhs, scratch, tile_off, s);
    else launch_split16<__bf16>(which, variant, args, count, nrhs, scratch, tile_off, s);
}

long long bf16_tiles(int M, int K) { return (long long)((M + 15) / 16) * ((K + KT - 1) / KT); }

void pack_bf16_slab(int elem, const double2* X, long long x_stride, const int* k_w, const int* n_w, int count,
                    bool transposed, void* out, const long long* tile_off, unsigned* tmax, hipStream_t s) {
    if (count <= 0) return;
    PackTilesArgs P{transposed ? 1 : 0, X, x_stride, k_w, n_w, nullptr, nullptr, nullptr, nullptr, out, tile_off, tmax};
    launch_pack(P, elem, (unsigned)count, s);
}

void pack_bf16_blocks(int elem, const float2* S, const long long* s_off, const int* nr, const int* nc,
                      long long count, void* out, const long long* tile_off, hipStream_t s) {
    for (long long b0 = 0; b0 < count; b0 += 65535) {
        const long long cnt = std::min<long long>(65535, count - b0);
        PackTilesArgs P{2, nullptr, 0, nullptr, nullptr, S, s_off + b0, nr + b0, nc + b0, out, tile_off + b0, nullptr};
        launch_pack(P, elem, (unsigned)cnt, s);
    }
}

}  // namespace midbf
