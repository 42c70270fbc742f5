// Factor construction (Sec. 3.1-3.5): trees, Mock-Chebyshev samples, batched
// interpolative decompositions per unrolled MSCS step, factor packing and
// the middle blocks.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "build.h"
#include "id.h"
#include "mfma.h"

namespace midbf {

namespace {

constexpr int BT = 256;

// ---- kernels ------------------------------------------------------------

struct CandArgs {
    int s, P, d, n, L, leaf, la, lb;
    long long id0, Ps;          // first ID of the wave; P^s
    long long nB;               // partners per node, P^lb
    const int* n_arr;           // per wave ID
    const int* k_prev;
    const long long* yoff_prev;
    const int* skel_prev;
    int* cand;                  // wave x nmax
    int nmax;
    const int* slot;            // scattered points: leaf slot table of the candidate tree, or null
    int n0;                     // slots per leaf
};

// Candidate points of each decomposition: the points of the leaf (s = 0) or
// the children's skeletons against the partner's parent.
__global__ void cand_kernel(CandArgs A) {
    const int w = blockIdx.x;
    const long long id = A.id0 + w;
    const long long a = id / A.nB, bb = id - (id / A.nB) * A.nB;
    const int ncand = A.n_arr[w];
    int* out = A.cand + (long long)w * A.nmax;
    if (A.s == 0) {
        if (A.slot) {
            for (int c = threadIdx.x; c < ncand; c += BT) out[c] = A.slot[a * A.n0 + c];
            return;
        }
        int origin[3];
        node_origin(a, A.L, A.d, A.n, origin);
        for (int c = threadIdx.x; c < ncand; c += BT) out[c] = (int)box_point(origin, A.leaf, c, A.d, A.n);
        return;
    }
    const long long pb = bb / A.P;
    int start = 0;
    for (int t = 0; t < A.P; ++t) {
        const long long idp = ((long long)A.P * a + t) * A.Ps + pb;
        const int len = A.k_prev[idp];
        const long long off = A.yoff_prev[idp];
        for (int c = threadIdx.x; c < len; c += BT) out[start + c] = A.skel_prev[off + c];
        start += len;
    }
}

struct GenArgs {
    PhaseDesc ph;
    int side, lb;
    long long id0, nB;
    int m;
    const int* samples;         // local indices within the partner box (m)
    int box_side;
    const int* n_arr;
    const int* cand;
    int nmax;
    double2* X;
    long long x_stride;
    const int* samp_tab;        // scattered points: per partner node m sample point numbers (-1: none), or null
};

// Sample matrix of decomposition w, row-major m x n (rows of missing samples zero):
//   row side:    X[i][c] = K(x = cand_c, xi = sample_i)   (X = K(cand, samples)^T)
//   column side: X[i][c] = K(x = sample_i, xi = cand_c)   (X = K(samples, cand))
__global__ void gen_kernel(GenArgs A) {
    const int w = blockIdx.y;
    const long long id = A.id0 + w;
    const long long bb = id - (id / A.nB) * A.nB;
    const int n = A.n_arr[w];
    int origin[3];
    node_origin(bb, A.lb, A.ph.d, A.ph.n, origin);
    const int* cand = A.cand + (long long)w * A.nmax;
    double2* X = A.X + (long long)w * A.x_stride;
    const long long total = (long long)A.m * n;
    for (long long e = (long long)blockIdx.x * BT + threadIdx.x; e < total; e += (long long)gridDim.x * BT) {
        const int i = (int)(e / n), c = (int)(e - (e / n) * n);
        const long long sp = A.samp_tab ? (long long)A.samp_tab[bb * A.m + i]
                                        : box_point(origin, A.box_side, A.samples[i], A.ph.d, A.ph.n);
        const long long cp = cand[c];
        if (sp < 0) X[e] = make_double2(0.0, 0.0);
        else X[e] = (A.side == SIDE_ROW) ? kernel_entry(A.ph, cp, sp) : kernel_entry(A.ph, sp, cp);
    }
}

struct PackArgs {
    int side;
    long long id0;
    const int* k_w;
    const int* n_w;
    const double2* X;
    long long x_stride;
    const int* perm_w;
    long long p_stride;
    const int* cand;
    int nmax;
    const long long* toff_w;    // per wave ID: element offset of T in the wave's chunk
    double2* T64;
    float2* T32;
    const long long* perm_off;  // level tables (global ID)
    const long long* y_off;
    int* perm;
    int* skel;
};

// Copy T of each decomposition into the factor store (column-major k x (n-k)
// for the column side, row-major for the row side), its candidate
// permutation, and its skeleton lattice points.
__global__ void pack_kernel(PackArgs A) {
    const int w = blockIdx.x;
    const long long id = A.id0 + w;
    const int k = A.k_w[w], n = A.n_w[w], nred = n - k;
    const double2* X = A.X + (long long)w * A.x_stride;
    const int* pw = A.perm_w + (long long)w * A.p_stride;
    const int* cand = A.cand + (long long)w * A.nmax;
    int* pd = A.perm + A.perm_off[id];
    for (int j = threadIdx.x; j < n; j += BT) pd[j] = pw[j];
    int* sk = A.skel + A.y_off[id];
    for (int i = threadIdx.x; i < k; i += BT) sk[i] = cand[pw[i]];
    const long long to = A.toff_w[w];
    const long long tot = (long long)k * nred;
    for (long long e = threadIdx.x; e < tot; e += BT) {
        int i, j;
        if (A.side == SIDE_COL) { j = (int)(e / k); i = (int)(e - (long long)j * k); }
        else { i = (int)(e / nred); j = (int)(e - (long long)i * nred); }
        const double2 v = X[(long long)i * n + k + j];
        if (A.T64) A.T64[to + e] = v;
        if (A.T32) A.T32[to + e] = make_float2((float)v.x, (float)v.y);
    }
}

// The inverse of pack_kernel's T mapping: a T block in the stored order back into the
// decomposition slab (X[i][k + j]), for factors read from a file.
struct UnpackArgs {
    int side;
    const int* k_w;
    const int* n_w;
    double2* X;
    long long x_stride;
    const long long* toff_w;
    const double2* T;
};

__global__ void unpack_kernel(UnpackArgs A) {
    const int w = blockIdx.x;
    const int k = A.k_w[w], n = A.n_w[w], nred = n - k;
    double2* X = A.X + (long long)w * A.x_stride;
    const long long to = A.toff_w[w];
    const long long tot = (long long)k * nred;
    for (long long e = threadIdx.x; e < tot; e += BT) {
        int i, j;
        if (A.side == SIDE_COL) { j = (int)(e / k); i = (int)(e - (long long)j * k); }
        else { i = (int)(e / nred); j = (int)(e - (long long)i * nred); }
        X[(long long)i * n + k + j] = A.T[to + e];
    }
}

struct MidGenArgs {
    PhaseDesc ph;
    const int* nr;
    const int* nc;
    const long long* off;       // element offset of block bi
    const long long* pts_off;   // offset of block bi's row points, then column points
    const int* pts;
    double2* S64;
    float2* S32;
};

// Middle block bi, column-major nr x nc: S = K(row skeletons, column skeletons).
__global__ void midgen_kernel(MidGenArgs A) {
    const long long bi = blockIdx.y;
    const int nr = A.nr[bi], nc = A.nc[bi];
    const int* rp = A.pts + A.pts_off[bi];
    const int* cp = rp + nr;
    const long long base = A.off[bi];
    const long long tot = (long long)nr * nc;
    for (long long e = (long long)blockIdx.x * BT + threadIdx.x; e < tot; e += (long long)gridDim.x * BT) {
        const int c = (int)(e / nr), r = (int)(e - (long long)c * nr);
        const double2 v = kernel_entry(A.ph, rp[r], cp[c]);
        if (A.S64) A.S64[base + e] = v;
        if (A.S32) A.S32[base + e] = make_float2((float)v.x, (float)v.y);
    }
}

__global__ void entries_kernel(PhaseDesc ph, const int* rows, int nrows, const int* cols, int ncols, double2* out) {
    const long long tot = (long long)nrows * ncols;
    for (long long e = (long long)blockIdx.x * BT + threadIdx.x; e < tot; e += (long long)gridDim.x * BT) {
        const int i = (int)(e / ncols), j = (int)(e - (long long)i * ncols);
        out[e] = kernel_entry(ph, rows[i], cols[j]);
    }
}

__global__ void copy_T_kernel(const double2* X, long long x_stride, const int* k_arr, int m, int n, double2* T) {
    const int b = blockIdx.x;
    const int k = k_arr[b], nred = n - k;
    const double2* src = X + (long long)b * x_stride;
    double2* dst = T + (long long)b * m * n;
    for (long long e = threadIdx.x; e < (long long)k * nred; e += BT) {
        const int i = (int)(e / nred), j = (int)(e - (long long)i * nred);
        dst[e] = src[(long long)i * n + k + j];
    }
}

// ---- host helpers -------------------------------------------------------

template <class T> T* dalloc(size_t count) {
    T* p = nullptr;
    if (count == 0) count = 1;
    MIDBF_HIP(hipMalloc((void**)&p, count * sizeof(T)));
    return p;
}

template <class T> void upload(T* dst, const std::vector<T>& src, hipStream_t s) {
    if (!src.empty()) MIDBF_HIP(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Local indices (C order inside a box of the given side) of the Mock-
// Chebyshev samples: per dimension q = ceil(count^(1/d)) Chebyshev-Lobatto
// nodes over [0, side-1] rounded to the nearest index (duplicates removed);
// the whole box when q >= side (Sec. 3.2).
std::vector<int> mock_chebyshev_local(int d, int side, long long count) {
    int q = 1;
    while (ipow(q, d) < count) ++q;
    std::vector<int> loc;
    if (q >= side) {
        for (int i = 0; i < side; ++i) loc.push_back(i);
    } else {
        for (int j = 0; j < q; ++j) {
            double node = 0.5 * (side - 1) * (1.0 - std::cos(M_PI * j / (q - 1)));
            int v = (int)std::floor(node + 0.5);
            if (loc.empty() || loc.back() != v) loc.push_back(v);
        }
    }
    std::vector<int> out;
    const int l = (int)loc.size();
    long long tot = ipow(l, d);
    out.reserve(tot);
    for (long long e = 0; e < tot; ++e) {
        long long r = e;
        int idx = 0;
        int mul = 1;
        int digits[3];
        for (int qd = d - 1; qd >= 0; --qd) { digits[qd] = loc[r % l]; r /= l; }
        idx = 0;
        for (int qd = 0; qd < d; ++qd) idx = idx * side + digits[qd];
        (void)mul;
        out.push_back(idx);
    }
    return out;
}

void free_level(LevelSide& lv) {
    auto f = [](void* p) { if (p) (void)hipFree(p); };
    f(lv.d_k); f(lv.d_n); f(lv.d_perm_off); f(lv.d_y_off); f(lv.d_perm); f(lv.d_skel);
    for (int q = 0; q < NPREC; ++q) f(lv.d_T[q]);
    for (void* c : lv.chunks) f(c);
    lv.d_k = lv.d_n = nullptr; lv.d_perm_off = lv.d_y_off = nullptr; lv.d_perm = lv.d_skel = nullptr;
    lv.d_src = nullptr;
    lv.d_src_lat = nullptr;
    for (int q = 0; q < NPREC; ++q) lv.d_T[q] = nullptr;
    lv.chunks.clear();
    lv.t64.clear();
}

struct Scratch {
    double2* X = nullptr; double2* V = nullptr; double2* Y = nullptr;
    int* perm = nullptr; int* cand = nullptr; int* k = nullptr; int* n = nullptr; long long* toff = nullptr;
    long long* tile_off = nullptr;
    int* samples = nullptr;
    int* samp_tab = nullptr;                 // scattered points: per partner node sample lists
    int* m_arr = nullptr;                    // scattered points: samples of each ID of a wave
    hipEvent_t ev[2] = {nullptr, nullptr};   // brackets of the ID launches
    long long wave = 0, xs = 0, vs = 0, ys = 0, nmax = 0;
    void release() {
        auto f = [](void* p) { if (p) (void)hipFree(p); };
        f(X); f(V); f(Y); f(perm); f(cand); f(k); f(n); f(toff); f(samples); f(tile_off); f(samp_tab); f(m_arr);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        *this = Scratch();
    }
};

// ---- scattered points (Sec. 3.5, closing paragraph) ----------------------------------------
// A point tree uses the boxes of the lattice tree: leaf of a point = the Z-order number of its box
// at level L (digit j, root first, holds bit L-1-j of every box coordinate; coordinate 1 is the
// most significant bit, Fig. 4).  Points are listed leaf by leaf and by increasing number inside a
// leaf, so node (level, i) holds one contiguous run of the list; an empty node holds none.

// Points leaf by leaf (order) and the start of every leaf's run (P^L + 1 entries).
void point_tree(const std::vector<double>& pts, int d, int L, std::vector<int>& order,
                std::vector<long long>& start) {
    const long long N = (long long)pts.size() / d;
    const int P = 1 << d, side = 1 << L;
    const long long nleaf = ipow(P, L);
    std::vector<long long> leaf(N);
    for (long long i = 0; i < N; ++i) {
        long long cell[3];
        for (int q = 0; q < d; ++q)
            cell[q] = std::min<long long>(side - 1, std::max<long long>(0, (long long)std::floor(pts[i * d + q] * side)));
        long long lf = 0;
        for (int j = 0; j < L; ++j) {
            const int bit = L - 1 - j;
            long long digit = 0;
            for (int q = 0; q < d; ++q) digit |= ((cell[q] >> bit) & 1) << (d - 1 - q);
            lf = lf * P + digit;
        }
        leaf[i] = lf;
    }
    start.assign(nleaf + 1, 0);
    for (long long i = 0; i < N; ++i) ++start[leaf[i] + 1];
    for (long long l = 0; l < nleaf; ++l) start[l + 1] += start[l];
    order.assign(N, 0);
    std::vector<long long> fill(start.begin(), start.end() - 1);
    for (long long i = 0; i < N; ++i) order[fill[leaf[i]]++] = (int)i;     // counting sort, stable in i
}

// Mock-Chebyshev samples of node (level, idx) for scattered points (Sec. 3.2): q = ceil(want^(1/d))
// Chebyshev-Lobatto nodes per dimension over the bounding box of the node's points; for every node
// of the tensor grid (C order) the nearest point (ties: the larger point number), duplicates
// removed in first-seen order.  A node with at most q^d points is taken whole.
std::vector<int> point_samples(const std::vector<double>& pts, int d, int L, const std::vector<int>& order,
                               const std::vector<long long>& start, int level, long long idx, long long want) {
    const long long w = ipow(1 << d, L - level);
    const long long a = start[idx * w], e = start[(idx + 1) * w];
    int q = 1;
    while (ipow(q, d) < want) ++q;
    std::vector<int> out;
    if (e - a <= ipow(q, d)) {
        out.assign(order.begin() + a, order.begin() + e);
        return out;
    }
    double lo[3], hi[3];
    for (int k = 0; k < d; ++k) { lo[k] = 1e300; hi[k] = -1e300; }
    for (long long t = a; t < e; ++t)
        for (int k = 0; k < d; ++k) {
            const double v = pts[(long long)order[t] * d + k];
            lo[k] = std::min(lo[k], v);
            hi[k] = std::max(hi[k], v);
        }
    std::vector<double> c(q);
    for (int j = 0; j < q; ++j) c[j] = q == 1 ? 0.5 : 0.5 * (1.0 - std::cos(M_PI * j / (q - 1)));
    const long long G = ipow(q, d);
    std::vector<char> seen;
    std::vector<int> picked;
    picked.reserve(G);
    for (long long gi = 0; gi < G; ++gi) {
        double g[3];
        long long r = gi;
        for (int k = d - 1; k >= 0; --k) { g[k] = lo[k] + (hi[k] - lo[k]) * c[r % q]; r /= q; }
        double best = 1e300;
        int bp = -1;
        for (long long t = a; t < e; ++t) {
            const int p = order[t];
            double s = 0.0;
            for (int k = 0; k < d; ++k) {
                const double dv = g[k] - pts[(long long)p * d + k];
                s += dv * dv;
            }
            if (s < best || (s == best && p > bp)) { best = s; bp = p; }
        }
        picked.push_back(bp);
    }
    std::vector<int> sorted(picked);
    std::sort(sorted.begin(), sorted.end());
    sorted.erase(std::unique(sorted.begin(), sorted.end()), sorted.end());
    seen.assign(sorted.size(), 0);
    for (int p : picked) {
        const size_t pos = std::lower_bound(sorted.begin(), sorted.end(), p) - sorted.begin();
        if (!seen[pos]) { seen[pos] = 1; out.push_back(p); }
    }
    return out;
}

// The decompositions of one step and side as read from a factor file: sample
// count, candidate count and rank per ID, pivot orders (concatenated) and the
// FP64 T blocks in pack_kernel's stored order (concatenated).
struct ReplayLevel {
    int m = 0;
    std::vector<int> n, k, perm;
    std::vector<double2> T;
};

// Decompositions of one step and side.  Returns false if some ID kept as
// many pivots as it had samples while more samples were available.  With rl,
// the decompositions come from a factor file instead of samples and pivoted QR.
bool build_level(midbf_plan* h, LevelSide& lv, const LevelSide* prev, long long want, hipStream_t st,
                 const ReplayLevel* rl = nullptr) {
    const int P = h->P, d = h->d;
    const int side_len = h->n >> lv.lb;
    const long long nid = lv.nid;
    const long long nB = ipow(P, lv.lb);
    const long long Ps = ipow(P, lv.s);
    // the candidate tree is this side's (rows: x, columns: xi), the samples come from the other
    const int ct = lv.side == SIDE_ROW ? 0 : 1, stt = 1 - ct;
    std::vector<int> samples;
    std::vector<int> m_part, size_part, samp_tab;      // scattered points, per partner node
    if (rl) lv.m = rl->m;
    else if (h->points) {
        std::vector<std::vector<int>> lists(nB);
        m_part.assign(nB, 0);
        size_part.assign(nB, 0);
        int mm = 1;
        const long long w = ipow(P, h->L - lv.lb);
        for (long long bb = 0; bb < nB; ++bb) {
            lists[bb] = point_samples(h->tree_pts[stt], d, h->L, h->tree_order[stt], h->tree_start[stt], lv.lb, bb,
                                      want);
            m_part[bb] = (int)lists[bb].size();
            size_part[bb] = (int)(h->tree_start[stt][(bb + 1) * w] - h->tree_start[stt][bb * w]);
            mm = std::max(mm, m_part[bb]);
        }
        lv.m = mm;
        samp_tab.assign((size_t)nB * mm, -1);
        for (long long bb = 0; bb < nB; ++bb)
            std::copy(lists[bb].begin(), lists[bb].end(), samp_tab.begin() + bb * mm);
    } else {
        samples = mock_chebyshev_local(d, side_len, want);
        lv.m = (int)samples.size();
    }
    MIDBF_CHECK(lv.m <= ID_MMAX, MIDBF_ERR_SHAPE, "too many samples per decomposition");
    // candidate counts
    lv.n.assign(nid, 0);
    for (long long id = 0; id < nid; ++id) {
        if (lv.s == 0) {
            const long long a = id / nB;
            lv.n[id] = h->points ? (int)(h->tree_start[ct][a + 1] - h->tree_start[ct][a]) : h->n0;
            continue;
        }
        const long long a = id / nB, pb = (id % nB) / P;
        int c = 0;
        for (int t = 0; t < P; ++t) c += prev->k[((long long)P * a + t) * Ps + pb];
        lv.n[id] = c;
    }
    lv.nmax = std::max(1, *std::max_element(lv.n.begin(), lv.n.end()));
    MIDBF_CHECK(lv.nmax <= ID_NMAX, MIDBF_ERR_SHAPE, "too many candidates per decomposition (rank too large)");
    if (rl) MIDBF_CHECK(rl->n == lv.n, MIDBF_ERR_IO, "factor file: candidate counts do not follow from its ranks");
    lv.perm_off.assign(nid + 1, 0);
    for (long long id = 0; id < nid; ++id) lv.perm_off[id + 1] = lv.perm_off[id] + lv.n[id];
    lv.total_n = lv.perm_off[nid];
    lv.perm_off.resize(nid);
    lv.k.assign(nid, 0);
    lv.y_off.assign(nid, 0);

    lv.d_k = dalloc<int>(nid);
    lv.d_n = dalloc<int>(nid);
    lv.d_perm_off = dalloc<long long>(nid);
    lv.d_y_off = dalloc<long long>(nid);
    lv.d_perm = dalloc<int>(lv.total_n);
    lv.d_skel = dalloc<int>(lv.total_n);
    upload(lv.d_n, lv.n, st);
    upload(lv.d_perm_off, lv.perm_off, st);
    for (int q = 0; q < NPREC; ++q)
        if (h->keep & (1u << q)) lv.d_T[q] = (void**)dalloc<void*>(nid);

    // wave size from the workspace budget
    const long long nmax = lv.nmax, m = lv.m;
    const long long per = (m * nmax + m * ID_NB + (long long)ID_ELL * nmax) * 16 + nmax * 8 + 64;
    long long wave = (long long)(h->p.build_workspace_bytes / per);
    wave = std::max<long long>(1, std::min<long long>(wave, nid));
    wave = std::min<long long>(wave, 65535);
    Scratch sc;
    sc.wave = wave; sc.nmax = nmax;
    sc.xs = m * nmax; sc.vs = m * ID_NB; sc.ys = (long long)ID_ELL * nmax;
    sc.X = dalloc<double2>(wave * sc.xs);
    sc.V = dalloc<double2>(wave * sc.vs);
    sc.Y = dalloc<double2>(wave * sc.ys);
    sc.perm = dalloc<int>(wave * nmax);
    sc.cand = dalloc<int>(wave * nmax);
    sc.k = dalloc<int>(wave);
    sc.toff = dalloc<long long>(wave);
    sc.tile_off = dalloc<long long>(wave);
    if (!rl && !h->points) {
        sc.samples = dalloc<int>(m);
        upload(sc.samples, samples, st);
    }
    if (!rl && h->points) {
        sc.samp_tab = dalloc<int>(samp_tab.size());
        upload(sc.samp_tab, samp_tab, st);
        sc.m_arr = dalloc<int>(wave);
    }
    for (hipEvent_t& e : sc.ev) MIDBF_HIP(hipEventCreate(&e));
    long long t_read = 0;      // replay: T entries of the waves done
    hipEvent_t* ev = sc.ev;

    bool saturated = false;
    long long yrun = 0;
    const long long box_pts = ipow(side_len, d);
    try {
        for (long long id0 = 0; id0 < nid; id0 += wave) {
            const int cnt = (int)std::min<long long>(wave, nid - id0);
            CandArgs ca{lv.s, P, d, h->n, h->L, h->leaf, lv.la, lv.lb, id0, Ps, nB, lv.d_n + id0,
                        prev ? prev->d_k : nullptr, prev ? prev->d_y_off : nullptr, prev ? prev->d_skel : nullptr,
                        sc.cand, (int)nmax, h->points ? h->d_slot[ct] : nullptr, h->n0};
            hipLaunchKernelGGL(cand_kernel, dim3(cnt), dim3(BT), 0, st, ca);
            MIDBF_HIP(hipGetLastError());
            std::vector<int> kw(cnt);
            if (!rl) {
                GenArgs ga{h->ph, lv.side, lv.lb, id0, nB, (int)m, sc.samples, side_len, lv.d_n + id0, sc.cand,
                           (int)nmax, sc.X, sc.xs, sc.samp_tab};
                if (h->points) {
                    std::vector<int> mw(cnt);
                    for (int w = 0; w < cnt; ++w) mw[w] = m_part[(id0 + w) % nB];
                    upload(sc.m_arr, mw, st);
                    MIDBF_HIP(hipStreamSynchronize(st));
                }
                const int gx = (int)std::min<long long>((m * nmax + BT - 1) / BT, 64);
                hipLaunchKernelGGL(gen_kernel, dim3(gx, cnt), dim3(BT), 0, st, ga);
                MIDBF_HIP(hipGetLastError());
                IdBatch ib{sc.X, sc.xs, sc.V, sc.vs, sc.Y, sc.ys, sc.perm, nmax, sc.k, lv.d_n + id0, 0, (int)m,
                           h->p.tol, h->p.k_cap, 0x5eedu + (unsigned)(lv.s * 2 + lv.side), h->p.fixed_rank, sc.m_arr};
                MIDBF_HIP(hipEventRecord(ev[0], st));
                launch_id_batch(ib, cnt, st);
                MIDBF_HIP(hipEventRecord(ev[1], st));
                MIDBF_HIP(hipMemcpyAsync(kw.data(), sc.k, cnt * sizeof(int), hipMemcpyDeviceToHost, st));
                MIDBF_HIP(hipStreamSynchronize(st));
                float id_ms = 0.f;
                MIDBF_HIP(hipEventElapsedTime(&id_ms, ev[0], ev[1]));
                h->stats.id_ms += id_ms;
                for (int w = 0; w < cnt; ++w) {
                    h->stats.id_flops += 8.0 * (double)m * lv.n[id0 + w] * kw[w];
                    h->stats.id_bytes += 16.0 * (double)m * lv.n[id0 + w];
                }
            } else {
                // ranks, pivot orders and T blocks of this wave from the file, into the slab layout
                // the packing below reads (T at X[i][k + j], pivots at perm + w * nmax)
                std::copy(rl->k.begin() + id0, rl->k.begin() + id0 + cnt, kw.begin());
                std::vector<int> pw((size_t)cnt * nmax, 0);
                std::vector<long long> tof(cnt);
                long long tsum = 0;
                for (int w = 0; w < cnt; ++w) {
                    const long long id = id0 + w;
                    std::copy(rl->perm.begin() + lv.perm_off[id], rl->perm.begin() + lv.perm_off[id] + lv.n[id],
                              pw.begin() + (size_t)w * nmax);
                    tof[w] = tsum;
                    tsum += (long long)kw[w] * (lv.n[id] - kw[w]);
                }
                upload(sc.k, kw, st);
                upload(sc.perm, pw, st);
                upload(sc.toff, tof, st);
                double2* stage = dalloc<double2>(std::max<long long>(tsum, 1));
                try {
                    MIDBF_HIP(hipMemcpyAsync(stage, rl->T.data() + t_read, tsum * sizeof(double2),
                                             hipMemcpyHostToDevice, st));
                    UnpackArgs ua{lv.side, sc.k, lv.d_n + id0, sc.X, sc.xs, sc.toff, stage};
                    hipLaunchKernelGGL(unpack_kernel, dim3(cnt), dim3(BT), 0, st, ua);
                    MIDBF_HIP(hipGetLastError());
                    MIDBF_HIP(hipStreamSynchronize(st));
                } catch (...) {
                    (void)hipFree(stage);
                    throw;
                }
                (void)hipFree(stage);
                t_read += tsum;
            }
            std::vector<long long> toff(cnt);
            long long tw = 0;
            for (int w = 0; w < cnt; ++w) {
                const long long id = id0 + w;
                const int k = kw[w], nn = lv.n[id];
                if (!rl && !h->points && k >= m && m < box_pts && m < nn) saturated = true;
                if (!rl && h->points) {
                    const int mp = m_part[id % nB];
                    if (k >= mp && mp < size_part[id % nB] && mp < nn) saturated = true;
                }
                lv.k[id] = k;
                lv.y_off[id] = yrun;
                yrun += k;
                toff[w] = tw;
                tw += (long long)k * (nn - k);
            }
            if (saturated) break;
            const std::vector<long long> yw(lv.y_off.begin() + id0, lv.y_off.begin() + id0 + cnt);
            upload(lv.d_y_off + id0, yw, st);
            upload(sc.toff, toff, st);
            double2* c64 = nullptr;
            float2* c32 = nullptr;
            if (h->keep & MIDBF_KEEP_FP64) {
                c64 = dalloc<double2>(tw);
                lv.chunks.push_back(c64);
                lv.t64.push_back({c64, tw});
            }
            if (h->keep & MIDBF_KEEP_FP32) { c32 = dalloc<float2>(tw); lv.chunks.push_back(c32); }
            PackArgs pa{lv.side, id0, sc.k, lv.d_n + id0, sc.X, sc.xs, sc.perm, nmax, sc.cand, (int)nmax, sc.toff,
                        c64, c32, lv.d_perm_off, lv.d_y_off, lv.d_perm, lv.d_skel};
            hipLaunchKernelGGL(pack_kernel, dim3(cnt), dim3(BT), 0, st, pa);
            MIDBF_HIP(hipGetLastError());
            // per-ID block pointers
            std::vector<void*> p64(cnt), p32(cnt);
            for (int w = 0; w < cnt; ++w) {
                p64[w] = c64 ? (void*)(c64 + toff[w]) : nullptr;
                p32[w] = c32 ? (void*)(c32 + toff[w]) : nullptr;
            }
            if (lv.d_T[PREC_FP64]) upload((void**)lv.d_T[PREC_FP64] + id0, p64, st);
            if (lv.d_T[PREC_FP32]) upload((void**)lv.d_T[PREC_FP32] + id0, p32, st);
            // split 16-bit fragment tiles: column side A = T (k x (n-k)), row side A = T^T
            std::vector<long long> tile_off(cnt);
            std::vector<void*> pbf(cnt);
            if (lv.d_T[PREC_BF16] || lv.d_T[PREC_FP16]) {
                long long tt = 0;
                for (int w = 0; w < cnt; ++w) {
                    const int k = kw[w], nn = lv.n[id0 + w];
                    tile_off[w] = tt;
                    tt += lv.side == SIDE_COL ? bf16_tiles(k, nn - k) : bf16_tiles(nn - k, k);
                }
                lv.bf16_bytes += tt * BF16_TILE_BYTES;
                upload(sc.tile_off, tile_off, st);
                for (int q : {PREC_BF16, PREC_FP16}) {
                    if (!lv.d_T[q]) continue;
                    char* cb = (char*)dalloc<char>((size_t)std::max<long long>(tt, 1) * BF16_TILE_BYTES);
                    lv.chunks.push_back(cb);
                    pack_bf16_slab(q == PREC_FP16 ? SPLIT16_FP16 : SPLIT16_BF16, sc.X, sc.xs, sc.k, lv.d_n + id0, cnt,
                                   lv.side == SIDE_ROW, cb, sc.tile_off, h->d_tmax, st);
                    for (int w = 0; w < cnt; ++w) pbf[w] = cb + tile_off[w] * BF16_TILE_BYTES;
                    upload((void**)lv.d_T[q] + id0, pbf, st);
                    MIDBF_HIP(hipStreamSynchronize(st));      // pbf is reused by the next copy
                }
            }
            MIDBF_HIP(hipStreamSynchronize(st));
        }
    } catch (...) {
        sc.release();
        throw;
    }
    sc.release();
    if (saturated) return false;
    upload(lv.d_k, lv.k, st);
    lv.total_k = yrun;
    lv.kmin = *std::min_element(lv.k.begin(), lv.k.end());
    lv.kmax = *std::max_element(lv.k.begin(), lv.k.end());
    lv.entries = 0;
    for (long long id = 0; id < nid; ++id) lv.entries += (long long)lv.k[id] * (lv.n[id] - lv.k[id]);
    MIDBF_HIP(hipStreamSynchronize(st));
    return true;
}

// The dense split 16-bit blocks of the groups of a row step s >= 1 (plan.h).
// Skipped (groups = 0) where a block exceeds the kernels' row tables.
void build_group_dense(midbf_plan* h, LevelSide& lv, const LevelSide& prev, hipStream_t st) {
    const int P = h->P;
    const long long G = lv.nid / P, Ps = ipow(P, lv.s);
    std::vector<int> nr(G), nc(G), in_len(G * P), out_len(G * P);
    std::vector<long long> toff(G), in_off(G * P), out_off(G * P);
    long long tiles = 0, entries = 0;
    int nr_max = 0, nc_max = 0;
    for (long long g = 0; g < G; ++g) {
        const long long a = g / Ps, ap = g - a * Ps;
        int sk = 0;
        for (int t = 0; t < P; ++t) {
            const long long id = g * P + t, idp = ((long long)P * a + t) * Ps + ap;
            in_off[g * P + t] = lv.y_off[id];
            in_len[g * P + t] = lv.k[id];
            out_off[g * P + t] = prev.y_off[idp];
            out_len[g * P + t] = prev.k[idp];
            sk += lv.k[id];
        }
        nr[g] = lv.n[g * P];
        nc[g] = sk;
        toff[g] = tiles;
        tiles += bf16_tiles(nr[g], nc[g]);
        entries += (long long)nr[g] * nc[g];
        nr_max = std::max(nr_max, nr[g]);
        nc_max = std::max(nc_max, nc[g]);
    }
    if (nr_max > BF16_CROW_MAX || nc_max > BF16_CROW_MAX) return;
    auto own = [&](auto* p) { lv.chunks.push_back((void*)p); return p; };
    lv.d_g_nr = own(dalloc<int>(G));
    lv.d_g_nc = own(dalloc<int>(G));
    lv.d_g_tile_off = own(dalloc<long long>(G));
    lv.d_g_in_off = own(dalloc<long long>(G * P));
    lv.d_g_in_len = own(dalloc<int>(G * P));
    lv.d_g_out_off = own(dalloc<long long>(G * P));
    lv.d_g_out_len = own(dalloc<int>(G * P));
    upload(lv.d_g_nr, nr, st);
    upload(lv.d_g_nc, nc, st);
    upload(lv.d_g_tile_off, toff, st);
    upload(lv.d_g_in_off, in_off, st);
    upload(lv.d_g_in_len, in_len, st);
    upload(lv.d_g_out_off, out_off, st);
    upload(lv.d_g_out_len, out_len, st);
    for (int q : {PREC_BF16, PREC_FP16}) {
        if (!lv.d_T[q]) continue;
        lv.g_T[q] = own(dalloc<char>((size_t)std::max<long long>(tiles, 1) * BF16_TILE_BYTES));
        pack_group_tiles(q == PREC_FP16 ? SPLIT16_FP16 : SPLIT16_BF16, P, lv.d_k, lv.d_perm_off, lv.d_perm,
                         lv.d_T[q], lv.d_g_nr, lv.d_g_nc, lv.d_g_tile_off, G, lv.g_T[q], st);
    }
    MIDBF_HIP(hipStreamSynchronize(st));
    lv.groups = G;
    lv.g_tiles = tiles;
    lv.g_entries = entries;
    lv.g_nr_max = nr_max;
    lv.g_nc_max = nc_max;
}

void build_middle(midbf_plan* h, hipStream_t st) {
    Middle& M = h->mid;
    const int P = h->P;
    const LevelSide& R = h->rows.back();
    const LevelSide& C = h->cols.back();
    const long long nb = ipow(P, h->b);
    const bool odd = (h->L % 2) == 1;
    M.pieces = odd ? 1 : P;
    M.nblk = nb * nb;
    std::vector<int> skR(R.total_k), skC(C.total_k);
    MIDBF_HIP(hipMemcpyAsync(skR.data(), R.d_skel, R.total_k * sizeof(int), hipMemcpyDeviceToHost, st));
    MIDBF_HIP(hipMemcpyAsync(skC.data(), C.d_skel, C.total_k * sizeof(int), hipMemcpyDeviceToHost, st));
    MIDBF_HIP(hipStreamSynchronize(st));
    M.nr.assign(M.nblk, 0);
    M.nc.assign(M.nblk, 0);
    M.off.assign(M.nblk, 0);
    std::vector<long long> in_off(M.nblk * M.pieces), out_off(M.nblk * M.pieces), pts_off(M.nblk);
    std::vector<int> in_len(M.nblk * M.pieces), out_len(M.nblk * M.pieces);
    std::vector<int> pts;
    long long tot = 0;
    const long long Pb = ipow(P, h->b);
    for (long long a = 0; a < nb; ++a) {
        for (long long bb = 0; bb < nb; ++bb) {
            const long long bi = a * nb + bb;
            pts_off[bi] = (long long)pts.size();
            int nr = 0, nc = 0;
            for (int t = 0; t < M.pieces; ++t) {
                const long long rid = odd ? bi : ((long long)P * a + t) * Pb + bb;
                const long long cid = odd ? bb * Pb + a : ((long long)P * bb + t) * Pb + a;
                out_off[bi * M.pieces + t] = R.y_off[rid];
                out_len[bi * M.pieces + t] = R.k[rid];
                in_off[bi * M.pieces + t] = C.y_off[cid];
                in_len[bi * M.pieces + t] = C.k[cid];
                nr += R.k[rid];
                nc += C.k[cid];
            }
            for (int t = 0; t < M.pieces; ++t) {
                const long long rid = odd ? bi : ((long long)P * a + t) * Pb + bb;
                for (int i = 0; i < R.k[rid]; ++i) pts.push_back(skR[R.y_off[rid] + i]);
            }
            for (int t = 0; t < M.pieces; ++t) {
                const long long cid = odd ? bb * Pb + a : ((long long)P * bb + t) * Pb + a;
                for (int i = 0; i < C.k[cid]; ++i) pts.push_back(skC[C.y_off[cid] + i]);
            }
            M.nr[bi] = nr;
            M.nc[bi] = nc;
            M.off[bi] = tot;
            tot += (long long)nr * nc;
        }
    }
    M.total = tot;
    M.nr_max = *std::max_element(M.nr.begin(), M.nr.end());
    M.nc_max = *std::max_element(M.nc.begin(), M.nc.end());
    M.d_nr = dalloc<int>(M.nblk);
    M.d_nc = dalloc<int>(M.nblk);
    M.d_off = dalloc<long long>(M.nblk);
    M.d_in_off = dalloc<long long>(in_off.size());
    M.d_out_off = dalloc<long long>(out_off.size());
    M.d_in_len = dalloc<int>(in_len.size());
    M.d_out_len = dalloc<int>(out_len.size());
    upload(M.d_nr, M.nr, st);
    upload(M.d_nc, M.nc, st);
    upload(M.d_off, M.off, st);
    upload(M.d_in_off, in_off, st);
    upload(M.d_out_off, out_off, st);
    upload(M.d_in_len, in_len, st);
    upload(M.d_out_len, out_len, st);
    int* d_pts = dalloc<int>(pts.size());
    long long* d_pts_off = dalloc<long long>(M.nblk);
    upload(d_pts, pts, st);
    upload(d_pts_off, pts_off, st);
    double2* S64 = nullptr;
    float2* S32 = nullptr;
    if (h->keep & MIDBF_KEEP_FP64) S64 = dalloc<double2>(tot);
    if (h->keep & (MIDBF_KEEP_FP32 | MIDBF_KEEP_BF16 | MIDBF_KEEP_FP16)) S32 = dalloc<float2>(tot);
    M.S[PREC_FP64] = S64;
    M.S[PREC_FP32] = S32;
    MidGenArgs ma{h->ph, M.d_nr, M.d_nc, M.d_off, d_pts_off, d_pts, S64, S32};
    const long long per = (long long)M.nr_max * M.nc_max;
    const int gx = (int)std::max<long long>(1, std::min<long long>((per + BT - 1) / BT, 256));
    for (long long b0 = 0; b0 < M.nblk; b0 += 65535) {
        const long long cnt = std::min<long long>(65535, M.nblk - b0);
        MidGenArgs mb = ma;
        mb.nr += b0; mb.nc += b0; mb.off += b0; mb.pts_off += b0;
        hipLaunchKernelGGL(midgen_kernel, dim3(gx, (unsigned)cnt), dim3(BT), 0, st, mb);
        MIDBF_HIP(hipGetLastError());
    }
    if (h->keep & (MIDBF_KEEP_BF16 | MIDBF_KEEP_FP16)) {
        std::vector<long long> toff(M.nblk);
        long long tt = 0;
        for (long long bi = 0; bi < M.nblk; ++bi) {
            toff[bi] = tt;
            tt += bf16_tiles(M.nr[bi], M.nc[bi]);
        }
        M.d_tile_off = dalloc<long long>(M.nblk);
        upload(M.d_tile_off, toff, st);
        M.bf16_bytes = tt * BF16_TILE_BYTES;
        for (int q : {PREC_BF16, PREC_FP16}) {
            if (!(h->keep & (1u << q))) continue;
            M.S[q] = dalloc<char>((size_t)std::max<long long>(tt, 1) * BF16_TILE_BYTES);
            pack_bf16_blocks(q == PREC_FP16 ? SPLIT16_FP16 : SPLIT16_BF16, S32, M.d_off, M.d_nr, M.d_nc, M.nblk,
                             M.S[q], M.d_tile_off, st);
        }
        // the same blocks as their phases, one copy for both 16-bit types
        M.ang_bytes = tt * ANGLE_TILE_BYTES;
        M.ang = dalloc<char>((size_t)std::max<long long>(tt, 1) * ANGLE_TILE_BYTES);
        pack_angle_tiles(h->ph, M.d_nr, M.d_nc, d_pts_off, d_pts, M.d_tile_off, M.nblk, M.ang, st);
        MIDBF_HIP(hipStreamSynchronize(st));
        if (!(h->keep & MIDBF_KEEP_FP32)) {
            (void)hipFree(S32);          // kept only as the source of the tiles
            M.S[PREC_FP32] = nullptr;
        }
    }
    MIDBF_HIP(hipStreamSynchronize(st));
    (void)hipFree(d_pts);
    (void)hipFree(d_pts_off);
}

}  // namespace

void destroy_plan(midbf_plan* h) {
    if (!h) return;
    for (auto& lv : h->rows) free_level(lv);
    for (auto& lv : h->cols) free_level(lv);
    Middle& M = h->mid;
    auto f = [](void* p) { if (p) (void)hipFree(p); };
    f(M.d_nr); f(M.d_nc); f(M.d_off); f(M.d_in_off); f(M.d_in_len); f(M.d_out_off); f(M.d_out_len);
    f(M.d_tile_off);
    f(M.ang);
    for (int q = 0; q < NPREC; ++q) f(M.S[q]);
    f(h->d_tmax);
    f(h->own_U);
    f(h->own_V);
    f(h->own_xp);
    f(h->own_wp);
    f(h->d_slot[0]);
    f(h->d_slot[1]);
    for (int q = 0; q < NPREC; ++q) {
        f(h->ws[q].buf[0]);
        f(h->ws[q].buf[1]);
        f(h->ws[q].scratch);
        f(h->ws[q].lat);
        f(h->ws[q].aux);
    }
    delete h;
}

namespace {

// ---- factor files --------------------------------------------------------------------------
// Little-endian binary: FileHead; for the low-rank phase U then V (N x r FP64 each); then for
// every step s = 0..b-1, the row side then the column side: int64 nid, int32 m, int32 0,
// int32 n[nid], int32 k[nid], int32 pivot orders (sum n), complex FP64 T blocks in pack_kernel's
// stored order (sum k (n - k)); then the magic again.
constexpr char FILE_MAGIC[8] = {'M', 'I', 'D', 'B', 'F', 'f', '1', '\n'};

struct FileHead {
    char magic[8];
    int32_t d, n, leaf_box, oversample_t, k_cap, phase, r, fixed_rank;
    double tol;
    int32_t L, b;
    int64_t N;
};

struct File {
    FILE* f = nullptr;
    File(const char* path, const char* mode) : f(std::fopen(path, mode)) {
        MIDBF_CHECK(f, MIDBF_ERR_IO, "cannot open the factor file");
    }
    ~File() { if (f) std::fclose(f); }
    void read(void* dst, size_t bytes) {
        MIDBF_CHECK(std::fread(dst, 1, bytes, f) == bytes, MIDBF_ERR_IO, "factor file truncated");
    }
    void write(const void* src, size_t bytes) {
        MIDBF_CHECK(std::fwrite(src, 1, bytes, f) == bytes, MIDBF_ERR_IO, "cannot write the factor file");
    }
    template <class T> void read_vec(std::vector<T>& v, long long count) {
        MIDBF_CHECK(count >= 0 && count < (1LL << 40), MIDBF_ERR_IO, "factor file: bad array size");
        v.resize((size_t)count);
        if (count) read(v.data(), (size_t)count * sizeof(T));
    }
};

// One level record, checked against the geometry before anything reaches the device.
void read_level(File& F, long long nid_expect, ReplayLevel& rl) {
    int64_t nid = 0;
    int32_t mz[2] = {0, 0};
    F.read(&nid, sizeof nid);
    F.read(mz, sizeof mz);
    MIDBF_CHECK(nid == nid_expect, MIDBF_ERR_IO, "factor file: decomposition count does not match its tree");
    rl.m = mz[0];
    MIDBF_CHECK(rl.m >= 1 && rl.m <= ID_MMAX, MIDBF_ERR_IO, "factor file: bad sample count");
    F.read_vec(rl.n, nid);
    F.read_vec(rl.k, nid);
    long long sn = 0, st = 0;
    for (long long i = 0; i < nid; ++i) {
        const int n = rl.n[i], k = rl.k[i];
        MIDBF_CHECK(n >= 1 && n <= ID_NMAX && k >= 0 && k <= n && k <= rl.m, MIDBF_ERR_IO,
                    "factor file: bad rank or candidate count");
        sn += n;
        st += (long long)k * (n - k);
    }
    F.read_vec(rl.perm, sn);
    std::vector<char> seen;
    long long off = 0;
    for (long long i = 0; i < nid; ++i) {
        const int n = rl.n[i];
        seen.assign(n, 0);
        for (int j = 0; j < n; ++j) {
            const int v = rl.perm[off + j];
            MIDBF_CHECK(v >= 0 && v < n && !seen[v], MIDBF_ERR_IO, "factor file: a pivot order is not a permutation");
            seen[v] = 1;
        }
        off += n;
    }
    F.read_vec(rl.T, st);
}

}  // namespace

midbf_plan* build_plan(const midbf_params& p, hipStream_t st, void* replay_file) {
    auto t0 = std::chrono::steady_clock::now();
    File* rf = (File*)replay_file;
    MIDBF_CHECK(p.d == 2 || p.d == 3, MIDBF_ERR_ARG, "d must be 2 or 3");
    MIDBF_CHECK(p.leaf_box >= 1 && p.n >= 2 * p.leaf_box && p.n % p.leaf_box == 0, MIDBF_ERR_SHAPE,
                "n must be a multiple of leaf_box and at least 2*leaf_box");
    int L = 0;
    while ((p.leaf_box << L) < p.n) ++L;
    MIDBF_CHECK((p.leaf_box << L) == p.n, MIDBF_ERR_SHAPE, "n / leaf_box must be a power of two");
    MIDBF_CHECK(p.n % 2 == 0, MIDBF_ERR_SHAPE, "n must be even");
    MIDBF_CHECK(p.tol > 0.0 && p.tol < 1.0, MIDBF_ERR_ARG, "tol must be in (0, 1)");
    MIDBF_CHECK(p.oversample_t >= 1, MIDBF_ERR_ARG, "oversample_t must be >= 1");
    MIDBF_CHECK(p.fixed_rank >= 0, MIDBF_ERR_ARG, "fixed_rank must be >= 0");
    if (p.phase == MIDBF_PHASE_LOWRANK)
        MIDBF_CHECK((rf || (p.U_dev && p.V_dev)) && p.r >= 1, MIDBF_ERR_ARG, "low-rank phase needs U, V and r");
    if (p.phase == MIDBF_PHASE_FIO_ELLIPSE || p.phase == MIDBF_PHASE_FIO_PIECEWISE)
        MIDBF_CHECK(p.d == 2, MIDBF_ERR_ARG, "this phase is two-dimensional");
    if (p.phase == MIDBF_PHASE_ISO3D) MIDBF_CHECK(p.d == 3, MIDBF_ERR_ARG, "this phase is three-dimensional");
    MIDBF_CHECK(p.phase >= MIDBF_PHASE_LINEAR && p.phase <= MIDBF_PHASE_HELMHOLTZ, MIDBF_ERR_ARG, "unknown phase");
    const bool points = p.x_points || p.xi_points;
    MIDBF_CHECK(points || p.phase != MIDBF_PHASE_HELMHOLTZ, MIDBF_ERR_ARG, "the Helmholtz phase is for point sets");
    MIDBF_CHECK(points || p.n_points == 0, MIDBF_ERR_ARG, "n_points is for point sets");
    if (points) {
        MIDBF_CHECK(p.x_points && p.xi_points, MIDBF_ERR_ARG, "scattered points need both x_points and xi_points");
        MIDBF_CHECK(p.phase == MIDBF_PHASE_LINEAR || p.phase == MIDBF_PHASE_LOWRANK ||
                        p.phase == MIDBF_PHASE_HELMHOLTZ,
                    MIDBF_ERR_ARG, "scattered points take the linear, Helmholtz or low-rank phase");
        MIDBF_CHECK(p.n_points >= 0, MIDBF_ERR_ARG, "n_points must be >= 0");
        MIDBF_CHECK(!rf, MIDBF_ERR_UNIMPLEMENTED, "factor files hold lattice factorizations");
        MIDBF_CHECK(!(p.precisions & (MIDBF_KEEP_BF16 | MIDBF_KEEP_FP16)), MIDBF_ERR_UNIMPLEMENTED,
                    "scattered points keep the FP64 and FP32 copies only");
    }

    midbf_plan* h = new midbf_plan();
    try {
        h->p = p;
        if (h->p.build_workspace_bytes == 0) h->p.build_workspace_bytes = (size_t)48 << 30;
        h->keep = p.precisions ? p.precisions
                               : (MIDBF_KEEP_FP64 | MIDBF_KEEP_FP32 | (points ? 0u : (unsigned)MIDBF_KEEP_BF16));
        MIDBF_CHECK((h->keep & ~(MIDBF_KEEP_FP64 | MIDBF_KEEP_FP32 | MIDBF_KEEP_BF16 | MIDBF_KEEP_FP16)) == 0,
                    MIDBF_ERR_ARG, "unknown precision bits");
        h->d = p.d; h->n = p.n; h->P = 1 << p.d; h->L = L; h->leaf = p.leaf_box;
        h->n0 = (int)ipow(p.leaf_box, p.d);
        h->N = points && p.n_points > 0 ? p.n_points : ipow(p.n, p.d);
        h->b = (L + 1) / 2;
        h->hstar = L - h->b + 1;
        if (p.phase == MIDBF_PHASE_LOWRANK) {
            // the plan keeps its own U and V: a factor file carries them, and the caller may free theirs
            const size_t cnt = (size_t)h->N * p.r;
            h->own_U = dalloc<double>(cnt);
            h->own_V = dalloc<double>(cnt);
            if (rf) {
                std::vector<double> hv;
                rf->read_vec(hv, (long long)cnt);
                MIDBF_HIP(hipMemcpy(h->own_U, hv.data(), cnt * sizeof(double), hipMemcpyHostToDevice));
                rf->read_vec(hv, (long long)cnt);
                MIDBF_HIP(hipMemcpy(h->own_V, hv.data(), cnt * sizeof(double), hipMemcpyHostToDevice));
            } else {
                MIDBF_HIP(hipMemcpyAsync(h->own_U, p.U_dev, cnt * sizeof(double), hipMemcpyDeviceToDevice, st));
                MIDBF_HIP(hipMemcpyAsync(h->own_V, p.V_dev, cnt * sizeof(double), hipMemcpyDeviceToDevice, st));
            }
            h->p.U_dev = h->own_U;
            h->p.V_dev = h->own_V;
        }
        if (points) {
            // own copies of the coordinates, host copies for the trees (xi mapped to [0, 1)^d), and
            // per side the leaf slot tables, n0 slots per leaf (the fullest leaf of either tree).
            // The row tree holds the x points, or for K^H the xi points.
            h->points = true;
            const bool adj = p.adjoint != 0;
            const size_t cnt = (size_t)h->N * p.d;
            h->own_xp = dalloc<double>(cnt);
            h->own_wp = dalloc<double>(cnt);
            MIDBF_HIP(hipMemcpyAsync(h->own_xp, p.x_points, cnt * sizeof(double), hipMemcpyDeviceToDevice, st));
            MIDBF_HIP(hipMemcpyAsync(h->own_wp, p.xi_points, cnt * sizeof(double), hipMemcpyDeviceToDevice, st));
            MIDBF_HIP(hipStreamSynchronize(st));
            h->tree_pts[0].resize(cnt);
            h->tree_pts[1].resize(cnt);
            MIDBF_HIP(hipMemcpy(h->tree_pts[adj ? 1 : 0].data(), h->own_xp, cnt * sizeof(double),
                                hipMemcpyDeviceToHost));
            MIDBF_HIP(hipMemcpy(h->tree_pts[adj ? 0 : 1].data(), h->own_wp, cnt * sizeof(double),
                                hipMemcpyDeviceToHost));
            // each set moved and scaled uniformly into [0, 1]^d by its bounding cube
            for (int t = 0; t < 2; ++t) {
                std::vector<double>& v = h->tree_pts[t];
                double lo[3], ext = 0.0;
                for (int k = 0; k < p.d; ++k) {
                    double mn = v[k], mx = v[k];
                    for (long long i = 0; i < h->N; ++i) {
                        mn = std::min(mn, v[i * p.d + k]);
                        mx = std::max(mx, v[i * p.d + k]);
                    }
                    lo[k] = mn;
                    ext = std::max(ext, mx - mn);
                }
                const double sc = ext > 0.0 ? ext : 1.0;
                for (long long i = 0; i < h->N; ++i)
                    for (int k = 0; k < p.d; ++k) v[i * p.d + k] = (v[i * p.d + k] - lo[k]) / sc;
            }
            int n0 = 1;
            const long long nleaf = ipow(h->P, L);
            for (int t = 0; t < 2; ++t) {
                point_tree(h->tree_pts[t], p.d, L, h->tree_order[t], h->tree_start[t]);
                for (long long l = 0; l < nleaf; ++l)
                    n0 = std::max<int>(n0, (int)(h->tree_start[t][l + 1] - h->tree_start[t][l]));
            }
            MIDBF_CHECK(n0 <= ID_NMAX, MIDBF_ERR_SHAPE, "a leaf holds more points than a decomposition takes");
            h->n0 = n0;
            for (int t = 0; t < 2; ++t) {
                std::vector<int> slot((size_t)nleaf * n0, -1);
                for (long long l = 0; l < nleaf; ++l)
                    for (long long c = h->tree_start[t][l]; c < h->tree_start[t][l + 1]; ++c)
                        slot[l * n0 + (c - h->tree_start[t][l])] = h->tree_order[t][c];
                h->d_slot[t] = dalloc<int>(slot.size());
                upload(h->d_slot[t], slot, st);
                MIDBF_HIP(hipStreamSynchronize(st));
            }
            h->p.x_points = h->own_xp;
            h->p.xi_points = h->own_wp;
        }
        h->ph = PhaseDesc{(int)p.phase, p.d, p.n, h->p.U_dev, h->p.V_dev, p.r, h->own_xp, h->own_wp, p.helmholtz_h,
                          p.adjoint != 0};
        h->rows.resize(h->b);
        h->cols.resize(h->b);
        if (h->keep & (MIDBF_KEEP_BF16 | MIDBF_KEEP_FP16)) {
            h->d_tmax = dalloc<unsigned>(1);
            MIDBF_HIP(hipMemsetAsync(h->d_tmax, 0, sizeof(unsigned), st));
        }
        long long khat[2] = {ipow(p.leaf_box, p.d), ipow(p.leaf_box, p.d)};
        for (int s = 0; s < h->b; ++s) {
            for (int side = 0; side < 2; ++side) {
                LevelSide& lv = side == SIDE_ROW ? h->rows[s] : h->cols[s];
                const LevelSide* prev = s == 0 ? nullptr : (side == SIDE_ROW ? &h->rows[s - 1] : &h->cols[s - 1]);
                long long want = (long long)p.oversample_t * khat[side];
                if (rf) {
                    ReplayLevel rl;
                    read_level(*rf, ipow(h->P, L + 1), rl);
                    lv = LevelSide();
                    lv.s = s; lv.side = side; lv.la = L - s; lv.lb = s + 1;
                    lv.nid = ipow(h->P, L + 1);
                    build_level(h, lv, prev, want, st, &rl);
                }
                for (int attempt = 0; !rf; ++attempt) {
                    lv = LevelSide();
                    lv.s = s; lv.side = side; lv.la = L - s; lv.lb = s + 1;
                    lv.nid = ipow(h->P, L + 1);
                    if (build_level(h, lv, prev, want, st)) break;
                    free_level(lv);
                    MIDBF_CHECK(attempt < 4, MIDBF_ERR_RANK_SATURATED, "rank saturated the samples");
                    want *= 2;    // the sample set was too small: enlarge it (Sec. 3.2)
                }
                khat[side] = lv.kmax;
                if (side == SIDE_ROW && s > 0 && (h->keep & (MIDBF_KEEP_BF16 | MIDBF_KEEP_FP16)))
                    build_group_dense(h, lv, *prev, st);
                if (side == SIDE_COL && (h->keep & (MIDBF_KEEP_BF16 | MIDBF_KEEP_FP16)) &&
                    (s == 0 ? h->n0 : lv.nmax) <= BF16_CROW_MAX) {
                    // input row of every candidate position, for the split up kernels
                    lv.d_src = dalloc<int>(std::max<long long>(lv.total_n, 1));
                    lv.chunks.push_back(lv.d_src);
                    const ApplyGeom G{h->d, h->n, h->P, h->L, h->leaf, h->n0};
                    pack_src_rows(G, s, ipow(h->P, s), lv.d_n, lv.d_perm_off, lv.d_perm, prev ? prev->d_k : nullptr,
                                  prev ? prev->d_y_off : nullptr, lv.nid, lv.d_src, st);
                    if (s == 1 && prev->entries == 0) {
                        lv.d_src_lat = dalloc<int>(std::max<long long>(lv.total_n, 1));
                        lv.chunks.push_back(lv.d_src_lat);
                        pack_src_lattice(prev->d_skel, lv.d_src, lv.total_n, lv.d_src_lat, st);
                    }
                    MIDBF_HIP(hipStreamSynchronize(st));
                }
            }
        }
        build_middle(h, st);
        // statistics
        midbf_stats& S = h->stats;
        S.L = h->L; S.b = h->b; S.hstar = h->hstar;
        S.k_min = 1 << 30; S.k_max = 0;
        long long ent = h->mid.total, idx = 0;
        for (auto* side : {&h->rows, &h->cols})
            for (auto& lv : *side) {
                S.ids += lv.nid;
                ent += lv.entries;
                idx += lv.total_n * 4 + lv.nid * (4 * 2 + 8 * 3);
                S.k_min = std::min(S.k_min, lv.kmin);
                S.k_max = std::max(S.k_max, lv.kmax);
                h->max_total_k = std::max(h->max_total_k, lv.total_k);
                h->max_total_n = std::max(h->max_total_n, lv.total_n);
                h->max_n = std::max(h->max_n, lv.nmax);
                h->max_k = std::max(h->max_k, lv.kmax);
            }
        S.entries = ent;
        S.bytes_fp64 = (h->keep & MIDBF_KEEP_FP64) ? ent * 16 : 0;
        S.bytes_fp32 = (h->keep & MIDBF_KEEP_FP32) ? ent * 8 : 0;
        long long bfb = h->mid.bf16_bytes;
        for (auto* side : {&h->rows, &h->cols})
            for (auto& lv : *side) bfb += lv.bf16_bytes + lv.g_tiles * BF16_TILE_BYTES;
        S.bytes_bf16 = (h->keep & MIDBF_KEEP_BF16) ? bfb : 0;
        S.bytes_fp16 = (h->keep & MIDBF_KEEP_FP16) ? bfb : 0;
        S.index_bytes = idx;
        if (h->d_tmax) {
            unsigned bits = 0;
            MIDBF_HIP(hipMemcpyAsync(&bits, h->d_tmax, sizeof(unsigned), hipMemcpyDeviceToHost, st));
            MIDBF_HIP(hipStreamSynchronize(st));
            float t;
            std::memcpy(&t, &bits, sizeof t);
            S.t_abs_max = t;
            // fp16 holds |x| < 65504; the factor tiles are not rescaled, so their
            // entries must fit as they are (with a margin for the lo parts)
            MIDBF_CHECK(!(h->keep & MIDBF_KEEP_FP16) || t < 32768.f, MIDBF_ERR_UNIMPLEMENTED,
                        "interpolation coefficients beyond the fp16 range: keep the split-bf16 copy instead");
        }
        S.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    } catch (...) {
        destroy_plan(h);
        throw;
    }
    return h;
}

void save_plan(midbf_plan* h, const char* path, hipStream_t st) {
    MIDBF_CHECK(path, MIDBF_ERR_ARG, "null path");
    MIDBF_CHECK(h->keep & MIDBF_KEEP_FP64, MIDBF_ERR_ARG, "saving needs the FP64 factor copy (MIDBF_KEEP_FP64)");
    MIDBF_CHECK(!h->points, MIDBF_ERR_UNIMPLEMENTED, "factor files hold lattice factorizations");
    MIDBF_CHECK(!h->p.adjoint, MIDBF_ERR_UNIMPLEMENTED, "factor files hold forward factorizations");
    MIDBF_HIP(hipStreamSynchronize(st));
    File F(path, "wb");
    FileHead H{};
    std::memcpy(H.magic, FILE_MAGIC, sizeof FILE_MAGIC);
    H.d = h->d; H.n = h->n; H.leaf_box = h->leaf; H.oversample_t = h->p.oversample_t; H.k_cap = h->p.k_cap;
    H.phase = h->p.phase; H.r = h->p.phase == MIDBF_PHASE_LOWRANK ? h->p.r : 0; H.fixed_rank = h->p.fixed_rank;
    H.tol = h->p.tol; H.L = h->L; H.b = h->b; H.N = h->N;
    F.write(&H, sizeof H);
    if (h->p.phase == MIDBF_PHASE_LOWRANK) {
        std::vector<double> hv((size_t)h->N * h->p.r);
        for (const double* src : {h->own_U, h->own_V}) {
            MIDBF_HIP(hipMemcpy(hv.data(), src, hv.size() * sizeof(double), hipMemcpyDeviceToHost));
            F.write(hv.data(), hv.size() * sizeof(double));
        }
    }
    std::vector<double2> buf;
    for (int s = 0; s < h->b; ++s)
        for (LevelSide* lv : {&h->rows[s], &h->cols[s]}) {
            const int64_t nid = lv->nid;
            const int32_t mz[2] = {lv->m, 0};
            F.write(&nid, sizeof nid);
            F.write(mz, sizeof mz);
            F.write(lv->n.data(), lv->n.size() * sizeof(int));
            F.write(lv->k.data(), lv->k.size() * sizeof(int));
            std::vector<int> perm((size_t)lv->total_n);
            if (!perm.empty())
                MIDBF_HIP(hipMemcpy(perm.data(), lv->d_perm, perm.size() * sizeof(int), hipMemcpyDeviceToHost));
            F.write(perm.data(), perm.size() * sizeof(int));
            long long want = 0, have = 0;
            for (long long i = 0; i < lv->nid; ++i) want += (long long)lv->k[i] * (lv->n[i] - lv->k[i]);
            for (const auto& c : lv->t64) {
                constexpr long long piece = 1LL << 24;      // 256 MB of complex FP64 at a time
                for (long long o = 0; o < c.second; o += piece) {
                    const long long cnt = std::min(piece, c.second - o);
                    buf.resize((size_t)cnt);
                    MIDBF_HIP(hipMemcpy(buf.data(), c.first + o, cnt * sizeof(double2), hipMemcpyDeviceToHost));
                    F.write(buf.data(), cnt * sizeof(double2));
                }
                have += c.second;
            }
            MIDBF_CHECK(have == want, MIDBF_ERR_IO, "internal: T chunks do not cover the level");
        }
    F.write(FILE_MAGIC, sizeof FILE_MAGIC);
}

midbf_plan* load_plan(const char* path, unsigned precisions, hipStream_t st, midbf_params* params_out) {
    MIDBF_CHECK(path, MIDBF_ERR_ARG, "null path");
    File F(path, "rb");
    FileHead H{};
    F.read(&H, sizeof H);
    MIDBF_CHECK(std::memcmp(H.magic, FILE_MAGIC, sizeof FILE_MAGIC) == 0, MIDBF_ERR_IO, "not a MIDBF factor file");
    midbf_params p{};
    p.d = H.d; p.n = H.n; p.tol = H.tol; p.leaf_box = H.leaf_box; p.oversample_t = H.oversample_t;
    p.k_cap = H.k_cap; p.phase = (midbf_phase_kind)H.phase; p.r = H.r; p.fixed_rank = H.fixed_rank;
    p.precisions = precisions;
    int L = 0;
    while (p.leaf_box >= 1 && (p.leaf_box << L) < p.n && L < 30) ++L;
    MIDBF_CHECK(H.L == L && H.b == (L + 1) / 2 && H.N == ipow(p.n, p.d) && p.d >= 2 && p.d <= 3, MIDBF_ERR_IO,
                "factor file: header does not describe a factorization");
    midbf_plan* h = build_plan(p, st, &F);
    try {
        char tail[sizeof FILE_MAGIC];
        F.read(tail, sizeof tail);
        MIDBF_CHECK(std::memcmp(tail, FILE_MAGIC, sizeof FILE_MAGIC) == 0, MIDBF_ERR_IO, "factor file: bad ending");
    } catch (...) {
        destroy_plan(h);
        throw;
    }
    if (params_out) *params_out = h->p;
    return h;
}

void kernel_entries(const midbf_params& p, const int* rows, int nrows, const int* cols, int ncols, void* out,
                    hipStream_t st) {
    PhaseDesc ph{(int)p.phase, p.d, p.n, p.U_dev, p.V_dev, p.r, p.x_points, p.xi_points, p.helmholtz_h,
                 p.adjoint != 0};
    const long long tot = (long long)nrows * ncols;
    if (tot == 0) return;
    const int gx = (int)std::min<long long>((tot + BT - 1) / BT, 4096);
    hipLaunchKernelGGL(entries_kernel, dim3(gx), dim3(BT), 0, st, ph, rows, nrows, cols, ncols, (double2*)out);
    MIDBF_HIP(hipGetLastError());
}

void id_batch(void* X, int batch, int m, int n, double tol, int kcap, int* k_out, int* perm_out, void* T_out,
              hipStream_t st) {
    MIDBF_CHECK(batch >= 0 && m >= 1 && n >= 1, MIDBF_ERR_ARG, "bad batch sizes");
    MIDBF_CHECK(m <= ID_MMAX && n <= ID_NMAX, MIDBF_ERR_SHAPE, "m or n too large");
    if (batch == 0) return;
    double2* V = dalloc<double2>((size_t)batch * m * ID_NB);
    double2* Y = dalloc<double2>((size_t)batch * ID_ELL * n);
    try {
        IdBatch ib{(double2*)X, (long long)m * n, V, (long long)m * ID_NB, Y, (long long)ID_ELL * n, perm_out, n,
                   k_out, nullptr, n, m, tol, kcap, 0x5eedu};
        launch_id_batch(ib, batch, st);
        hipLaunchKernelGGL(copy_T_kernel, dim3(batch), dim3(BT), 0, st, (const double2*)X, (long long)m * n, k_out, m,
                           n, (double2*)T_out);
        MIDBF_HIP(hipGetLastError());
        MIDBF_HIP(hipStreamSynchronize(st));
    } catch (...) {
        (void)hipFree(V);
        (void)hipFree(Y);
        throw;
    }
    (void)hipFree(V);
    (void)hipFree(Y);
}

}  // namespace midbf
