// Apply of the MIDBF factor product g = U^L...U^h S V^h...V^L f and of its
// adjoint (Sec. 3.3-3.5), level by level, FP64 or FP32 with accumulation in
// the same precision.
//
// Vectors between levels: the level buffer of step s holds, for each
// decomposition id (in id order), k_id rows of nrhs values; row-major
// (right-hand side fastest), starting at row y_off[id].
//
// Workgroup = the 2^d decompositions that share one candidate vector:
//   going up (V side), (B, A_t) for the children A_t of one row node share
//   the concatenation of y[child(B), parent(A_t)];
//   going down (U side), (A, B_t) for the children B_t of one column node
//   share the candidate set of A, and their outputs are summed into it.
// The 2^d-way butterfly permutations are index math on the Z-order numbers,
// so each workgroup gathers its inputs and scatters its outputs directly and
// no atomics are needed.
#include <algorithm>

#include "apply.h"

namespace midbf {

namespace {

constexpr int AT = 256;   // threads per workgroup
constexpr int AW = AT / 64;

template <class C> __device__ inline C czero() { return cplx_traits<C>::zero(); }

// Factor blocks are read through pointers loaded from tables; marking them
// global lets the compiler issue global (not flat) loads and batch them.
#if defined(__HIP_DEVICE_COMPILE__)
template <class C> using gconst = __attribute__((address_space(1))) const C;
#else
template <class C> using gconst = const C;      // host pass: never executed
#endif
template <class C> __device__ __forceinline__ const gconst<C>* gptr(const C* p) { return (const gconst<C>*)p; }

// loads per batch: 8 complex FP32 or 4 complex FP64 values per lane
template <class C> constexpr int load_batch() { return sizeof(C) == 8 ? 8 : 4; }
__device__ inline double2 ld_c(const double2* p) { return *p; }
__device__ inline float2 ld_c(const float2* p) { return *p; }

__device__ inline double2 sub2(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline float2 sub2(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

template <class C> __device__ inline C wave_sum_c(C v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v.x += __shfl_xor(v.x, o, 64);
        v.y += __shfl_xor(v.y, o, 64);
    }
    return v;
}

// Point number of slot c of leaf a: the lattice point of the box, or with a
// slot table (scattered points) the table's entry (-1 past the leaf's points).
__device__ inline long long leaf_slot_point(const ApplyGeom& G, const int* slot, const int* origin, long long a,
                                            int c) {
    return slot ? (long long)slot[a * G.n0 + c] : box_point(origin, G.leaf, c, G.d, G.n);
}

// Gather the candidate vector of group (a, partner) into LDS: either the
// leaf's points from an external column-major block or the P child pieces
// of the previous level buffer.
template <class C, int RT>
__device__ int gather_candidates(C* s_x, const ApplyGeom& G, int s, long long a, long long partner, long long Ps,
                                 const C* ext, long long ld, const C* prev_buf, const int* k_prev,
                                 const long long* yoff_prev, int nrhs, int r0, int nr, const int* slot) {
    const int tid = threadIdx.x;
    if (s == 0) {
        int origin[3];
        node_origin(a, G.L, G.d, G.n, origin);
        for (int e = tid; e < G.n0 * RT; e += AT) {
            const int c = e / RT, r = e - c * RT;
            C v = czero<C>();
            const long long p = leaf_slot_point(G, slot, origin, a, c);
            if (r < nr && p >= 0) v = ext[(long long)(r0 + r) * ld + p];
            s_x[e] = v;
        }
        return G.n0;
    }
    int len[MAX_P];
    long long off[MAX_P];
    child_pieces(len, off, G.P, a, partner, Ps, k_prev, yoff_prev);
    int start = 0;
#pragma unroll
    for (int t = 0; t < MAX_P; ++t) {
        if (t < G.P) {
            for (int e = tid; e < len[t] * RT; e += AT) {
                const int c = e / RT, r = e - c * RT;
                s_x[(start + c) * RT + r] = (r < nr) ? prev_buf[(off[t] + c) * nrhs + r0 + r] : czero<C>();
            }
            start += len[t];
        }
    }
    return start;
}

// Scatter a candidate vector (LDS) of group (a, partner) back to the leaf's
// points of an external block or to the P child pieces of the previous level.
template <class C, int RT>
__device__ void scatter_candidates(const C* s_w, const ApplyGeom& G, int s, long long a, long long partner,
                                   long long Ps, C* ext, long long ld, C* prev_buf, const int* k_prev,
                                   const long long* yoff_prev, int nrhs, int r0, int nr, const int* slot) {
    const int tid = threadIdx.x;
    if (s == 0) {
        int origin[3];
        node_origin(a, G.L, G.d, G.n, origin);
        for (int e = tid; e < G.n0 * RT; e += AT) {
            const int c = e / RT, r = e - c * RT;
            const long long p = leaf_slot_point(G, slot, origin, a, c);
            if (r < nr && p >= 0) ext[(long long)(r0 + r) * ld + p] = s_w[e];
        }
        return;
    }
    int len[MAX_P];
    long long off[MAX_P];
    child_pieces(len, off, G.P, a, partner, Ps, k_prev, yoff_prev);
    int start = 0;
#pragma unroll
    for (int t = 0; t < MAX_P; ++t) {
        if (t < G.P) {
            for (int e = tid; e < len[t] * RT; e += AT) {
                const int c = e / RT, r = e - c * RT;
                if (r < nr) prev_buf[(off[t] + c) * nrhs + r0 + r] = s_w[(start + c) * RT + r];
            }
            start += len[t];
        }
    }
}

// ---- forward, going up: y[id] = x[skel] + T x[red]  (T column-major k x (n-k)) ----
// Wave t handles decomposition t of the group: its redundant inputs are first
// gathered into a per-wave LDS strip (x[red] in order), then each lane owns
// OPL outputs (o = lane + 64u) and sweeps the columns of T once; every column
// read is OPL coalesced 64-lane loads.
// Single right-hand side: rows o = o0 + lane + 64u (u < U) of T x_red,
// accumulated over the columns in order; each batch of JB columns is loaded
// before it is used, so JB * U loads per lane are in flight.
template <class C, int U>
__device__ __forceinline__ void up_rows1(C (&acc)[4], const C* __restrict__ T, int k, int nred, const C* strip,
                                         int o0, int lane) {
    constexpr int JB = load_batch<C>();
    const gconst<C>* Tg = gptr(T);
    int orow[U];
#pragma unroll
    for (int u = 0; u < U; ++u) orow[u] = min(o0 + lane + 64 * u, k - 1);     // clamped: no divergence
    int j = 0;
    for (; j + JB <= nred; j += JB) {
        C tv[JB][U];
#pragma unroll
        for (int q = 0; q < JB; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) tv[q][u] = Tg[(long long)(j + q) * k + orow[u]];
#pragma unroll
        for (int q = 0; q < JB; ++q) {
            const C xv = strip[j + q];
#pragma unroll
            for (int u = 0; u < U; ++u) cfma(acc[u], tv[q][u], xv);
        }
    }
    for (; j < nred; ++j) {
        const C xv = strip[j];
#pragma unroll
        for (int u = 0; u < U; ++u) cfma(acc[u], Tg[(long long)j * k + orow[u]], xv);
    }
}

template <class C, int RT, int OPL>
__device__ __forceinline__ void up_body(const UpArgs& A, long long g, int tile, unsigned char* smem_raw) {
    C* s_x = reinterpret_cast<C*>(smem_raw);
    const int r0 = tile * RT;
    const int nr = min(RT, A.nrhs - r0);
    const long long a = g / A.Ps, ap = g - (g / A.Ps) * A.Ps;
    const int ncand = gather_candidates<C, RT>(s_x, A.G, A.s, a, ap, A.Ps, (const C*)A.ext, A.ld, (const C*)A.in,
                                               A.k_prev, A.yoff_prev, A.nrhs, r0, nr, A.lev.slot);
    C* s_red = s_x + (size_t)A.ncand_max * RT;     // single RHS: AW strips of ncand_max values
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    C* out = (C*)A.out;
    C* strip = s_red + (size_t)wave * A.ncand_max;
    for (int t = wave; t < A.G.P; t += AW) {
        const long long id = g * A.G.P + t;
        const int k = A.lev.k[id], nred = A.lev.n[id] - k;
        const int* perm = A.lev.perm + A.lev.perm_off[id];
        const C* T = (const C*)A.lev.T[id];
        const long long yo = A.lev.y_off[id];
        if constexpr (RT == 1) {
            for (int j = lane; j < nred; j += 64) strip[j] = s_x[perm[k + j]];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        for (int o0 = 0; o0 < k; o0 += 64 * OPL) {
            C acc[OPL][RT];
#pragma unroll
            for (int u = 0; u < OPL; ++u)
#pragma unroll
                for (int r = 0; r < RT; ++r) acc[u][r] = czero<C>();
            int o[OPL];
#pragma unroll
            for (int u = 0; u < OPL; ++u) o[u] = o0 + lane + 64 * u;
            const int uact = min(OPL, (k - o0 + 63) / 64);     // wave-uniform
            if constexpr (RT == 1) {
                static_assert(OPL == 4, "single-RHS path keeps four rows per lane");
                C acc1[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) acc1[u] = czero<C>();
                switch (uact) {
                    case 1: up_rows1<C, 1>(acc1, T, k, nred, strip, o0, lane); break;
                    case 2: up_rows1<C, 2>(acc1, T, k, nred, strip, o0, lane); break;
                    case 3: up_rows1<C, 3>(acc1, T, k, nred, strip, o0, lane); break;
                    default: up_rows1<C, 4>(acc1, T, k, nred, strip, o0, lane); break;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[u][0] = acc1[u];
            } else {
#pragma unroll 4
                for (int j = 0; j < nred; ++j) {
                    C xv[RT];
                    const int pj = perm[k + j];
#pragma unroll
                    for (int r = 0; r < RT; ++r) xv[r] = s_x[pj * RT + r];
                    const C* Tj = T + (long long)j * k;
#pragma unroll
                    for (int u = 0; u < OPL; ++u) {
                        if (u < uact) {                               // wave-uniform
                            const C tv = Tj[min(o[u], k - 1)];
#pragma unroll
                            for (int r = 0; r < RT; ++r) cfma(acc[u][r], tv, xv[r]);
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < OPL; ++u) {
                if (o[u] < k) {
                    const int ps = perm[o[u]];
#pragma unroll
                    for (int r = 0; r < RT; ++r)
                        if (r < nr) out[(yo + o[u]) * A.nrhs + r0 + r] = cadd(acc[u][r], s_x[ps * RT + r]);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

template <class C, int RT, int OPL>
__global__ __launch_bounds__(AT) void up_kernel(UpArgs A) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    up_body<C, RT, OPL>(A, blockIdx.x, blockIdx.y, smem_raw);
}

// ---- forward, going down: w(cand) = sum_t Pi_t [z_t ; T_t^T z_t]  (T row-major k x (n-k)) ----
template <class C, int RT>
__device__ __forceinline__ void down_body(const DownArgs& A, long long g, int tile, unsigned char* smem_raw) {
    const int r0 = tile * RT;
    const int nr = min(RT, A.nrhs - r0);
    const long long a = g / A.Ps, bp = g - (g / A.Ps) * A.Ps;
    const int ncand = A.lev.n[g * A.G.P];
    C* s_w = reinterpret_cast<C*>(smem_raw);
    C* s_z = s_w + (size_t)A.ncand_max * RT;
    const int tid = threadIdx.x;
    for (int e = tid; e < ncand * RT; e += AT) s_w[e] = czero<C>();
    const C* zin = (const C*)A.in;
    for (int t = 0; t < A.G.P; ++t) {
        const long long id = g * A.G.P + t;
        const int k = A.lev.k[id], nred = A.lev.n[id] - k;
        const int* perm = A.lev.perm + A.lev.perm_off[id];
        const C* T = (const C*)A.lev.T[id];
        const long long yo = A.lev.y_off[id];
        __syncthreads();
        for (int e = tid; e < k * RT; e += AT) {
            const int i = e / RT, r = e - i * RT;
            s_z[e] = (r < nr) ? zin[(yo + i) * A.nrhs + r0 + r] : czero<C>();
        }
        __syncthreads();
        for (int e = tid; e < k * RT; e += AT) {
            const int i = e / RT, r = e - i * RT;
            const int ps = perm[i];
            s_w[ps * RT + r] = cadd(s_w[ps * RT + r], s_z[e]);
        }
        const gconst<C>* Tg = gptr(T);
        constexpr int IB = load_batch<C>();
        for (int j = tid; j < nred; j += AT) {
            C acc[RT];
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = czero<C>();
            int i = 0;
            for (; i + IB <= k; i += IB) {
                C tv[IB];
#pragma unroll
                for (int q = 0; q < IB; ++q) tv[q] = Tg[(long long)(i + q) * nred + j];
#pragma unroll
                for (int q = 0; q < IB; ++q)
#pragma unroll
                    for (int r = 0; r < RT; ++r) cfma(acc[r], tv[q], s_z[(i + q) * RT + r]);
            }
            for (; i < k; ++i) {
                const C tv = Tg[(long long)i * nred + j];
#pragma unroll
                for (int r = 0; r < RT; ++r) cfma(acc[r], tv, s_z[i * RT + r]);
            }
            const int pr = perm[k + j];
#pragma unroll
            for (int r = 0; r < RT; ++r) s_w[pr * RT + r] = cadd(s_w[pr * RT + r], acc[r]);
        }
    }
    __syncthreads();
    scatter_candidates<C, RT>(s_w, A.G, A.s, a, bp, A.Ps, (C*)A.ext, A.ld, (C*)A.out, A.k_prev, A.yoff_prev,
                              A.nrhs, r0, nr, A.lev.slot);
}

template <class C, int RT>
__global__ __launch_bounds__(AT) void down_kernel(DownArgs A) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    down_body<C, RT>(A, blockIdx.x, blockIdx.y, smem_raw);
}

// ---- middle: z(rows) = S x(cols), S column-major nr x nc ----
// Entries [c0, c0 + cw) of the concatenation of a block's vector pieces
// (offsets off[t], lengths len[t]) into LDS, RT right-hand sides each.
template <class C, int RT>
__device__ void stage_pieces(C* s, const C* src, const long long* off, const int* len, int pieces, int c0, int cw,
                             int nrhs, int r0, int nrr) {
    int start = 0;
    for (int t = 0; t < pieces; ++t) {
        const int l = len[t];
        const int lo = max(c0, start), hi = min(c0 + cw, start + l);
        for (int e = threadIdx.x; e < (hi - lo) * RT; e += AT) {
            const int c = lo + e / RT, r = e - (e / RT) * RT;
            s[(c - c0) * RT + r] = (r < nrr) ? src[(off[t] + (c - start)) * nrhs + r0 + r] : czero<C>();
        }
        start += l;
    }
}

// position of entry `row` of the concatenated pieces
__device__ inline long long piece_offset(const long long* off, const int* len, int pieces, int row) {
    int t = 0, base = 0;
    while (t + 1 < pieces && row >= base + len[t]) {
        base += len[t];
        ++t;
    }
    return off[t] + (row - base);
}

// acc += S(row, c0 + c) x_c for c < cw (x staged in LDS from entry c0), in
// order, with batches of loads issued before use.
template <class C, int RT>
__device__ __forceinline__ void middle_cols(C (&acc)[RT], const gconst<C>* Sg, int nr, int row, int c0, int cw,
                                            const C* s_x) {
    constexpr int CB = load_batch<C>();
    int c = 0;
    for (; c + CB <= cw; c += CB) {
        C sv[CB];
#pragma unroll
        for (int q = 0; q < CB; ++q) sv[q] = Sg[(long long)(c0 + c + q) * nr + row];
#pragma unroll
        for (int q = 0; q < CB; ++q)
#pragma unroll
            for (int r = 0; r < RT; ++r) cfma(acc[r], sv[q], s_x[(c + q) * RT + r]);
    }
    for (; c < cw; ++c) {
        const C sv = Sg[(long long)(c0 + c) * nr + row];
#pragma unroll
        for (int r = 0; r < RT; ++r) cfma(acc[r], sv, s_x[c * RT + r]);
    }
}

template <class C, int RT>
__device__ __forceinline__ void middle_body(const MidArgs& A, long long bi, int tile, unsigned char* smem_raw) {
    C* s_x = reinterpret_cast<C*>(smem_raw);
    const int r0 = tile * RT;
    const int nrr = min(RT, A.nrhs - r0);
    const int nr = A.nr[bi], nc = A.nc[bi];
    const int tid = threadIdx.x;
    const C* xin = (const C*)A.in;
    C* zout = (C*)A.out;
    const long long* in_off = A.in_off + bi * A.pieces;
    const int* in_len = A.in_len + bi * A.pieces;
    const long long* out_off = A.out_off + bi * A.pieces;
    const int* out_len = A.out_len + bi * A.pieces;
    const gconst<C>* Sg = gptr((const C*)A.S + A.off[bi]);
    if (nc <= A.chunk) {
        // the whole input vector fits in LDS: stage it once
        stage_pieces<C, RT>(s_x, xin, in_off, in_len, A.pieces, 0, nc, A.nrhs, r0, nrr);
        __syncthreads();
        for (int row = tid; row < nr; row += AT) {
            C acc[RT];
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = czero<C>();
            middle_cols<C, RT>(acc, Sg, nr, row, 0, nc, s_x);
            const long long off = piece_offset(out_off, out_len, A.pieces, row);
#pragma unroll
            for (int r = 0; r < RT; ++r)
                if (r < nrr) zout[off * A.nrhs + r0 + r] = acc[r];
        }
        return;
    }
    // larger blocks: per batch of rows, the input in chunks of A.chunk entries
    for (int row0 = 0; row0 < nr; row0 += AT) {
        const int row = row0 + tid;
        C acc[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[r] = czero<C>();
        for (int c0 = 0; c0 < nc; c0 += A.chunk) {
            const int cw = min(A.chunk, nc - c0);
            __syncthreads();
            stage_pieces<C, RT>(s_x, xin, in_off, in_len, A.pieces, c0, cw, A.nrhs, r0, nrr);
            __syncthreads();
            if (row < nr) middle_cols<C, RT>(acc, Sg, nr, row, c0, cw, s_x);
        }
        if (row < nr) {
            const long long off = piece_offset(out_off, out_len, A.pieces, row);
#pragma unroll
            for (int r = 0; r < RT; ++r)
                if (r < nrr) zout[off * A.nrhs + r0 + r] = acc[r];
        }
    }
}

template <class C, int RT>
__global__ __launch_bounds__(AT) void middle_kernel(MidArgs A) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    middle_body<C, RT>(A, blockIdx.x, blockIdx.y, smem_raw);
}

// ---- adjoint going up (row side): out_i = x[skel_i] + sum_j conj(T_ij) x[red_j], T row-major ----
template <class C, int RT>
__global__ __launch_bounds__(AT) void adj_up_kernel(UpArgs A) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* s_x = reinterpret_cast<C*>(smem_raw);
    const long long g = blockIdx.x;
    const int r0 = blockIdx.y * RT;
    const int nr = min(RT, A.nrhs - r0);
    const long long a = g / A.Ps, bp = g - (g / A.Ps) * A.Ps;
    gather_candidates<C, RT>(s_x, A.G, A.s, a, bp, A.Ps, (const C*)A.ext, A.ld, (const C*)A.in, A.k_prev,
                             A.yoff_prev, A.nrhs, r0, nr, A.lev.slot);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    C* out = (C*)A.out;
    for (int t = 0; t < A.G.P; ++t) {
        const long long id = g * A.G.P + t;
        const int k = A.lev.k[id], nred = A.lev.n[id] - k;
        const int* perm = A.lev.perm + A.lev.perm_off[id];
        const C* T = (const C*)A.lev.T[id];
        const long long yo = A.lev.y_off[id];
        for (int i = wave; i < k; i += AW) {
            C acc[RT];
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = czero<C>();
            const C* Ti = T + (long long)i * nred;
            for (int j = lane; j < nred; j += 64) {
                const C tv = Ti[j];
                const int pj = perm[k + j];
#pragma unroll
                for (int r = 0; r < RT; ++r) cfmac(acc[r], tv, s_x[pj * RT + r]);
            }
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = wave_sum_c(acc[r]);
            if (lane == 0) {
                const int ps = perm[i];
#pragma unroll
                for (int r = 0; r < RT; ++r)
                    if (r < nr) out[(yo + i) * A.nrhs + r0 + r] = cadd(acc[r], s_x[ps * RT + r]);
            }
        }
    }
}

// ---- adjoint middle: x(cols) = S^H z(rows) ----
// The rows of z are staged in LDS in chunks of A.chunk entries; the
// workgroup owns its block's outputs and adds each chunk's part to them.
template <class C, int RT>
__global__ __launch_bounds__(AT) void adj_middle_kernel(MidArgs A) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* s_z = reinterpret_cast<C*>(smem_raw);
    const long long bi = blockIdx.x;
    const int r0 = blockIdx.y * RT;
    const int nrr = min(RT, A.nrhs - r0);
    const int nr = A.nr[bi], nc = A.nc[bi];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const C* zin = (const C*)A.in;
    C* xout = (C*)A.out;
    const long long* in_off = A.in_off + bi * A.pieces;
    const int* in_len = A.in_len + bi * A.pieces;
    const C* S = (const C*)A.S + A.off[bi];
    for (int q0 = 0; q0 < nr; q0 += A.chunk) {
        const int qw = min(A.chunk, nr - q0);
        __syncthreads();
        stage_pieces<C, RT>(s_z, zin, A.out_off + bi * A.pieces, A.out_len + bi * A.pieces, A.pieces, q0, qw,
                            A.nrhs, r0, nrr);
        __syncthreads();
        for (int col = wave; col < nc; col += AW) {
            C acc[RT];
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = czero<C>();
            const C* Sc = S + (long long)col * nr + q0;
            for (int row = lane; row < qw; row += 64) {
                const C sv = Sc[row];
#pragma unroll
                for (int r = 0; r < RT; ++r) cfmac(acc[r], sv, s_z[row * RT + r]);
            }
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = wave_sum_c(acc[r]);
            if (lane == 0) {
                const long long off = piece_offset(in_off, in_len, A.pieces, col);
#pragma unroll
                for (int r = 0; r < RT; ++r)
                    if (r < nrr) {
                        C* dst = xout + off * A.nrhs + r0 + r;
                        *dst = q0 == 0 ? acc[r] : cadd(*dst, acc[r]);
                    }
            }
        }
    }
}

// ---- adjoint going down (column side): w(cand) = sum_t Pi_t [z_t ; T_t^H z_t], T column-major ----
template <class C, int RT>
__global__ __launch_bounds__(AT) void adj_down_kernel(DownArgs A) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const long long g = blockIdx.x;
    const int r0 = blockIdx.y * RT;
    const int nr = min(RT, A.nrhs - r0);
    const long long a = g / A.Ps, ap = g - (g / A.Ps) * A.Ps;
    const int ncand = A.lev.n[g * A.G.P];
    C* s_w = reinterpret_cast<C*>(smem_raw);
    C* s_z = s_w + (size_t)A.ncand_max * RT;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int e = tid; e < ncand * RT; e += AT) s_w[e] = czero<C>();
    const C* zin = (const C*)A.in;
    for (int t = 0; t < A.G.P; ++t) {
        const long long id = g * A.G.P + t;
        const int k = A.lev.k[id], nred = A.lev.n[id] - k;
        const int* perm = A.lev.perm + A.lev.perm_off[id];
        const C* T = (const C*)A.lev.T[id];
        const long long yo = A.lev.y_off[id];
        __syncthreads();
        for (int e = tid; e < k * RT; e += AT) {
            const int i = e / RT, r = e - i * RT;
            s_z[e] = (r < nr) ? zin[(yo + i) * A.nrhs + r0 + r] : czero<C>();
        }
        __syncthreads();
        for (int e = tid; e < k * RT; e += AT) {
            const int i = e / RT, r = e - i * RT;
            const int ps = perm[i];
            s_w[ps * RT + r] = cadd(s_w[ps * RT + r], s_z[e]);
        }
        for (int j = wave; j < nred; j += AW) {
            C acc[RT];
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = czero<C>();
            const C* Tj = T + (long long)j * k;
            for (int i = lane; i < k; i += 64) {
                const C tv = Tj[i];
#pragma unroll
                for (int r = 0; r < RT; ++r) cfmac(acc[r], tv, s_z[i * RT + r]);
            }
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = wave_sum_c(acc[r]);
            if (lane == 0) {
                const int pr = perm[k + j];
#pragma unroll
                for (int r = 0; r < RT; ++r) s_w[pr * RT + r] = cadd(s_w[pr * RT + r], acc[r]);
            }
        }
    }
    __syncthreads();
    scatter_candidates<C, RT>(s_w, A.G, A.s, a, ap, A.Ps, (C*)A.ext, A.ld, (C*)A.out, A.k_prev, A.yoff_prev,
                              A.nrhs, r0, nr, A.lev.slot);
}

// ---- a batch of forward transforms in one persistent launch ----
// Every workgroup takes one segment at a time from the queue (one atomic
// add), waits until the segment's dependency stage is complete, runs the same
// body as that stage's own level kernel on each of its items, and counts the
// segment's items complete (one release and atomic add per segment).
// Deadlock freedom: segments are handed out in queue order and depend only on
// earlier segments, so the earliest unfinished one is either held by a
// running workgroup whose dependencies are all complete, or not yet handed
// out while every earlier segment is done; either way some workgroup makes
// progress, whatever the number of resident workgroups.  Waits poll with
// s_sleep and give up after spin_limit polls (counted in the control block),
// so no wait can hang the device.
__device__ inline unsigned ld_relaxed(const unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class C, int RT>
__global__ __launch_bounds__(AT) void persistent_kernel(PersistArgs P) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_seg;
    unsigned* next = P.ctl;
    unsigned* fin = P.ctl + 1;
    unsigned* timeouts = P.ctl + 2;
    unsigned* done = P.ctl + BATCH_CTL_HEAD;
    // The queue's bookkeeping is done by wave 0 as a whole (a branch the compiler
    // sees as wave-uniform), never by a single lane inside the loop: a lane-divergent
    // branch there lets the compiler restructure the loop so that the lanes of wave 0
    // leave it at different iterations, which breaks the barriers.  Only lane 0
    // contributes to each atomic (the other lanes add 0).
    const bool wave0 = __builtin_amdgcn_readfirstlane(threadIdx.x) < 64;
    const unsigned lane0 = threadIdx.x == 0 ? 1u : 0u;
    for (;;) {
        if (wave0) {
            const unsigned v = __hip_atomic_fetch_add(next, lane0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int si = __builtin_amdgcn_readfirstlane((int)v);
            s_seg = si;
        }
        __syncthreads();
        const int si = __builtin_amdgcn_readfirstlane(s_seg);
        __syncthreads();               // s_seg is rewritten by the next step
        if (si >= P.nseg) break;
        const BatchSegment sg = P.seg[si];
        const int q = __builtin_amdgcn_readfirstlane(sg.stage);
        const int cnt = __builtin_amdgcn_readfirstlane(sg.count);
        const long long item0 = (long long)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane(
                                                 (int)((unsigned long long)sg.item0 >> 32)) << 32) |
                                            (unsigned)__builtin_amdgcn_readfirstlane((int)sg.item0));
        const int dep = P.st[q].dep;
        if (dep >= 0) {
            if (wave0) {
                // poll without cache maintenance; one acquire fence once the count is reached
                const unsigned need = (unsigned)P.st[dep].items;
                long long polls = 0;
                while (__builtin_amdgcn_readfirstlane((int)ld_relaxed(done + dep)) < (int)need) {
                    if (++polls > P.spin_limit) {
                        __hip_atomic_fetch_add(timeouts, lane0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(4);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            // wave 0's acquire (agent scope) invalidated this CU's L1 and the stale L2
            // lines; the barrier orders every thread's reads after it
            __syncthreads();
        }
        const int tiles = P.st[q].tiles;
        const int kind = P.st[q].kind;
        for (int u = 0; u < cnt; ++u) {
            const long long item = item0 + u;
            const long long g = item / tiles;
            const int tile = (int)(item - g * tiles);
            if (kind == 0) {
                const UpArgs A = P.st[q].a.up;
                up_body<C, RT, (RT == 1 ? 4 : 1)>(A, g, tile, smem_raw);
            } else if (kind == 1) {
                const MidArgs A = P.st[q].a.mid;
                middle_body<C, RT>(A, g, tile, smem_raw);
            } else {
                const DownArgs A = P.st[q].a.down;
                down_body<C, RT>(A, g, tile, smem_raw);
            }
            __syncthreads();               // the LDS is free for the next item
        }
        // every thread's stores of this segment complete (workgroup scope), then wave 0's
        // release at agent scope publishes them (the L2 write-back covers all of them)
        __threadfence_block();
        __syncthreads();
        if (wave0) __hip_atomic_fetch_add(done + q, lane0 * (unsigned)cnt, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the last workgroup out clears the queue and the counts for the next run
    if (threadIdx.x == 0) {
        const unsigned f = __hip_atomic_fetch_add(fin, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (f == gridDim.x - 1) {
            for (int q = 0; q < P.nst; ++q) __hip_atomic_store(done + q, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(next, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(fin, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <class C, int RT>
void launch_level(LevelKernel which, const void* args, dim3 grid, size_t smem, hipStream_t s) {
    switch (which) {
        case LevelKernel::Up:
            if constexpr (RT == 1)
                hipLaunchKernelGGL((up_kernel<C, RT, 4>), grid, dim3(AT), smem, s, *(const UpArgs*)args);
            else
                hipLaunchKernelGGL((up_kernel<C, RT, 1>), grid, dim3(AT), smem, s, *(const UpArgs*)args);
            break;
        case LevelKernel::Down:
            hipLaunchKernelGGL((down_kernel<C, RT>), grid, dim3(AT), smem, s, *(const DownArgs*)args);
            break;
        case LevelKernel::Middle:
            hipLaunchKernelGGL((middle_kernel<C, RT>), grid, dim3(AT), smem, s, *(const MidArgs*)args);
            break;
        case LevelKernel::AdjUp:
            hipLaunchKernelGGL((adj_up_kernel<C, RT>), grid, dim3(AT), smem, s, *(const UpArgs*)args);
            break;
        case LevelKernel::AdjMiddle:
            hipLaunchKernelGGL((adj_middle_kernel<C, RT>), grid, dim3(AT), smem, s, *(const MidArgs*)args);
            break;
        case LevelKernel::AdjDown:
            hipLaunchKernelGGL((adj_down_kernel<C, RT>), grid, dim3(AT), smem, s, *(const DownArgs*)args);
            break;
    }
    MIDBF_HIP(hipGetLastError());
}

template <class C, int RT>
const void* persistent_fn() {
    return reinterpret_cast<const void*>(&persistent_kernel<C, RT>);
}

const void* persistent_for(int prec, int rt) {
    if (prec == PREC_FP64) return rt == 1 ? persistent_fn<double2, 1>() : persistent_fn<double2, APPLY_RT64>();
    return rt == 1 ? persistent_fn<float2, 1>() : persistent_fn<float2, APPLY_RT>();
}

}  // namespace

int persistent_capacity(int prec, int rt, size_t smem) {
    int dev = 0, cus = 0, per = 0;
    MIDBF_HIP(hipGetDevice(&dev));
    MIDBF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    MIDBF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, persistent_for(prec, rt), AT, smem));
    return std::max(1, per) * std::max(1, cus);
}

void launch_persistent(int prec, int rt, const PersistArgs& P, int grid, size_t smem, hipStream_t s) {
    MIDBF_CHECK(grid >= 1 && P.nseg >= 1 && P.nst >= 1, MIDBF_ERR_SHAPE, "persistent batch launch shape out of range");
    if (prec == PREC_FP64) {
        if (rt == 1) hipLaunchKernelGGL((persistent_kernel<double2, 1>), dim3(grid), dim3(AT), smem, s, P);
        else hipLaunchKernelGGL((persistent_kernel<double2, APPLY_RT64>), dim3(grid), dim3(AT), smem, s, P);
    } else {
        if (rt == 1) hipLaunchKernelGGL((persistent_kernel<float2, 1>), dim3(grid), dim3(AT), smem, s, P);
        else hipLaunchKernelGGL((persistent_kernel<float2, APPLY_RT>), dim3(grid), dim3(AT), smem, s, P);
    }
    MIDBF_HIP(hipGetLastError());
}

void launch_level_kernel(LevelKernel which, int prec, int rt, const void* args, dim3 grid, size_t smem,
                         hipStream_t s) {
    if (prec == PREC_FP64) {
        if (rt == 1) launch_level<double2, 1>(which, args, grid, smem, s);
        else launch_level<double2, APPLY_RT64>(which, args, grid, smem, s);
    } else {
        if (rt == 1) launch_level<float2, 1>(which, args, grid, smem, s);
        else launch_level<float2, APPLY_RT>(which, args, grid, smem, s);
    }
}

}  // namespace midbf
