// Phase recovery on the GPU (Section 2): exp(2 pi i U V^T) ~ K from O(1)
// rows and columns of K, on the lattices of the library or on scattered points.
//
//   * recovery paths on the lattices: the dimension-ordered comb trees of the
//     x and xi lattices (an MST of unit axis edges of the lattice's Delaunay
//     graph, Alg. 5), rooted at x = 0 and xi = 0.  The path from the root to a
//     node first moves along coordinate 0, then 1, ...; so the whole path is d
//     rounds of independent 1-D line walks (round s: every line along axis s
//     that leaves the axis-(s-1) lines), one workgroup per vector;
//   * recovery paths on scattered points (Alg. 5): the Euclidean minimum
//     spanning tree by Prim's algorithm on the device (the Delaunay graph only
//     thins the candidate edges: it holds every edge of this tree), then a
//     breadth-first order from point 0 on the host, neighbours by increasing
//     number; a walk then runs the path's depth levels in turn;
//   * Alg. 4 along those walks: v(ed) = u(ed) - round(u(ed) - v(bg)) with
//     u = angle(K) / 2 pi, block roots (Partition2 cuts) taking their anchors;
//   * Alg. 6: tau schedule on the root column / row, per-block root rows and
//     columns, sampled rows and columns anchored on them;
//   * branch reconciliation for integer frequency lattices (rows whose steps
//     exceed the unwrap limit): screening of every recovered vector by its
//     largest in-block step, integer-shift fit of each row against the
//     accepted columns;
//   * Alg. 1 inside the accepted samples: column-pivoted QR of the sampled
//     intersection for the pivots, orthonormal bases (two-pass classical
//     Gram-Schmidt), the core M = Qc(I,:)^+ A(I,J) (Qr(J,:)^+)^T and its SVD
//     (one-sided Jacobi), then U = Qc U_M, V = Qr V_M S (Alg. 7).
#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>
#include <vector>

#include "recover.h"

namespace midbf {

namespace {

constexpr int WT = 1024;             // threads of the vector kernels
constexpr int MAXS = 64;             // sampled rows / columns kept (r q + flagged nodes)
constexpr int MAXR = 16;             // rank
constexpr double TAU_AMB = 0.4;      // largest in-block step of an accepted vector
constexpr double FIT_TOL = 1e-6;     // residual of an exact integer-shift fit
constexpr int DMAX = 16;             // flagged nodes tolerated by the tau schedule

struct Lattice {
    int d, n;
    long long N;
    int q[3];             // root coordinates
    long long stride[3];  // C order: the last coordinate is contiguous
};

Lattice make_lattice(int d, int n, int qv) {
    Lattice L{};
    L.d = d;
    L.n = n;
    L.N = 1;
    for (int k = 0; k < d; ++k) L.N *= n;
    long long s = 1;
    for (int k = d - 1; k >= 0; --k) {
        L.stride[k] = s;
        s *= n;
        L.q[k] = qv;
    }
    return L;
}

long long lattice_root(const Lattice& L) {
    long long r = 0;
    for (int k = 0; k < L.d; ++k) r += L.q[k] * L.stride[k];
    return r;
}

int manhattan_depth(const Lattice& L, long long p) {
    int dep = 0;
    for (int k = 0; k < L.d; ++k) dep += std::abs((int)((p / L.stride[k]) % L.n) - L.q[k]);
    return dep;
}

// Visit every edge (parent -> node) of the comb tree in an order where the
// parent is final first; f(p, parent) per edge, barriers between rounds.
template <class F>
__device__ void comb_walk(const Lattice& L, F&& f) {
    for (int s = 0; s < L.d; ++s) {
        __syncthreads();
        long long nlines = 1;
        for (int k = 0; k < s; ++k) nlines *= L.n;
        for (long long task = threadIdx.x; task < 2 * nlines; task += WT) {
            const long long line = task >> 1;
            const int dir = (task & 1) ? -1 : 1;
            long long t = line, start = 0;
            for (int k = s - 1; k >= 0; --k) {
                start += (t % L.n) * L.stride[k];
                t /= L.n;
            }
            for (int k = s; k < L.d; ++k) start += L.q[k] * L.stride[k];
            long long par = start;
            for (int c = L.q[s] + dir; c >= 0 && c < L.n; c += dir) {
                const long long p = par + dir * L.stride[s];
                f(p, par);
                par = p;
            }
        }
    }
    __syncthreads();
}

// A general recovery path: rows (pred, node) grouped by depth, level l holding
// rows lev_off[l] .. lev_off[l+1]; the walk runs the levels in turn.
struct PathWalk {
    const int* path;             // (N - 1) x 2, or null: the lattice's comb tree
    const long long* lev_off;
    int nlev;
    long long root;
};

struct UnwrapArgs {
    Lattice L;
    PathWalk pw;
    const double2* kv;            // the sampled row or column of K
    double* u;                    // wrapped phase angle(K) / 2 pi (out)
    double* v;                    // recovered phase (out)
    double* inc;                  // |v(p) - v(parent)| per node, 0 at the path root (out) or null
    const int* root_block;        // block whose root the node is, else -1; null: the path root only
    const double* anchor_vecs;    // anchor of block b: anchor_vecs[b * N + anchor_index]; null: raw u
    long long anchor_index;
    double* maxinc;               // out: largest |v(p) - v(parent)| over edges inside one block
};

__global__ __launch_bounds__(WT) void unwrap_kernel(UnwrapArgs A) {
    __shared__ double s_max[WT / 64];
    const long long N = A.L.N;
    for (long long p = threadIdx.x; p < N; p += WT) A.u[p] = atan2(A.kv[p].y, A.kv[p].x) / (2.0 * M_PI);
    __syncthreads();
    auto anchor = [&](int b, long long p) {
        return A.anchor_vecs ? A.anchor_vecs[(long long)b * N + A.anchor_index] : A.u[p];
    };
    const long long root = [&] {
        if (A.pw.path) return A.pw.root;
        long long r = 0;
        for (int k = 0; k < A.L.d; ++k) r += A.L.q[k] * A.L.stride[k];
        return r;
    }();
    if (threadIdx.x == 0) {
        A.v[root] = anchor(0, root);
        if (A.inc) A.inc[root] = 0.0;
    }
    double mx = 0.0;
    auto step = [&](long long p, long long par) {
        const int rb = A.root_block ? A.root_block[p] : -1;
        const double vpar = A.v[par];
        double vp;
        if (rb >= 0) {
            vp = anchor(rb, p);
        } else {
            const double up = A.u[p];
            vp = up - round(up - vpar);           // Alg. 4 (round half away from zero)
        }
        A.v[p] = vp;
        const double dl = fabs(vp - vpar);
        if (A.inc) A.inc[p] = dl;
        if (rb < 0) mx = fmax(mx, dl);
    };
    if (A.pw.path) {
        for (int l = 0; l < A.pw.nlev; ++l) {
            __syncthreads();
            for (long long e = A.pw.lev_off[l] + threadIdx.x; e < A.pw.lev_off[l + 1]; e += WT)
                step(A.pw.path[2 * e + 1], A.pw.path[2 * e]);
        }
        __syncthreads();
    } else {
        comb_walk(A.L, step);
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < WT / 64; ++w) m = fmax(m, s_max[w]);
        *A.maxinc = m;
    }
}

// Euclidean minimum spanning tree of N points (Prim's algorithm, one
// workgroup): per step every thread updates the keys (squared distance to the
// tree, FP64) of its points outside the tree against the point just added,
// then the block adds the nearest outside point (ties: the smaller number).
__global__ __launch_bounds__(WT) void prim_kernel(const double* pts, long long N, int d, long long root, double* key,
                                                  int* parent, unsigned char* in) {
    __shared__ double s_v[WT / 64];
    __shared__ long long s_i[WT / 64];
    __shared__ long long s_u;
    for (long long v = threadIdx.x; v < N; v += WT) {
        key[v] = INFINITY;
        parent[v] = -1;
        in[v] = v == root;
    }
    if (threadIdx.x == 0) s_u = root;
    __syncthreads();
    for (long long it = 1; it < N; ++it) {
        const long long u = s_u;
        double pu[3] = {0, 0, 0};
        for (int k = 0; k < d; ++k) pu[k] = pts[u * d + k];
        double best = INFINITY;
        long long bi = N;
        for (long long v = threadIdx.x; v < N; v += WT) {
            if (in[v]) continue;
            double s = 0.0;
            for (int k = 0; k < d; ++k) {
                const double dv = pts[v * d + k] - pu[k];
                s += dv * dv;
            }
            double kv = key[v];
            if (s < kv) {
                kv = s;
                key[v] = s;
                parent[v] = (int)u;
            }
            if (kv < best || (kv == best && v < bi)) { best = kv; bi = v; }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o, 64);
            const long long oi = __shfl_xor(bi, o, 64);
            if (ob < best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if ((threadIdx.x & 63) == 0) { s_v[threadIdx.x >> 6] = best; s_i[threadIdx.x >> 6] = bi; }
        __syncthreads();
        if (threadIdx.x == 0) {
            double b = s_v[0];
            long long i = s_i[0];
            for (int w = 1; w < WT / 64; ++w)
                if (s_v[w] < b || (s_v[w] == b && s_i[w] < i)) { b = s_v[w]; i = s_i[w]; }
            s_u = i < N ? i : u;
            if (i < N) in[i] = 1;
        }
        __syncthreads();
    }
}

// Integer-shift fit of a recovered row against the accepted columns:
// D_j = AC(i, j) - v(C_j) = m . xi_{C_j} + a, solved in least squares
// (normal equations), rounded half away from zero, kept if the residual is
// below FIT_TOL; then row = v + m . xi + a.
struct FitArgs {
    const double* v;
    const double* AC;        // N x ncol, column-major
    const long long* C;
    const double* xi;        // N x d, row-major
    int ncol, d;
    long long N, i;
    double* row_out;         // N values, written when accepted
    int* result;             // [0] accepted, [1..d] m, [d+1] a
};

__global__ __launch_bounds__(WT) void fit_kernel(FitArgs A) {
    __shared__ double s_coef[4];
    __shared__ int s_ok;
    const int d1 = A.d + 1;
    if (threadIdx.x == 0) {
        double G[4][4] = {}, b[4] = {};
        for (int j = 0; j < A.ncol; ++j) {
            const long long c = A.C[j];
            const double D = A.AC[(long long)j * A.N + A.i] - A.v[c];
            double x[4];
            for (int k = 0; k < A.d; ++k) x[k] = A.xi[c * A.d + k];
            x[A.d] = 1.0;
            for (int r = 0; r < d1; ++r) {
                b[r] += x[r] * D;
                for (int s = 0; s < d1; ++s) G[r][s] += x[r] * x[s];
            }
        }
        // Gaussian elimination with partial pivoting
        int ok = 1;
        for (int k = 0; k < d1; ++k) {
            int p = k;
            for (int r = k + 1; r < d1; ++r)
                if (fabs(G[r][k]) > fabs(G[p][k])) p = r;
            if (G[p][k] == 0.0) {
                ok = 0;
                break;
            }
            if (p != k) {
                for (int s = 0; s < d1; ++s) {
                    const double t = G[k][s];
                    G[k][s] = G[p][s];
                    G[p][s] = t;
                }
                const double t = b[k];
                b[k] = b[p];
                b[p] = t;
            }
            for (int r = k + 1; r < d1; ++r) {
                const double f = G[r][k] / G[k][k];
                for (int s = k; s < d1; ++s) G[r][s] -= f * G[k][s];
                b[r] -= f * b[k];
            }
        }
        double coef[4] = {};
        if (ok) {
            for (int k = d1 - 1; k >= 0; --k) {
                double t = b[k];
                for (int s = k + 1; s < d1; ++s) t -= G[k][s] * coef[s];
                coef[k] = t / G[k][k];
            }
            for (int k = 0; k < d1; ++k) coef[k] = round(coef[k]);
            double res = 0.0;
            for (int j = 0; j < A.ncol; ++j) {
                const long long c = A.C[j];
                const double D = A.AC[(long long)j * A.N + A.i] - A.v[c];
                double f = coef[A.d];
                for (int k = 0; k < A.d; ++k) f += A.xi[c * A.d + k] * coef[k];
                res = fmax(res, fabs(D - f));
            }
            ok = res <= FIT_TOL;
        }
        for (int k = 0; k < d1; ++k) s_coef[k] = coef[k];
        s_ok = ok;
        A.result[0] = ok;
        for (int k = 0; k < d1; ++k) A.result[1 + k] = (int)coef[k];
    }
    __syncthreads();
    if (!s_ok) return;
    for (long long p = threadIdx.x; p < A.N; p += WT) {
        double f = 0.0;
        for (int k = 0; k < A.d; ++k) f += A.xi[p * A.d + k] * s_coef[k];
        A.row_out[p] = A.v[p] + (f + s_coef[A.d]);
    }
}

// Column-pivoted QR (Householder, exact residual norms) of an m x n matrix in
// LDS, single thread; writes the full pivot order.
__device__ void cpqr_pivots(double* A, int m, int n, int lda, int* piv) {
    for (int j = 0; j < n; ++j) piv[j] = j;
    const int kmax = m < n ? m : n;
    for (int k = 0; k < kmax; ++k) {
        int p = k;
        double best = -1.0;
        for (int j = k; j < n; ++j) {
            double s = 0.0;
            for (int i = k; i < m; ++i) s += A[j * lda + i] * A[j * lda + i];
            if (s > best) {
                best = s;
                p = j;
            }
        }
        if (p != k) {
            for (int i = 0; i < m; ++i) {
                const double t = A[k * lda + i];
                A[k * lda + i] = A[p * lda + i];
                A[p * lda + i] = t;
            }
            const int t = piv[k];
            piv[k] = piv[p];
            piv[p] = t;
        }
        const double alpha = A[k * lda + k];
        double xn = 0.0;
        for (int i = k + 1; i < m; ++i) xn += A[k * lda + i] * A[k * lda + i];
        if (xn == 0.0) continue;
        const double beta = -copysign(sqrt(alpha * alpha + xn), alpha);
        const double tauh = (beta - alpha) / beta;
        const double scl = 1.0 / (alpha - beta);
        for (int i = k + 1; i < m; ++i) A[k * lda + i] *= scl;
        A[k * lda + k] = beta;
        for (int j = k + 1; j < n; ++j) {
            double w = A[j * lda + k];
            for (int i = k + 1; i < m; ++i) w += A[k * lda + i] * A[j * lda + i];
            w *= tauh;
            A[j * lda + k] -= w;
            for (int i = k + 1; i < m; ++i) A[j * lda + i] -= w * A[k * lda + i];
        }
    }
}

// Pivots of the sampled intersection A(R, C) (columns) and of its transpose (rows).
__global__ void pivots_kernel(const double* AR, const long long* C, int nR, int nC, long long N, int* pc, int* pr) {
    __shared__ double S[MAXS * MAXS];
    for (int e = threadIdx.x; e < nR * nC; e += blockDim.x) {
        const int rho = e % nR, c = e / nR;
        S[c * MAXS + rho] = AR[(long long)rho * N + C[c]];
    }
    __syncthreads();
    if (threadIdx.x == 0) cpqr_pivots(S, nR, nC, MAXS, pc);
    __syncthreads();
    for (int e = threadIdx.x; e < nR * nC; e += blockDim.x) {
        const int rho = e % nR, c = e / nR;
        S[rho * MAXS + c] = AR[(long long)rho * N + C[c]];      // transpose: nC x nR
    }
    __syncthreads();
    if (threadIdx.x == 0) cpqr_pivots(S, nC, nR, MAXS, pr);
}

// Q (N x r, column-major) = orthonormal basis of the vectors src + idx[k] * N
// (two passes of classical Gram-Schmidt).
__global__ __launch_bounds__(WT) void cgs2_kernel(const double* src, const int* idx, int r, long long N, double* Q) {
    __shared__ double s_part[WT / 64][MAXR];
    __shared__ double s_h[MAXR];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < r; ++k) {
        double* w = Q + (long long)k * N;
        const double* a = src + (long long)idx[k] * N;
        for (long long p = threadIdx.x; p < N; p += WT) w[p] = a[p];
        for (int pass = 0; pass < 2 && k > 0; ++pass) {
            __syncthreads();
            double h[MAXR];
            for (int j = 0; j < k; ++j) h[j] = 0.0;
            for (long long p = threadIdx.x; p < N; p += WT) {
                const double wp = w[p];
                for (int j = 0; j < k; ++j) h[j] += Q[(long long)j * N + p] * wp;
            }
            for (int j = 0; j < k; ++j) {
                double t = h[j];
                for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
                if (lane == 0) s_part[wave][j] = t;
            }
            __syncthreads();
            if (threadIdx.x < k) {
                double t = 0.0;
                for (int ww = 0; ww < WT / 64; ++ww) t += s_part[ww][threadIdx.x];
                s_h[threadIdx.x] = t;
            }
            __syncthreads();
            for (long long p = threadIdx.x; p < N; p += WT) {
                double t = w[p];
                for (int j = 0; j < k; ++j) t -= Q[(long long)j * N + p] * s_h[j];
                w[p] = t;
            }
        }
        __syncthreads();
        double t = 0.0;
        for (long long p = threadIdx.x; p < N; p += WT) t += w[p] * w[p];
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        if (lane == 0) s_part[wave][0] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int ww = 0; ww < WT / 64; ++ww) s += s_part[ww][0];
            s_h[0] = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
        }
        __syncthreads();
        const double inv = s_h[0];
        for (long long p = threadIdx.x; p < N; p += WT) w[p] *= inv;
        __syncthreads();
    }
}

// One-sided Jacobi SVD of B (m x n, m >= n, column-major, leading dim ldb):
// on return B's columns are U * sigma, V (n x n, leading dim ldv) the right
// vectors, sig the column norms.
__device__ void jacobi_svd(double* B, int m, int n, int ldb, double* V, int ldv, double* sig) {
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) V[j * ldv + i] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        bool rotated = false;
        for (int p = 0; p < n - 1; ++p)
            for (int qq = p + 1; qq < n; ++qq) {
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = 0; i < m; ++i) {
                    const double x = B[p * ldb + i], y = B[qq * ldb + i];
                    al += x * x;
                    be += y * y;
                    ga += x * y;
                }
                if (fabs(ga) <= 1e-15 * sqrt(al * be) || ga == 0.0) continue;
                rotated = true;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                for (int i = 0; i < m; ++i) {
                    const double x = B[p * ldb + i], y = B[qq * ldb + i];
                    B[p * ldb + i] = c * x - s * y;
                    B[qq * ldb + i] = s * x + c * y;
                }
                for (int i = 0; i < n; ++i) {
                    const double x = V[p * ldv + i], y = V[qq * ldv + i];
                    V[p * ldv + i] = c * x - s * y;
                    V[qq * ldv + i] = s * x + c * y;
                }
            }
        if (!rotated) break;
    }
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += B[j * ldb + i] * B[j * ldb + i];
        sig[j] = sqrt(s);
    }
}

// pinv(B) for B (m x n, m >= n): V diag(1/sigma) U^T with cutoff 1e-15 sigma_max
// (written as P, n x m, column-major leading dim ldp).  B is destroyed.
__device__ void pinv_tall(double* B, int m, int n, int ldb, double* V, double* sig, double* P, int ldp) {
    jacobi_svd(B, m, n, ldb, V, MAXR, sig);
    double smax = 0.0;
    for (int j = 0; j < n; ++j) smax = fmax(smax, sig[j]);
    for (int i = 0; i < m; ++i)
        for (int a = 0; a < n; ++a) {
            double t = 0.0;
            for (int j = 0; j < n; ++j)
                if (sig[j] > 1e-15 * smax) t += V[j * MAXR + a] * B[j * ldb + i] / (sig[j] * sig[j]);
            P[i * ldp + a] = t;     // column i of P (n x m)
        }
}

struct CoreArgs {
    const double* Qc;        // N x r, column-major
    const double* Qr;
    const double* AR;        // nR x N, row-major
    const long long* I;      // 2r global row indices
    const int* It;           // their positions in the accepted rows
    const long long* J;      // 2r global column indices
    int r;
    long long N;
    double* UM;              // r x r, column-major (out)
    double* VM;              // r x r, column-major (out)
    double* sig;             // r (out)
};

// M = Qc(I,:)^+ A(I,J) (Qr(J,:)^+)^T and its SVD (Alg. 1's core), single thread.
__global__ void core_kernel(CoreArgs A) {
    __shared__ double B[2 * MAXR * MAXR], V[MAXR * MAXR], Pc[MAXR * 2 * MAXR], Pr[MAXR * 2 * MAXR];
    __shared__ double AIJ[2 * MAXR * 2 * MAXR], T1[MAXR * 2 * MAXR], M[MAXR * MAXR], sg[MAXR];
    if (threadIdx.x != 0) return;
    const int r = A.r, m = 2 * r, ldb = 2 * MAXR;
    // pinv(Qc(I,:))  (r x 2r)
    for (int k = 0; k < r; ++k)
        for (int a = 0; a < m; ++a) B[k * ldb + a] = A.Qc[(long long)k * A.N + A.I[a]];
    pinv_tall(B, m, r, ldb, V, sg, Pc, MAXR);
    // pinv(Qr(J,:))  (r x 2r)
    for (int k = 0; k < r; ++k)
        for (int b = 0; b < m; ++b) B[k * ldb + b] = A.Qr[(long long)k * A.N + A.J[b]];
    pinv_tall(B, m, r, ldb, V, sg, Pr, MAXR);
    // A(I, J)  (2r x 2r, column-major leading dim 2 MAXR)
    for (int b = 0; b < m; ++b)
        for (int a = 0; a < m; ++a) AIJ[b * ldb + a] = A.AR[(long long)A.It[a] * A.N + A.J[b]];
    // T1 = Pc A(I,J)  (r x 2r), M = T1 Pr^T  (r x r)
    for (int b = 0; b < m; ++b)
        for (int i = 0; i < r; ++i) {
            double t = 0.0;
            for (int a = 0; a < m; ++a) t += Pc[a * MAXR + i] * AIJ[b * ldb + a];
            T1[b * MAXR + i] = t;
        }
    for (int j = 0; j < r; ++j)
        for (int i = 0; i < r; ++i) {
            double t = 0.0;
            for (int b = 0; b < m; ++b) t += T1[b * MAXR + i] * Pr[b * MAXR + j];
            M[j * MAXR + i] = t;
        }
    // SVD of M: M = U_M diag(sig) V_M^T
    jacobi_svd(M, r, r, MAXR, V, MAXR, sg);
    for (int j = 0; j < r; ++j) {
        A.sig[j] = sg[j];
        for (int i = 0; i < r; ++i) {
            A.UM[j * r + i] = sg[j] > 0.0 ? M[j * MAXR + i] / sg[j] : (i == j ? 1.0 : 0.0);
            A.VM[j * r + i] = V[j * MAXR + i];
        }
    }
}

// U = Qc U_M, V = Qr V_M diag(sig): N x r row-major outputs.
__global__ void factors_kernel(const double* Qc, const double* Qr, const double* UM, const double* VM,
                               const double* sig, int r, long long N, double* U, double* V) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    for (int j = 0; j < r; ++j) {
        double u = 0.0, v = 0.0;
        for (int k = 0; k < r; ++k) {
            u += Qc[(long long)k * N + p] * UM[j * r + k];
            v += Qr[(long long)k * N + p] * VM[j * r + k];
        }
        U[p * r + j] = u;
        V[p * r + j] = v * sig[j];
    }
}

uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// The seeded order of 0..N-1: sorted by splitmix64(seed + 2 i + stream), then i.
std::vector<long long> sample_order(long long N, uint64_t seed, int stream) {
    std::vector<std::pair<uint64_t, long long>> key(N);
    for (long long i = 0; i < N; ++i) key[i] = {splitmix64(seed + 2ull * (uint64_t)i + (uint64_t)stream), i};
    std::sort(key.begin(), key.end());
    std::vector<long long> out(N);
    for (long long i = 0; i < N; ++i) out[i] = key[i].second;
    return out;
}

struct DevBuf {
    void* p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    template <class T> T* alloc(size_t count) {
        MIDBF_HIP(hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)));
        return (T*)p;
    }
};

// The recovery path of scattered points (Alg. 5 with the tree computed
// directly): rows (pred, node) in breadth-first order from root, neighbours in
// increasing number; levels by depth; the row of every node (-1: the root).
struct HostPath {
    std::vector<int> P;
    std::vector<long long> lev, rowpos;
};

HostPath points_path(const double* pts, long long N, int d, long long root, hipStream_t st) {
    MIDBF_CHECK(N >= 1 && root >= 0 && root < N && (d == 2 || d == 3), MIDBF_ERR_ARG, "bad point set");
    DevBuf b_pts, b_key, b_par, b_in;
    double* d_pts = b_pts.alloc<double>((size_t)N * d);
    double* d_key = b_key.alloc<double>(N);
    int* d_par = b_par.alloc<int>(N);
    unsigned char* d_in = b_in.alloc<unsigned char>(N);
    MIDBF_HIP(hipMemcpyAsync(d_pts, pts, (size_t)N * d * sizeof(double), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(prim_kernel, dim3(1), dim3(WT), 0, st, (const double*)d_pts, N, d, root, d_key, d_par, d_in);
    MIDBF_HIP(hipGetLastError());
    std::vector<int> parent(N);
    MIDBF_HIP(hipMemcpyAsync(parent.data(), d_par, N * sizeof(int), hipMemcpyDeviceToHost, st));
    MIDBF_HIP(hipStreamSynchronize(st));
    // undirected adjacency, neighbours sorted
    std::vector<long long> deg(N + 1, 0);
    for (long long v = 0; v < N; ++v)
        if (v != root) {
            MIDBF_CHECK(parent[v] >= 0 && parent[v] < N, MIDBF_ERR_HIP, "spanning tree incomplete");
            ++deg[v + 1];
            ++deg[parent[v] + 1];
        }
    for (long long v = 0; v < N; ++v) deg[v + 1] += deg[v];
    std::vector<int> adj(deg[N]);
    std::vector<long long> fill(deg.begin(), deg.end() - 1);
    for (long long v = 0; v < N; ++v)
        if (v != root) {
            adj[fill[v]++] = parent[v];
            adj[fill[parent[v]]++] = (int)v;
        }
    for (long long v = 0; v < N; ++v) std::sort(adj.begin() + deg[v], adj.begin() + deg[v + 1]);
    HostPath H;
    H.P.reserve(2 * (N - 1));
    H.rowpos.assign(N, -1);
    std::vector<int> depth(N, -1);
    std::vector<long long> queue{root};
    depth[root] = 0;
    for (size_t h = 0; h < queue.size(); ++h) {
        const long long u = queue[h];
        for (long long e = deg[u]; e < deg[u + 1]; ++e) {
            const int v = adj[e];
            if (depth[v] >= 0) continue;
            depth[v] = depth[u] + 1;
            H.rowpos[v] = (long long)H.P.size() / 2;
            H.P.push_back((int)u);
            H.P.push_back(v);
            queue.push_back(v);
        }
    }
    MIDBF_CHECK((long long)queue.size() == N, MIDBF_ERR_HIP, "spanning tree not connected");
    H.lev.push_back(0);
    for (long long e = 1; e < N - 1 + 1; ++e)
        if (e == N - 1 || depth[H.P[2 * e + 1]] != depth[H.P[2 * (e - 1) + 1]]) H.lev.push_back(e);
    return H;
}

}  // namespace

void recovery_path_points(const double* pts, long long N, int d, long long root, int* P_out, hipStream_t st) {
    const HostPath H = points_path(pts, N, d, root, st);
    std::copy(H.P.begin(), H.P.end(), P_out);
}

void phase_recover_run(int d, int n, const double* X1, const double* X2, midbf_sample_cb cb, void* user, int r,
                       int q, double tau, uint64_t seed, hipStream_t st, double* U_dev, double* V_dev,
                       phase_recover_info* info_out, long long Npts) {
    MIDBF_CHECK(d == 2 || d == 3, MIDBF_ERR_ARG, "d must be 2 or 3");
    MIDBF_CHECK(Npts > 0 || (n >= 2 && n % 2 == 0), MIDBF_ERR_ARG, "n must be even and >= 2");
    MIDBF_CHECK(Npts == 0 || (X1 && X2 && Npts >= 2), MIDBF_ERR_ARG, "scattered points need x and xi coordinates");
    MIDBF_CHECK(cb && U_dev && V_dev, MIDBF_ERR_ARG, "null sampler or output");
    MIDBF_CHECK(r >= 1 && r <= MAXR && q >= 1 && r * q <= 32, MIDBF_ERR_ARG, "need 1 <= r <= 16 and r q <= 32");
    MIDBF_CHECK(tau > 0.0 && tau <= 0.5, MIDBF_ERR_ARG, "tau must lie in (0, 1/2]");
    // the two recovery paths: the lattices' comb trees (the x lattice enters only through its
    // path), or the point sets' spanning trees rooted at point 0
    const bool pts = Npts > 0;
    const Lattice Lx = pts ? Lattice{} : make_lattice(d, n, 0), Lk = pts ? Lattice{} : make_lattice(d, n, n / 2);
    const long long N = pts ? Npts : Lx.N;
    const long long r1 = pts ? 0 : lattice_root(Lx), r2 = pts ? 0 : lattice_root(Lk);
    HostPath Hx, Hk;
    DevBuf b_px, b_pk, b_lx, b_lk;
    PathWalk Wx{}, Wk{};
    if (pts) {
        Hx = points_path(X1, N, d, r1, st);
        Hk = points_path(X2, N, d, r2, st);
        int* dpx = b_px.alloc<int>(Hx.P.size());
        int* dpk = b_pk.alloc<int>(Hk.P.size());
        long long* dlx = b_lx.alloc<long long>(Hx.lev.size());
        long long* dlk = b_lk.alloc<long long>(Hk.lev.size());
        MIDBF_HIP(hipMemcpyAsync(dpx, Hx.P.data(), Hx.P.size() * sizeof(int), hipMemcpyHostToDevice, st));
        MIDBF_HIP(hipMemcpyAsync(dpk, Hk.P.data(), Hk.P.size() * sizeof(int), hipMemcpyHostToDevice, st));
        MIDBF_HIP(hipMemcpyAsync(dlx, Hx.lev.data(), Hx.lev.size() * sizeof(long long), hipMemcpyHostToDevice, st));
        MIDBF_HIP(hipMemcpyAsync(dlk, Hk.lev.data(), Hk.lev.size() * sizeof(long long), hipMemcpyHostToDevice, st));
        Wx = PathWalk{dpx, dlx, (int)Hx.lev.size() - 1, r1};
        Wk = PathWalk{dpk, dlk, (int)Hk.lev.size() - 1, r2};
    }
    phase_recover_info info{};
    // xi coordinates (row-major N x d) for the integer-shift fit
    std::vector<double> xi((size_t)N * d);
    for (long long p = 0; p < N; ++p)
        for (int k = 0; k < d; ++k)
            xi[p * d + k] = X2 ? X2[p * d + k] : (double)((p / Lk.stride[k]) % n - n / 2);

    double* hb = nullptr;
    MIDBF_HIP(hipHostMalloc((void**)&hb, (size_t)N * 16));
    struct HostFree {
        double* p;
        ~HostFree() { (void)hipHostFree(p); }
    } hb_guard{hb};
    DevBuf b_kv, b_u, b_v, b_inc, b_max, b_xi, b_rbr, b_rbc, b_rootrow, b_rootcol, b_AC, b_AR, b_C, b_fit, b_piv,
        b_Qc, b_Qr, b_idx, b_core, b_IJ;
    double2* d_kv = b_kv.alloc<double2>(N);
    double* d_u = b_u.alloc<double>(N);
    double* d_v = b_v.alloc<double>(N);
    double* d_inc = b_inc.alloc<double>(N);
    double* d_max = b_max.alloc<double>(1);
    double* d_xi = b_xi.alloc<double>((size_t)N * d);
    int* d_rbr = b_rbr.alloc<int>(N);
    int* d_rbc = b_rbc.alloc<int>(N);
    MIDBF_HIP(hipMemcpyAsync(d_xi, xi.data(), xi.size() * sizeof(double), hipMemcpyHostToDevice, st));

    auto fetch = [&](int is_row, long long idx) {
        MIDBF_HIP(hipStreamSynchronize(st));          // the previous copy out of hb has finished
        ++info.callbacks;
        if (cb(user, is_row, idx, hb) != 0) throw Error(MIDBF_ERR_RECOVERY, "the sampler failed");
        MIDBF_HIP(hipMemcpyAsync(d_kv, hb, (size_t)N * 16, hipMemcpyHostToDevice, st));
    };
    auto unwrap = [&](const Lattice& L, const int* root_block, const double* anchors, long long aidx, double* v_out,
                      bool want_inc) {
        UnwrapArgs a{};
        a.L = L;
        a.L.N = N;
        a.pw = &L == &Lx ? Wx : Wk;
        a.kv = d_kv;
        a.u = d_u;
        a.v = v_out;
        a.inc = want_inc ? d_inc : nullptr;
        a.root_block = root_block;
        a.anchor_vecs = anchors;
        a.anchor_index = aidx;
        a.maxinc = d_max;
        hipLaunchKernelGGL(unwrap_kernel, dim3(1), dim3(WT), 0, st, a);
        MIDBF_HIP(hipGetLastError());
    };
    auto read_max = [&] {
        double m = 0.0;
        MIDBF_HIP(hipMemcpyAsync(&m, d_max, sizeof(double), hipMemcpyDeviceToHost, st));
        MIDBF_HIP(hipStreamSynchronize(st));
        return m;
    };

    // ---- Alg. 6: tau schedule on the root column (over x) and root row (over xi)
    std::vector<double> inc_r(N), inc_c(N);
    fetch(0, r2);
    unwrap(Lx, nullptr, nullptr, 0, d_v, true);
    MIDBF_HIP(hipMemcpyAsync(inc_r.data(), d_inc, N * sizeof(double), hipMemcpyDeviceToHost, st));
    fetch(1, r1);
    unwrap(Lk, nullptr, nullptr, 0, d_v, true);
    MIDBF_HIP(hipMemcpyAsync(inc_c.data(), d_inc, N * sizeof(double), hipMemcpyDeviceToHost, st));
    MIDBF_HIP(hipStreamSynchronize(st));
    auto flagged = [&](const std::vector<double>& inc, const Lattice& L, long long root, double t) {
        const HostPath& H = &L == &Lx ? Hx : Hk;
        std::vector<std::pair<long long, long long>> f;
        for (long long p = 0; p < N; ++p)
            if (p != root && inc[p] >= t) f.push_back({pts ? H.rowpos[p] : (long long)manhattan_depth(L, p), p});
        std::sort(f.begin(), f.end());                // path order (lattice: depth, then node number)
        std::vector<long long> D{root};
        for (auto& e : f) D.push_back(e.second);
        return D;
    };
    std::vector<long long> Dr, Dc;
    double t_cur = tau;
    for (;;) {
        Dr = flagged(inc_r, Lx, r1, t_cur);
        Dc = flagged(inc_c, Lk, r2, t_cur);
        if (t_cur == tau) {
            info.disc_rows_initial = (int)Dr.size() - 1;
            info.disc_cols_initial = (int)Dc.size() - 1;
        }
        if (((int)Dr.size() - 1 <= DMAX && (int)Dc.size() - 1 <= DMAX) || t_cur >= 0.5) break;
        t_cur += 1.0 / 40.0;
    }
    MIDBF_CHECK((int)Dr.size() + r * q <= MAXS && (int)Dc.size() + r * q <= MAXS, MIDBF_ERR_RECOVERY,
                "too many discontinuities flagged at tau = 1/2");
    info.tau = t_cur;
    info.disc_rows = (int)Dr.size() - 1;
    info.disc_cols = (int)Dc.size() - 1;

    // ---- Partition2: block roots (blocks numbered in the order of D)
    std::vector<int> rbr(N, -1), rbc(N, -1);
    for (size_t b = 0; b < Dr.size(); ++b) rbr[Dr[b]] = (int)b;
    for (size_t b = 0; b < Dc.size(); ++b) rbc[Dc[b]] = (int)b;
    MIDBF_HIP(hipMemcpyAsync(d_rbr, rbr.data(), N * sizeof(int), hipMemcpyHostToDevice, st));
    MIDBF_HIP(hipMemcpyAsync(d_rbc, rbc.data(), N * sizeof(int), hipMemcpyHostToDevice, st));
    // recovered root row of every row block (over xi, raw anchors at the column-block roots)
    // and root column of every column block (over x, raw anchors at the row-block roots)
    double* d_rootrow = b_rootrow.alloc<double>((size_t)Dr.size() * N);
    double* d_rootcol = b_rootcol.alloc<double>((size_t)Dc.size() * N);
    for (size_t s = 0; s < Dr.size(); ++s) {
        fetch(1, Dr[s]);
        unwrap(Lk, d_rbc, nullptr, 0, d_rootrow + s * N, false);
    }
    for (size_t t = 0; t < Dc.size(); ++t) {
        fetch(0, Dc[t]);
        unwrap(Lx, d_rbr, nullptr, 0, d_rootcol + t * N, false);
    }

    // ---- sampled columns: anchored on the root rows, screened
    const int want = r * q;
    const int wantC = want + (int)Dc.size(), wantR = want + (int)Dr.size();
    double* d_AC = b_AC.alloc<double>((size_t)wantC * N);
    double* d_AR = b_AR.alloc<double>((size_t)wantR * N);
    std::vector<long long> C, R;
    std::vector<std::array<int, 4>> shifts;
    auto candidates = [&](const std::vector<long long>& D, int stream) {
        std::vector<long long> cand(D);
        std::vector<char> inD(N, 0);
        for (long long x : D) inD[x] = 1;
        for (long long x : sample_order(N, seed, stream))
            if (!inD[x]) cand.push_back(x);
        return cand;
    };
    for (long long j : candidates(Dc, 1)) {
        fetch(0, j);
        double* dst = d_AC + (size_t)C.size() * N;
        unwrap(Lx, d_rbr, d_rootrow, j, dst, false);
        if (read_max() < TAU_AMB) {
            C.push_back(j);
            if ((int)C.size() == wantC) break;
        } else {
            ++info.rejected_cols;
        }
    }
    MIDBF_CHECK((int)C.size() == wantC, MIDBF_ERR_RECOVERY, "too few columns passed the screening");
    long long* d_C = b_C.alloc<long long>(C.size());
    MIDBF_HIP(hipMemcpyAsync(d_C, C.data(), C.size() * sizeof(long long), hipMemcpyHostToDevice, st));

    // ---- sampled rows: anchored on the root columns, screened, integer-shift fit
    int* d_fit = b_fit.alloc<int>(8);
    for (long long i : candidates(Dr, 0)) {
        fetch(1, i);
        unwrap(Lk, d_rbc, d_rootcol, i, d_v, false);
        if (read_max() >= TAU_AMB) {
            ++info.rejected_rows;
            continue;
        }
        FitArgs fa{};
        fa.v = d_v;
        fa.AC = d_AC;
        fa.C = d_C;
        fa.xi = d_xi;
        fa.ncol = (int)C.size();
        fa.d = d;
        fa.N = N;
        fa.i = i;
        fa.row_out = d_AR + (size_t)R.size() * N;
        fa.result = d_fit;
        hipLaunchKernelGGL(fit_kernel, dim3(1), dim3(WT), 0, st, fa);
        MIDBF_HIP(hipGetLastError());
        int res[8] = {};
        MIDBF_HIP(hipMemcpyAsync(res, d_fit, sizeof(res), hipMemcpyDeviceToHost, st));
        MIDBF_HIP(hipStreamSynchronize(st));
        if (!res[0]) {
            ++info.rejected_rows;
            continue;
        }
        R.push_back(i);
        shifts.push_back({res[1], res[2], res[3], res[4]});
        if ((int)R.size() == wantR) break;
    }
    MIDBF_CHECK((int)R.size() == wantR, MIDBF_ERR_RECOVERY, "too few rows passed the screening and fit");

    // ---- Alg. 1 inside the accepted samples
    const int nR = (int)R.size(), nC = (int)C.size();
    int* d_piv = b_piv.alloc<int>(2 * MAXS);
    hipLaunchKernelGGL(pivots_kernel, dim3(1), dim3(256), 0, st, (const double*)d_AR, (const long long*)d_C, nR, nC,
                       N, d_piv, d_piv + MAXS);
    MIDBF_HIP(hipGetLastError());
    std::vector<int> piv(2 * MAXS);
    MIDBF_HIP(hipMemcpyAsync(piv.data(), d_piv, piv.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    MIDBF_HIP(hipStreamSynchronize(st));
    std::vector<int> pc(piv.begin(), piv.begin() + nC), pr(piv.begin() + MAXS, piv.begin() + MAXS + nR);
    MIDBF_CHECK(nR >= 2 * r && nC >= 2 * r, MIDBF_ERR_RECOVERY, "too few samples for the rank");
    std::vector<int> It(pr.begin(), pr.begin() + r), Jt(pc.begin(), pc.begin() + r);
    for (int t = 0; t < nR && (int)It.size() < 2 * r; ++t)
        if (std::find(pr.begin(), pr.begin() + r, t) == pr.begin() + r) It.push_back(t);
    for (int t = 0; t < nC && (int)Jt.size() < 2 * r; ++t)
        if (std::find(pc.begin(), pc.begin() + r, t) == pc.begin() + r) Jt.push_back(t);
    std::vector<long long> I(2 * r), J(2 * r);
    for (int a = 0; a < 2 * r; ++a) {
        I[a] = R[It[a]];
        J[a] = C[Jt[a]];
    }
    // index block: [pc r][pr r][It 2r] ints, then [I 2r][J 2r] int64
    int* d_idx = b_idx.alloc<int>(4 * MAXR);
    std::vector<int> hidx(4 * MAXR, 0);
    for (int k = 0; k < r; ++k) {
        hidx[k] = pc[k];
        hidx[MAXR + k] = pr[k];
    }
    for (int a = 0; a < 2 * r; ++a) hidx[2 * MAXR + a] = It[a];
    long long* d_IJ = b_IJ.alloc<long long>(4 * MAXR);
    std::vector<long long> hIJ(4 * MAXR, 0);
    for (int a = 0; a < 2 * r; ++a) {
        hIJ[a] = I[a];
        hIJ[2 * MAXR + a] = J[a];
    }
    MIDBF_HIP(hipMemcpyAsync(d_idx, hidx.data(), hidx.size() * sizeof(int), hipMemcpyHostToDevice, st));
    MIDBF_HIP(hipMemcpyAsync(d_IJ, hIJ.data(), hIJ.size() * sizeof(long long), hipMemcpyHostToDevice, st));
    double* d_Qc = b_Qc.alloc<double>((size_t)r * N);
    double* d_Qr = b_Qr.alloc<double>((size_t)r * N);
    hipLaunchKernelGGL(cgs2_kernel, dim3(1), dim3(WT), 0, st, (const double*)d_AC, (const int*)d_idx, r, N, d_Qc);
    MIDBF_HIP(hipGetLastError());
    hipLaunchKernelGGL(cgs2_kernel, dim3(1), dim3(WT), 0, st, (const double*)d_AR, (const int*)(d_idx + MAXR), r, N,
                       d_Qr);
    MIDBF_HIP(hipGetLastError());
    double* d_core = b_core.alloc<double>(2 * MAXR * MAXR + MAXR);
    CoreArgs ca{};
    ca.Qc = d_Qc;
    ca.Qr = d_Qr;
    ca.AR = d_AR;
    ca.I = d_IJ;
    ca.It = d_idx + 2 * MAXR;
    ca.J = d_IJ + 2 * MAXR;
    ca.r = r;
    ca.N = N;
    ca.UM = d_core;
    ca.VM = d_core + MAXR * MAXR;
    ca.sig = d_core + 2 * MAXR * MAXR;
    hipLaunchKernelGGL(core_kernel, dim3(1), dim3(64), 0, st, ca);
    MIDBF_HIP(hipGetLastError());
    hipLaunchKernelGGL(factors_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, (const double*)d_Qc,
                       (const double*)d_Qr, (const double*)ca.UM, (const double*)ca.VM, (const double*)ca.sig, r, N,
                       U_dev, V_dev);
    MIDBF_HIP(hipGetLastError());
    MIDBF_HIP(hipStreamSynchronize(st));

    info.n_rows = nR;
    info.n_cols = nC;
    for (int a = 0; a < nR && a < PHASE_RECOVER_MAX_SAMPLES; ++a) {
        info.rows[a] = R[a];
        for (int k = 0; k < 4; ++k) info.shift[a][k] = shifts[a][k];
    }
    for (int a = 0; a < nC && a < PHASE_RECOVER_MAX_SAMPLES; ++a) info.cols[a] = C[a];
    if (info_out) *info_out = info;
}

}  // namespace midbf
