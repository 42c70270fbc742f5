// Batched FP64 interpolative decomposition by column-pivoted QR (Sec. 3.2,
// rank rule of Sec. 3.5), one workgroup per decomposition.
//
// X (m x n, row-major, in global memory) is factored as
//     X[:, perm] = Q [R11 R12; 0 R22],   T = R11^{-1} R12,
// so that X[:, perm[k:]] ~ X[:, perm[:k]] T.  The rank k is the smallest
// number of pivots after which every remaining column has residual norm
// <= tol * (largest column norm); with one pivot at a time this is the rule
// k = #{j : |R_jj| > tol |R_11|}.
//
// A sample matrix here is several MB of complex FP64 (hundreds of samples x
// hundreds of candidates), far beyond one CU's LDS and registers, so the
// factorization is blocked: pivots are chosen NB at a time by classical
// pivoted QR of a small random sketch Y = Omega X_trail (ELL x columns,
// Omega uniform in [-1, 1) from a counter hash), the chosen columns get an
// unpivoted Householder panel QR, and the rest of the matrix is updated once
// per panel with the block reflector I - V T V^H.  Residual norms used by the
// rank rule are recomputed exactly after every panel.  The matrix is read
// about four times per panel instead of once per pivot.
#include "common.h"
#include "id.h"

namespace midbf {

namespace {

constexpr int NT = ID_THREADS;
constexpr int NW = NT / 64;
constexpr int NB = ID_NB;
constexpr int ELL = ID_ELL;
constexpr int CHUNK = 32;       // rows of V (or of the sketch weights) staged in LDS at a time
constexpr int U = 4;            // rows loaded together per thread (memory-level parallelism)

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Sum over the block; every thread receives the total.
__device__ double block_sum(double v, double* s_red) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += s_red[w];
    return t;
}

__device__ double block_max(double v, double* s_red) {
    v = wave_max(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = s_red[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) t = fmax(t, s_red[w]);
    return t;
}

__device__ int block_max_int(int v, int* s_redi) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_redi[threadIdx.x >> 6] = v;
    __syncthreads();
    int t = s_redi[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) t = max(t, s_redi[w]);
    return t;
}

// Arg-max over the block: the larger value wins, ties go to the smaller index.
__device__ int block_argmax(double v, int idx, double* s_red, int* s_redi) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        double ov = __shfl_xor(v, o, 64);
        int oi = __shfl_xor(idx, o, 64);
        if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) { s_red[threadIdx.x >> 6] = v; s_redi[threadIdx.x >> 6] = idx; }
    __syncthreads();
    double bv = s_red[0];
    int bi = s_redi[0];
#pragma unroll
    for (int w = 1; w < NW; ++w)
        if (s_red[w] > bv || (s_red[w] == bv && s_redi[w] < bi)) { bv = s_red[w]; bi = s_redi[w]; }
    return bi;
}

// splitmix64 finalizer (Steele, Lea, Flood 2014) -> uniform in [-1, 1)
__device__ inline double omega(unsigned seed, int panel, int q, int i) {
    unsigned long long z = ((unsigned long long)seed << 40) ^ ((unsigned long long)(panel & 0xff) << 32) ^
                           ((unsigned long long)q << 24) ^ (unsigned long long)i;
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Householder reflector H = I - tau v v^H with H^H [alpha; x] = [beta; 0],
// beta real, v(0) = 1 (the LAPACK zlarfg convention).  Returns tau and the
// scale 1/(alpha - beta) for the rest of v.
__device__ inline void householder(double2 alpha, double xnorm2, double& beta, double2& tau, double2& scal) {
    if (xnorm2 == 0.0 && alpha.y == 0.0) {
        beta = alpha.x;
        tau = make_double2(0.0, 0.0);
        scal = make_double2(0.0, 0.0);
        return;
    }
    double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xnorm2);
    beta = (alpha.x >= 0.0) ? -nrm : nrm;
    tau = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
    scal = cdiv(make_double2(1.0, 0.0), make_double2(alpha.x - beta, alpha.y));
}

}  // namespace

__global__ __launch_bounds__(NT, ID_WAVES_PER_SIMD) void id_kernel(IdBatch B) {
    const int bid = blockIdx.x;
    const int tid = threadIdx.x;
    const int m = B.m;
    const int n = B.n_arr ? B.n_arr[bid] : B.n_uniform;
    double2* X = B.X + (long long)bid * B.x_stride;
    double2* V = B.Vw + (long long)bid * B.v_stride;
    double2* Y = B.Yw + (long long)bid * B.y_stride;
    int* perm = B.perm + (long long)bid * B.p_stride;

    __shared__ float s_ynrm[ID_NMAX];      // sketch column norms: they only choose pivots
    __shared__ double2 s_stage[CHUNK * NB];
    __shared__ double2 s_T[NB * NB];
    __shared__ double2 s_R11[NB * NB];     // R11 of the panel just factored (upper triangle)
    __shared__ double2 s_S11[NB * NB];     // R11 of the sketch's own QR for the same pivots (upper triangle)
    __shared__ double2 s_red2[NW * 2 * NB];
    __shared__ double2 s_vec[2 * NB];
    __shared__ double2 s_v[ELL];
    __shared__ double s_red[NW];
    __shared__ int s_redi[NW];
    __shared__ int s_swap[NB];
    __shared__ double2 s_tau, s_scal;
    double* s_om = reinterpret_cast<double*>(s_stage);   // ELL x CHUNK sketch block

    if (n <= 0 || m <= 0) {
        if (tid == 0) B.k_out[bid] = 0;
        return;
    }

    // (0) sketch Y = Omega X (ELL x n) and the reference norm (largest column norm); the sketch
    //     rows are formed in two halves (two reads of X, few live accumulators), rows of X are read
    //     U at a time (in-range addresses, padding rows weighted by zero)
    constexpr int EH = ELL / 2;
    double cmax = 0.0;
    for (int c0 = 0; c0 < n; c0 += NT) {
        const int c = c0 + tid;
        const bool act = c < n;
        const int cc = act ? c : n - 1;
        double yn = 0.0;
        for (int h = 0; h < 2; ++h) {
            double2 acc[EH];
#pragma unroll
            for (int q = 0; q < EH; ++q) acc[q] = make_double2(0.0, 0.0);
            double nrm = 0.0;
            for (int i0 = 0; i0 < m; i0 += CHUNK) {
                const int rows = min(CHUNK, m - i0);
                __syncthreads();
                for (int e = tid; e < EH * CHUNK; e += NT) {
                    int q = e / CHUNK, ii = e - q * CHUNK;
                    s_om[e] = (ii < rows) ? omega(B.seed, 0, h * EH + q, i0 + ii) : 0.0;
                }
                __syncthreads();
                for (int ii = 0; ii < rows; ii += U) {
                    double2 x[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) x[u] = X[(long long)(i0 + min(ii + u, rows - 1)) * n + cc];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        nrm += (ii + u < rows) ? cabs2(x[u]) : 0.0;
#pragma unroll
                        for (int q = 0; q < EH; ++q) {
                            const double w = s_om[q * CHUNK + ii + u];
                            acc[q].x = fma(w, x[u].x, acc[q].x);
                            acc[q].y = fma(w, x[u].y, acc[q].y);
                        }
                    }
                }
            }
            if (act) {
#pragma unroll
                for (int q = 0; q < EH; ++q) {
                    Y[(long long)(h * EH + q) * n + c] = acc[q];
                    yn += cabs2(acc[q]);
                }
                if (h == 0) {
                    perm[c] = c;
                    cmax = fmax(cmax, nrm);
                }
            }
        }
        if (act) s_ynrm[c] = (float)yn;
    }
    const double ref2 = block_max(cmax, s_red);
    if (ref2 == 0.0) {
        if (tid == 0) B.k_out[bid] = 0;
        return;
    }
    const double thresh2 = B.tol * B.tol * ref2;
    // the fixed-rank variant factors exactly kstop pivots; the adaptive one stops by the rank rule.
    // Rows past a decomposition's own sample count are zero and add no rank.
    const int mn = min(B.m_arr ? min(B.m_arr[bid], m) : m, n);
    const int kstop = B.kfixed > 0 ? min(B.kfixed, mn) : mn;

    int k = -1, j0 = 0;
    while (k < 0 && j0 < kstop) {
        const int nbp = min(NB, kstop - j0);

        // (1) classical pivoted QR of the sketch of the trailing columns: choose nbp pivots
        for (int jj = 0; jj < nbp; ++jj) {
            const int col = j0 + jj;
            double bv = -1.0;
            int bi = col;                   // a valid column whatever the norms hold
            for (int c = col + tid; c < n; c += NT) {
                double v = (double)s_ynrm[c];
                if (v > bv) { bv = v; bi = c; }
            }
            const int p = block_argmax(bv, bi, s_red, s_redi);
            if (tid == 0) s_swap[jj] = p;
            if (p != col) {
                if (tid < ELL) {
                    double2 t = Y[(long long)tid * n + col];
                    Y[(long long)tid * n + col] = Y[(long long)tid * n + p];
                    Y[(long long)tid * n + p] = t;
                }
                if (tid == 0) { float t = s_ynrm[col]; s_ynrm[col] = s_ynrm[p]; s_ynrm[p] = t; }
            }
            __syncthreads();
            if (tid < 64) {
                const int q = tid;
                double2 yq = (q >= jj && q < ELL) ? Y[(long long)q * n + col] : make_double2(0.0, 0.0);
                double xs = wave_sum((q > jj && q < ELL) ? cabs2(yq) : 0.0);
                double2 alpha = make_double2(__shfl(yq.x, jj, 64), __shfl(yq.y, jj, 64));
                double beta;
                double2 tau, scal;
                householder(alpha, xs, beta, tau, scal);
                if (q < ELL) s_v[q] = (q < jj) ? make_double2(0.0, 0.0) : (q == jj ? make_double2(1.0, 0.0) : cmul(yq, scal));
                if (q == 0) s_tau = tau;
                if (q == jj) Y[(long long)q * n + col] = make_double2(beta, 0.0);
            }
            __syncthreads();
            const double2 ctau = cconj(s_tau);
            for (int c = col + 1 + tid; c < n; c += NT) {
                double2 w = make_double2(0.0, 0.0);
#pragma unroll 4
                for (int q = jj; q < ELL; ++q) cfmac(w, s_v[q], Y[(long long)q * n + c]);
                const double2 cw = cmul(ctau, w);
                double yn = 0.0;
#pragma unroll 4
                for (int q = jj; q < ELL; ++q) {
                    const double2 y = csub(Y[(long long)q * n + c], cmul(s_v[q], cw));
                    Y[(long long)q * n + c] = y;
                    if (q > jj) yn += cabs2(y);
                }
                s_ynrm[c] = (float)yn;
            }
            __syncthreads();
        }
        // the sketch's R11 for these pivots
        for (int e = tid; e < NB * NB; e += NT) {
            const int q = e / NB, jj = e - q * NB;
            s_S11[e] = (q <= jj && jj < nbp) ? Y[(long long)q * n + j0 + jj] : make_double2(0.0, 0.0);
        }

        // (2) move the chosen columns to the front of the trailing block
        for (int i = tid; i < m; i += NT) {
            double2* row = X + (long long)i * n;
            for (int jj = 0; jj < nbp; ++jj) {
                const int a = j0 + jj, b = s_swap[jj];
                if (a != b) { double2 t = row[a]; row[a] = row[b]; row[b] = t; }
            }
        }
        if (tid == 0) {
            for (int jj = 0; jj < nbp; ++jj) {
                const int a = j0 + jj, b = s_swap[jj];
                if (a != b) { int t = perm[a]; perm[a] = perm[b]; perm[b] = t; }
            }
        }
        __syncthreads();

        // (3) unpivoted Householder QR of the panel X[j0:m, j0:j0+nbp]
        for (int jj = 0; jj < nbp; ++jj) {
            const int col = j0 + jj;
            double xs = 0.0;
            for (int i = col + 1 + tid; i < m; i += NT) xs += cabs2(X[(long long)i * n + col]);
            xs = block_sum(xs, s_red);
            if (tid == 0) {
                double2 alpha = X[(long long)col * n + col];
                double beta;
                double2 tau, scal;
                householder(alpha, xs, beta, tau, scal);
                s_tau = tau;
                s_scal = scal;
                X[(long long)col * n + col] = make_double2(beta, 0.0);
            }
            __syncthreads();
            const double2 scal = s_scal;
            for (int i = j0 + tid; i < m; i += NT) {
                double2 v;
                if (i < col) v = make_double2(0.0, 0.0);
                else if (i == col) v = make_double2(1.0, 0.0);
                else {
                    v = cmul(X[(long long)i * n + col], scal);
                    X[(long long)i * n + col] = make_double2(0.0, 0.0);
                }
                V[(long long)i * NB + jj] = v;
            }
            __syncthreads();
            // w_c = v^H X[:, c] for the panel columns right of col, z_q = V[:, q]^H v for q < jj:
            // thread (g, o) sums output o over the rows col + g + 8 r (one accumulator per thread)
            const int ncw = j0 + nbp - col - 1;
            {
                const int o = tid & (2 * NB - 1), g = tid >> 5;
                const bool wcol = o < NB;
                const bool useful = wcol ? (o < ncw) : (o - NB < jj);
                const long long off = wcol ? (long long)(col + 1 + o) : (long long)(o - NB);
                constexpr int RS = NT / (2 * NB);
                double2 acc = make_double2(0.0, 0.0);
                if (useful) {       // every address below is in range: o < ncw, or o - NB < jj
                    for (int i0 = col + g; i0 < m; i0 += 4 * RS) {
                        double2 vv[4], xx[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int i = min(i0 + u * RS, m - 1);
                            vv[u] = V[(long long)i * NB + jj];
                            xx[u] = wcol ? X[(long long)i * n + off] : V[(long long)i * NB + off];
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if (i0 + u * RS < m) {
                                if (wcol) cfmac(acc, vv[u], xx[u]);
                                else cfmac(acc, xx[u], vv[u]);
                            }
                        }
                    }
                }
                acc.x += __shfl_xor(acc.x, 2 * NB, 64);
                acc.y += __shfl_xor(acc.y, 2 * NB, 64);
                if ((tid & 63) < 2 * NB) s_red2[(tid >> 6) * 2 * NB + o] = acc;
            }
            __syncthreads();
            if (tid < 2 * NB) {
                double2 t = make_double2(0.0, 0.0);
                for (int w = 0; w < NW; ++w) t = cadd(t, s_red2[w * 2 * NB + tid]);
                s_vec[tid] = t;
            }
            __syncthreads();
            if (tid < NB) {            // column jj of T: thread q computes entry q
                const int q = tid;
                const double2 tau = s_tau;
                double2 t = make_double2(0.0, 0.0);
                for (int l = q; l < jj; ++l) cfma(t, s_T[q * NB + l], s_vec[NB + l]);
                s_T[q * NB + jj] = q < jj ? cmul(make_double2(-tau.x, -tau.y), t)
                                          : (q == jj ? tau : make_double2(0.0, 0.0));
            }
            const double2 ctau = cconj(s_tau);
            if (ncw > 0) {
                // thread (column, row) pairs, four rows per thread loaded together
                const int cc = tid % NB;
                const double2 coef = cmul(ctau, s_vec[min(cc, ncw - 1)]);
                const int total = m - col;
                for (int r0 = tid / NB; r0 < total; r0 += 4 * (NT / NB)) {
                    double2 xv[4], vv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int i = col + min(r0 + u * (NT / NB), total - 1);
                        xv[u] = X[(long long)i * n + col + 1 + min(cc, ncw - 1)];
                        vv[u] = V[(long long)i * NB + jj];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (cc < ncw && r0 + u * (NT / NB) < total)
                            X[(long long)(col + r0 + u * (NT / NB)) * n + col + 1 + cc] = csub(xv[u], cmul(vv[u], coef));
                }
            }
            __syncthreads();
        }
        // the panel's R11
        for (int e = tid; e < NB * NB; e += NT) {
            const int u = e / NB, v = e - u * NB;
            s_R11[e] = (u <= v && v < nbp) ? X[(long long)(j0 + u) * n + j0 + v] : make_double2(0.0, 0.0);
        }

        // (4) trailing update X[j0:m, j0+nbp:n] <- (I - V T V^H)^H X with exact residual norms, the
        //     first pivot count of this panel that satisfies the rank rule, and the sketch of the new
        //     trailing block from the old one: [S12 - S11 R11^{-1} R12; S22] (Duersch and Gu's update),
        //     so no pass over X is spent on sketching after the first panel
        int fmax = 0;
        for (int c0 = j0 + nbp; c0 < n; c0 += NT) {
            const int c = c0 + tid;
            const bool act = c < n;
            const int cc = act ? c : n - 1;
            double2 W[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) W[q] = make_double2(0.0, 0.0);
            for (int i0 = j0; i0 < m; i0 += CHUNK) {
                const int rows = min(CHUNK, m - i0);
                __syncthreads();
                for (int e = tid; e < CHUNK * NB; e += NT) {
                    int ii = e / NB, q = e - ii * NB;
                    s_stage[e] = (ii < rows && q < nbp) ? V[(long long)(i0 + ii) * NB + q] : make_double2(0.0, 0.0);
                }
                __syncthreads();
                for (int ii = 0; ii < rows; ii += U) {
                    double2 x[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) x[u] = X[(long long)(i0 + min(ii + u, rows - 1)) * n + cc];
#pragma unroll
                    for (int u = 0; u < U; ++u)
#pragma unroll
                        for (int q = 0; q < NB; ++q) cfmac(W[q], s_stage[(ii + u) * NB + q], x[u]);
                }
            }
            // W <- T^H W in place (row q needs rows l <= q, so go from the last row up)
#pragma unroll
            for (int q = NB - 1; q >= 0; --q) {
                double2 t = make_double2(0.0, 0.0);
#pragma unroll
                for (int l = 0; l <= q; ++l) cfmac(t, s_T[l * NB + q], W[l]);
                W[q] = t;
            }
            double nn = 0.0;
            for (int i0 = j0; i0 < m; i0 += CHUNK) {
                const int rows = min(CHUNK, m - i0);
                __syncthreads();
                for (int e = tid; e < CHUNK * NB; e += NT) {
                    int ii = e / NB, q = e - ii * NB;
                    s_stage[e] = (ii < rows && q < nbp) ? V[(long long)(i0 + ii) * NB + q] : make_double2(0.0, 0.0);
                }
                __syncthreads();
                // rows j0 .. j0+nbp become R12 and stay out of the residual norm
                const int skip = i0 == j0 ? nbp : 0;
                for (int ii = 0; ii < rows; ii += U) {
                    double2 x[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) x[u] = X[(long long)(i0 + min(ii + u, rows - 1)) * n + cc];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
#pragma unroll
                        for (int q = 0; q < NB; ++q) x[u] = csub(x[u], cmul(s_stage[(ii + u) * NB + q], W[q]));
                        if (act && ii + u < rows) {
                            X[(long long)(i0 + ii + u) * n + c] = x[u];
                            if (ii + u >= skip) nn += cabs2(x[u]);
                        }
                    }
                }
            }
            double2 r12[NB];        // R12 of this column (rows j0 .. j0+nbp, written above by this thread)
#pragma unroll
            for (int u = 0; u < NB; ++u)
                r12[u] = (act && u < nbp) ? X[(long long)(j0 + u) * n + c] : make_double2(0.0, 0.0);
            if (act) {
                double res = nn;
                int f = nbp;
#pragma unroll
                for (int jj = NB - 1; jj >= 0; --jj) {
                    if (jj < nbp) {
                        if (res <= thresh2) f = jj; else break;
                        res += cabs2(r12[jj]);
                    }
                }
                fmax = max(fmax, f);
                // z = R11^{-1} R12 (in r12), then the sketch rows 0..nbp of this column lose S11 z
#pragma unroll
                for (int u = NB - 1; u >= 0; --u) {
                    if (u < nbp) {
                        double2 t = r12[u];
#pragma unroll
                        for (int v = u + 1; v < NB; ++v)
                            if (v < nbp) t = csub(t, cmul(s_R11[u * NB + v], r12[v]));
                        const double d = s_R11[u * NB + u].x;
                        r12[u] = d != 0.0 ? make_double2(t.x / d, t.y / d) : make_double2(0.0, 0.0);
                    }
                }
                double yn = 0.0;
#pragma unroll
                for (int q = 0; q < ELL; ++q) {
                    double2 y = Y[(long long)q * n + c];
                    if (q < nbp) {
#pragma unroll
                        for (int u = 0; u < NB; ++u)
                            if (u >= q && u < nbp) y = csub(y, cmul(s_S11[q * NB + u], r12[u]));
                        Y[(long long)q * n + c] = y;
                    }
                    yn += cabs2(y);
                }
                s_ynrm[c] = (float)yn;
            }
        }
        // panel columns: column j0+cc is excluded once cc pivots are taken
        if (tid < nbp) {
            const int cc = tid, c = j0 + cc;
            int f = cc;
            double res = 0.0;
            for (int jj = cc - 1; jj >= 0; --jj) {
                res += cabs2(X[(long long)(j0 + jj + 1) * n + c]);
                if (res <= thresh2) f = jj; else break;
            }
            fmax = max(fmax, f);
        }
        const int F = block_max_int(fmax, s_redi);
        if (B.kfixed <= 0 && F < nbp) k = j0 + F + 1;
        j0 += nbp;
    }
    if (k < 0) k = kstop;
    if (B.kcap > 0 && k > B.kcap) k = B.kcap;
    __syncthreads();

    // (5) T = R11^{-1} R12 in place over X[0:k, k:n] (back substitution, one column per thread)
    for (int c0 = k; c0 < n; c0 += NT) {
        const int c = c0 + tid;
        const bool act = c < n;
        for (int i = k - 1; i >= 0; --i) {
            if (act) {
                const double2* ri = X + (long long)i * n;
                double2 acc = ri[c];
                for (int l = i + 1; l < k; ++l) acc = csub(acc, cmul(ri[l], X[(long long)l * n + c]));
                X[(long long)i * n + c] = cdiv(acc, ri[i]);
            }
        }
    }
    if (tid == 0) B.k_out[bid] = k;
}

void launch_id_batch(const IdBatch& B, int batch, hipStream_t s) {
    if (batch <= 0) return;
    hipLaunchKernelGGL(id_kernel, dim3(batch), dim3(NT), 0, s, B);
    MIDBF_HIP(hipGetLastError());
}

}  // namespace midbf
