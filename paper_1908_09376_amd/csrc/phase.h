// Kernel entries K(x, xi) = exp(2 pi i Phi(x, xi)) evaluated in FP64 on the
// device (Scenario 1 of Table 1; Sec. 3 preamble).  Phi is reduced mod 1
// before the exponential: the x . xi part exactly in integers (x = a/n and
// xi = b - n/2 make n * x . xi an integer), the smooth part in FP64.
#pragma once

#include "common.h"

namespace midbf {

struct PhaseDesc {
    int kind;             // midbf_phase_kind
    int d, n;
    const double* U;      // MIDBF_PHASE_LOWRANK: N x r row-major
    const double* V;
    int r;
    const double* xp;     // scattered points: x and xi coordinates (N x d row-major), or null
    const double* wp;
    double hh;            // MIDBF_PHASE_HELMHOLTZ: h
    int transpose;        // nonzero: the kernel of K^H, conj(K(x_q, xi_p)) (rows p are xi points)
};

// Smooth (non-bilinear) part of the phase at x = a/n, xi = b - n/2.
__device__ inline double phase_smooth(const PhaseDesc& ph, const int* a, const int* b) {
    const double inv_n = 1.0 / ph.n;
    const int h = ph.n / 2;
    switch (ph.kind) {
        case MIDBF_PHASE_FIO_ELLIPSE: {
            // Section 4, Example 1
            double x1 = a[0] * inv_n, x2 = a[1] * inv_n;
            double xi1 = b[0] - h, xi2 = b[1] - h;
            double c1 = (2.0 + sinpi(2.0 * x1) * sinpi(2.0 * x2)) * (1.0 / 16.0);
            double c2 = (2.0 + cospi(2.0 * x1) * cospi(2.0 * x2)) * (1.0 / 16.0);
            return sqrt(c1 * c1 * xi1 * xi1 + c2 * c2 * xi2 * xi2);
        }
        case MIDBF_PHASE_FIO_PIECEWISE: {
            double x1 = a[0] * inv_n, x2 = a[1] * inv_n;
            double xi1 = b[0] - h, xi2 = b[1] - h;
            double c = (x1 < 0.5) ? (2.0 + sinpi(2.0 * x1)) * (1.0 / 16.0)
                                  : (3.0 + cospi(2.0 * x2)) * (1.0 / 16.0);
            return c * sqrt(xi1 * xi1 + xi2 * xi2);
        }
        case MIDBF_PHASE_ISO3D: {
            double s = 1.0, r2 = 0.0;
            for (int q = 0; q < 3; ++q) {
                s *= sinpi(2.0 * a[q] * inv_n);
                double xq = b[q] - h;
                r2 += xq * xq;
            }
            return (3.0 + s) * (1.0 / 100.0) * sqrt(r2);
        }
        default:
            return 0.0;
    }
}

// frac(Phi(x_p, xi_q)) in [0, 1) for point numbers p (x side), q (xi side).
__device__ inline double phase_frac_xxi(const PhaseDesc& ph, long long p, long long q) {
    if (ph.kind == MIDBF_PHASE_LOWRANK) {
        const double* u = ph.U + p * ph.r;
        const double* v = ph.V + q * ph.r;
        double s = 0.0;
        for (int l = 0; l < ph.r; ++l) s = fma(u[l], v[l], s);
        return s - floor(s);
    }
    if (ph.xp) {            // given point sets, in FP64: Phi = x . xi, or h |x - xi|
        const double* x = ph.xp + p * ph.d;
        const double* w = ph.wp + q * ph.d;
        double s = 0.0;
        if (ph.kind == MIDBF_PHASE_HELMHOLTZ) {
            for (int l = 0; l < ph.d; ++l) {
                const double dl = x[l] - w[l];
                s = fma(dl, dl, s);
            }
            s = ph.hh * sqrt(s);
        } else {
            for (int l = 0; l < ph.d; ++l) s = fma(x[l], w[l], s);
        }
        return s - floor(s);
    }
    int a[3], b[3];
    unravel(p, ph.d, ph.n, a);
    unravel(q, ph.d, ph.n, b);
    const int h = ph.n / 2;
    long long dot = 0;
    for (int l = 0; l < ph.d; ++l) dot += (long long)a[l] * (long long)(b[l] - h);
    long long md = dot % ph.n;
    if (md < 0) md += ph.n;
    double t = (double)md / (double)ph.n + phase_smooth(ph, a, b);
    return t - floor(t);
}

// The phase of entry (p, q) of the factored kernel, as frac in [0, 1): Phi(x_p, xi_q), or for
// K^H the phase of conj(K(x_q, xi_p)), frac(-Phi(x_q, xi_p)).
__device__ inline double phase_frac(const PhaseDesc& ph, long long p, long long q) {
    if (!ph.transpose) return phase_frac_xxi(ph, p, q);
    const double f = phase_frac_xxi(ph, q, p);
    return f > 0.0 ? 1.0 - f : 0.0;
}

__device__ inline double2 kernel_entry(const PhaseDesc& ph, long long p, long long q) {
    double fr = phase_frac(ph, p, q);
    double s, c;
    sincospi(2.0 * fr, &s, &c);
    return make_double2(c, s);
}

}  // namespace midbf
