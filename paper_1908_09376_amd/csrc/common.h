// Shared definitions of the MIDBF library: complex helpers, error plumbing,
// lattice / Z-order index math.  Host and device.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <stdexcept>
#include <string>

#include "../../include/midbf.h"

namespace midbf {

// ---------------------------------------------------------------- errors ----
struct Error : std::runtime_error {
    midbf_status code;
    Error(midbf_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define MIDBF_HIP(call)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            throw ::midbf::Error(e_ == hipErrorOutOfMemory ? MIDBF_ERR_OOM : MIDBF_ERR_HIP, \
                                 std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

#define MIDBF_CHECK(cond, code, msg)                                                     \
    do {                                                                                 \
        if (!(cond)) throw ::midbf::Error((code), (msg));                                \
    } while (0)

// ------------------------------------------------------------- complex ----
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cmulc(double2 a, double2 b) {  // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double2 cdiv(double2 a, double2 b) {
    double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
// acc += a * b
__host__ __device__ inline void cfma(double2& acc, double2 a, double2 b) {
    acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}
__host__ __device__ inline void cfma(float2& acc, float2 a, float2 b) {
    acc.x = fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x));
    acc.y = fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y));
}
// acc += conj(a) * b
__host__ __device__ inline void cfmac(double2& acc, double2 a, double2 b) {
    acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
}
__host__ __device__ inline void cfmac(float2& acc, float2 a, float2 b) {
    acc.x = fmaf(a.x, b.x, fmaf(a.y, b.y, acc.x));
    acc.y = fmaf(a.x, b.y, fmaf(-a.y, b.x, acc.y));
}

template <class C> struct cplx_traits;
template <> struct cplx_traits<double2> {
    using real = double;
    __host__ __device__ static double2 zero() { return make_double2(0.0, 0.0); }
};
template <> struct cplx_traits<float2> {
    using real = float;
    __host__ __device__ static float2 zero() { return make_float2(0.f, 0.f); }
};
__host__ __device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }

// ---------------------------------------------------------- lattice math ----
// Point number p of a d-dimensional lattice of side n in C order (last
// coordinate fastest) <-> integer coordinates.
__host__ __device__ inline void unravel(long long p, int d, int n, int* a) {
    for (int q = d - 1; q >= 0; --q) {
        a[q] = (int)(p % n);
        p /= n;
    }
}
__host__ __device__ inline long long ravel(const int* a, int d, int n) {
    long long p = 0;
    for (int q = 0; q < d; ++q) p = p * n + a[q];
    return p;
}

// Origin (lattice index units) of node `idx` at tree `level`: the Z-order
// digits of idx, root first; within a digit, coordinate 1 is the most
// significant bit (Sec. 3.1, Fig. 4).
__host__ __device__ inline void node_origin(long long idx, int level, int d, int n, int* origin) {
    for (int q = 0; q < d; ++q) origin[q] = 0;
    const int P = 1 << d;
    for (int j = 0; j < level; ++j) {
        int t = (int)((idx >> (d * (level - 1 - j))) & (P - 1));
        int half = n >> (j + 1);
        for (int q = 0; q < d; ++q) origin[q] += ((t >> (d - 1 - q)) & 1) * half;
    }
}

// Lattice point number of the `local`-th point (local C order) of the box
// with the given origin and side.
__host__ __device__ inline long long box_point(const int* origin, int side, int local, int d, int n) {
    int a[3];
    for (int q = d - 1; q >= 0; --q) {
        a[q] = origin[q] + local % side;
        local /= side;
    }
    return ravel(a, d, n);
}

inline long long ipow(long long b, int e) {
    long long r = 1;
    while (e-- > 0) r *= b;
    return r;
}

}  // namespace midbf
