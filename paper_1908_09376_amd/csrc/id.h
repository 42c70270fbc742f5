// Batched interpolative decomposition (Sec. 3.2): launch interface.
#pragma once

#include "common.h"

namespace midbf {

constexpr int ID_THREADS = 256;   // one workgroup per decomposition
constexpr int ID_WAVES_PER_SIMD = 4;   // occupancy target: four decompositions per CU hide each other's latency
constexpr int ID_NB = 16;         // pivots per panel
constexpr int ID_ELL = 24;        // sketch rows (panel width + 8 oversampling)
constexpr int ID_NMAX = 2048;     // largest candidate count
constexpr int ID_MMAX = 4096;     // largest sample count

struct IdBatch {
    double2* X;          // decomposition b: X + b*x_stride, m x n row-major (overwritten: R, then T)
    long long x_stride;
    double2* Vw;         // workspace: m x ID_NB per decomposition
    long long v_stride;
    double2* Yw;         // workspace: ID_ELL x n per decomposition
    long long y_stride;
    int* perm;           // output: n column numbers per decomposition, skeleton first
    long long p_stride;
    int* k_out;          // output: rank per decomposition
    const int* n_arr;    // per-decomposition column count (nullptr: n_uniform)
    int n_uniform;
    int m;               // rows (samples), the same for the batch
    double tol;
    int kcap;            // 0: none
    unsigned seed;
    int kfixed;          // > 0: keep exactly min(kfixed, m, n) pivots (the rank rule is not used)
    const int* m_arr;    // per-decomposition count of real sample rows (rows beyond are zero), or null: m
};

void launch_id_batch(const IdBatch& B, int batch, hipStream_t s);

}  // namespace midbf
