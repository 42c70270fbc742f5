// Phase recovery entry (host): see phase_recover in include/midbf.h.
#pragma once

#include "common.h"

namespace midbf {

// Npts > 0: scattered points, X1 and X2 the host x and xi coordinates (Npts x d);
// 0: the lattices of side n.
void phase_recover_run(int d, int n, const double* X1, const double* X2, midbf_sample_cb cb, void* user, int r,
                       int q, double tau, uint64_t seed, hipStream_t st, double* U_dev, double* V_dev,
                       phase_recover_info* info, long long Npts = 0);
// The recovery path of a scattered point set (Alg. 5): P_out gets (N - 1) x 2 rows (pred, node).
void recovery_path_points(const double* pts, long long N, int d, long long root, int* P_out, hipStream_t st);

}  // namespace midbf
