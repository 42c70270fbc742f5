// Phase recovery entry (host): see phase_recover in include/midbf.h.
#pragma once

#include "common.h"

namespace midbf {

void phase_recover_run(int d, int n, const double* X1, const double* X2, midbf_sample_cb cb, void* user, int r,
                       int q, double tau, uint64_t seed, hipStream_t st, double* U_dev, double* V_dev,
                       phase_recover_info* info);

}  // namespace midbf
