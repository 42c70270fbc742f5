// Factor construction entry points (host).
#pragma once

#include "plan.h"

namespace midbf {

midbf_plan* build_plan(const midbf_params& p, hipStream_t st);
void destroy_plan(midbf_plan* h);
void kernel_entries(const midbf_params& p, const int* rows, int nrows, const int* cols, int ncols, void* out,
                    hipStream_t st);
void id_batch(void* X, int batch, int m, int n, double tol, int kcap, int* k_out, int* perm_out, void* T_out,
              hipStream_t st);

}  // namespace midbf
