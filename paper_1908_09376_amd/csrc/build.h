// Factor construction entry points (host).
#pragma once

#include "plan.h"

namespace midbf {

// replay_file: internal; null builds from samples, else the decompositions come from a factor file
midbf_plan* build_plan(const midbf_params& p, hipStream_t st, void* replay_file = nullptr);
// The factorization as a file (needs the FP64 copy) and back, with the given precisions kept.
void save_plan(midbf_plan* h, const char* path, hipStream_t st);
midbf_plan* load_plan(const char* path, unsigned precisions, hipStream_t st, midbf_params* params_out);
void destroy_plan(midbf_plan* h);
void kernel_entries(const midbf_params& p, const int* rows, int nrows, const int* cols, int ncols, void* out,
                    hipStream_t st);
void id_batch(void* X, int batch, int m, int n, double tol, int kcap, int* k_out, int* perm_out, void* T_out,
              hipStream_t st);

}  // namespace midbf
