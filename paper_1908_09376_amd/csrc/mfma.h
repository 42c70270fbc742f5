// Matrix-core (MFMA) level kernels for many right-hand sides.
#pragma once

#include "apply.h"

namespace midbf {

constexpr int MFMA_NRHS = 64;        // right-hand sides per workgroup
constexpr int MFMA_MIN_NRHS = 16;    // below this the VALU kernels are used
constexpr int MFMA_CROW_MAX = 2048;  // largest candidate vector / middle block side

// count = grid size in x: IDs (up), groups (down) or middle blocks.
void launch_mfma_kernel(LevelKernel which, const void* args, long long count, int nrhs, hipStream_t s);

// Going down: per-ID contributions into `scratch` (total_n x nrhs complex64),
// then the per-group sums into the previous level buffer / external output.
void launch_mfma_down(const DownArgs& a, long long nid, long long groups, void* scratch, hipStream_t s);

}  // namespace midbf
