// Matrix-core (MFMA) level kernels for many right-hand sides.
#pragma once

#include "apply.h"

namespace midbf {

constexpr int MFMA_NRHS = 64;        // right-hand sides per workgroup
constexpr int MFMA_MIN_NRHS = 16;    // below this the VALU kernels are used
constexpr int MFMA_CROW_MAX = 2048;  // largest candidate vector / middle block side

constexpr int MFMA_VARIANTS = 10;     // tile variants (rows per wave, K chunk, pipelining)

// One matrix-core level kernel.  count = workgroups in x: IDs (up, down),
// groups (down-sum) or middle blocks.  Going down, each ID writes its
// contribution to `scratch` (total_n x nrhs complex64) and the down-sum kernel
// adds the 2^d contributions of every group into the previous level buffer /
// external output.
void launch_mfma_kernel(LevelKernel which, int variant, const void* args, long long count, int nrhs, void* scratch,
                        hipStream_t s);

}  // namespace midbf
