// pca2d.h -- host interface of the 2D-PCA support kernels (pca2d.hip).
#pragma once

#include "common.h"

namespace pj {

// given: subtract `mean` as it is; else compute it first (and write it)
int launch_center(int J, int64_t mn, const float* X, float* mean, float* out, bool given, hipStream_t s);
int launch_symmetrize(int n, float* G, int64_t ld, hipStream_t s);
int launch_sqdist(int T, int J, int64_t d, const float* F, int64_t ldf, const float* Y, int64_t ldy, float* out,
                  int64_t ldo, hipStream_t s);

}  // namespace pj
