// moments.h -- host interface of the block second-moment kernel (moments.hip).
#pragma once

#include <algorithm>

#include "common.h"

namespace pj {

struct MomentsGeom {
    int64_t G;         // blocks per row, ceil(K / L)
    int64_t nblk;      // rows * G
    int ntile;         // 64 x 64 tiles per side of M
    int nchunk;        // contiguous block ranges summed separately
    int64_t chunk;     // blocks per range
    int64_t ws_bytes;  // FP64 partials (0 with one range)
};
MomentsGeom moments_geom(int64_t rows, int64_t K, int L);
int launch_moments(const float* X, int64_t ld, int64_t rows, int64_t K, int L, double* M, void* ws, hipStream_t st);

}  // namespace pj
