// conv.h -- host interface of the projected cross-correlation kernels
// (conv.hip): workspace geometry and launch arguments.
#pragma once

#include "common.h"

namespace pj {

// Projected cross-correlation (conv.hip).
struct ConvGeom {
    int64_t nout;      // W - N + 1 valid outputs
    int64_t nc, ncp;   // kernel phases per projection (N + L - 2) / L + 1, padded to 4
    int64_t rows;      // output rows a (outputs m = a L + b)
    int64_t tiles_m;   // row tiles of the reduced cross-correlation
    int64_t nbp;       // length of each projected-signal row
    int64_t k_nrb, k_nkb;
    int64_t tiles_n;   // column tiles (phases b)
    int nsplit;        // contiguous projection ranges contracted by separate workgroups
    bool small;        // L <= kSmallL: vector-ALU path (kernel phases in plain layout)
    int64_t sc_bytes, k_bytes, part_bytes, total;
};
ConvGeom conv_geom(int64_t W, int64_t N, int L, int r);

struct ConvArgs {
    const float* s; int64_t W;
    const float* k; int64_t N;
    int reverse;          // 1: convolution (kernel reversed), 0: cross-correlation
    int L, r;
    const float* C;       // C[t][l]
    const float* DT;      // D^T[u][l] = D[l][u]
    float* y;
    void* ws;
    int64_t period = 0;   // > 0: s is periodic with this period (a multiple of L); W is then the
                          // length of the periodic extension that the outputs read
};
int launch_conv(const ConvArgs& a, hipStream_t s);

// Block rate: outputs at m = aL only (nd of them), the rest interpolated.
struct ConvBlockGeom {
    int64_t nout;      // W - N + 1 outputs
    int64_t nd;        // computed outputs a = 0 .. nd - 1 (m = aL <= W - N)
    int64_t ncb;       // aligned kernel blocks ceil(N / L)
    int64_t nbp;       // length of each projected-signal row (>= nd + ncb)
    int64_t sc_bytes, kd_bytes, yd_bytes, total;
};
ConvBlockGeom conv_block_geom(int64_t W, int64_t N, int L, int r);
int launch_conv_block(const ConvArgs& a, hipStream_t s);

}  // namespace pj
