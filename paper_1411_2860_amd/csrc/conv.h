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
    bool half_m;       // row tile halved (too few tiles for the chip otherwise)
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
    const float* CT;      // C^T[l][t] = C[t][l]
    float* y;
    void* ws;
    int64_t period = 0;   // > 0: s is periodic with this period (a multiple of L); W is then the
                          // length of the periodic extension that the outputs read
};
int launch_conv(const ConvArgs& a, hipStream_t s);
// Step 1 alone: sc[l][i] = sum_t s[iL + t] C[t, l] for l < r, i < nbp (zero past
// the signal), rows of length nbp.
int launch_conv_signal_rows(const ConvArgs& a, float* sc, int64_t nbp, hipStream_t s);

// The same full-rate result through F-point FFTs (fft.hip): overlap-save
// segments of P = F - T + 1 output rows, T = (N + L - 2) / L + 1 taps per phase.
struct ConvFftGeom {
    int64_t nout, rows, T;
    int F, logF;
    int64_t P, nseg, nbp;
    bool ok;                 // T fits the largest transform with P >= 1
    int64_t sc_bytes, tw_bytes, hf_bytes, sf_bytes, yf_bytes, total;
};
ConvFftGeom conv_fft_geom(int64_t W, int64_t N, int L, int r);
int launch_conv_fft(const ConvArgs& a, hipStream_t s);
bool conv_prefers_fft(int64_t W, int64_t N, int L, int r);   // the choice proj_conv1d makes

// Block rate: outputs at m = aL only (nd of them), the rest interpolated.
enum BlockForm {
    BF_SMALL = 0,      // L <= 8: one launch, projections inside the workgroups
    BF_PROJECTED = 1,  // channels = the r projected signal rows, taps = D-projected kernel blocks
    BF_DIRECT = 2      // channels = the L polyphase rows of the raw signal, taps = Q_r-reconstructed kernel blocks
};
struct ConvBlockGeom {
    int64_t nout;      // W - N + 1 outputs
    int64_t nd;        // computed outputs a = 0 .. nd - 1 (m = aL <= W - N)
    int64_t ncb;       // aligned kernel blocks ceil(N / L)
    int64_t ntp;       // taps per channel padded to 8
    int64_t nbp;       // length of each projected-signal row (>= nd + ncb)
    int form;          // BlockForm
    int nch;           // channels (r or L)
    int nsplit;        // channel ranges contracted by separate workgroups
    int64_t sc_bytes, h_bytes, part_bytes, total;
};
ConvBlockGeom conv_block_geom(int64_t W, int64_t N, int L, int r);
int launch_conv_block(const ConvArgs& a, hipStream_t s);

// ---- vector-ALU reduced cross-correlation (corr.hip) ----------------------
// Blocks of at most 8 samples, both rates, in one launch: rows a < nrows of
//   Y[a, p] = sum_{l<r} sum_{c<ntap} sc_l[a + c] kd_l[cL - p]
// with both projections computed in the workgroups; full rate writes
// y[aL + p] (p < L), block rate y[aL] = Y[a, 0] and interpolates between.
struct CorrSmallArgs {
    const float* s; int64_t W; int64_t period;   // signal (periodic when period > 0)
    const float* k; int64_t N; int reverse;
    int L, r;
    const float* C; const float* DT;
    int64_t nrows, ntap, nout;
    float* y;
    int block;
};
int launch_corr_small(const CorrSmallArgs& a, hipStream_t s);
int corr_small_max_L();
int corr_rows_per_tile();

// Block rate, longer blocks: yd[a] = sum_ch sum_c X(ch, a + c) H(ch, c),
// X from channel rows (src 0: x[ch * xld + i], i < xn) or from the polyphase
// rows of the raw signal (src 1: x[i L + ch], i L + ch < xn); channel ranges
// over grid.y with partials summed by a second launch, then interpolated.
struct CorrBlockArgs {
    const float* x; int64_t xld, xn; int L;
    int nch;
    const float* h; int64_t hld;     // H(ch, c) = h[ch * hld + c], hld a multiple of 8
    int64_t nd, nout;
    int nsplit;
    float* part;                     // nsplit x nd (nsplit > 1)
    float* y;
};
int launch_corr_block(const CorrBlockArgs& a, int src, hipStream_t s);
// Kernel-side taps of the block rate (L <= 256), on aligned kernel blocks
// c < hld, zero for c >= ncb: launch_kblock_taps writes h[l hld + c] =
// sum_u D[l, u] k'(cL + u) for l < r; launch_ktilde writes those into kd
// (r x hld) and then h[t hld + c] = sum_{l<r} C[t, l] kd[l hld + c] for t < L.
int launch_ktilde(const float* k, int64_t N, int reverse, int L, int r, int64_t ncb, const float* CT, const float* DT,
                  float* kd, float* h, int64_t hld, hipStream_t s);
int launch_kblock_taps(const float* k, int64_t N, int reverse, int L, int r, int64_t ncb, int64_t hld,
                       const float* DT, float* h, hipStream_t s);

}  // namespace pj
