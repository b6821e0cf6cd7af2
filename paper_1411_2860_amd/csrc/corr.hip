// corr.hip -- the reduced cross-correlation as a sum of short stride-1
// correlations on the vector ALUs (paper Sec. III-A eq. (10)-(14): after the
// projection each of the r channels is a down-sampled signal correlated with
// a down-sampled kernel, and the r results are accumulated).
//
// Every output row a of a tile accumulates
//     Y[a, p] = sum_ch sum_c X(ch, a + c) H(p, ch, c)
// over its channels ch and taps c, for NPH phases p.  Two uses:
//   * blocks of at most 8 samples (both output rates): X(l, i) = sc_l[i] is
//     the projected signal and H(p, l, c) = kd_l[cL - p] the kernel projected
//     at phase p; y[aL + p] = Y[a, p] (full rate, NPH = L) or y[aL] = Y[a, 0]
//     with the outputs between two aligned lags interpolated (block rate).
//     Both projections are computed inside the workgroup from the raw
//     signal and kernel, so the whole call is one launch.
//   * the block rate for longer blocks (NPH = 1), where either X is the
//     projected signal and H the aligned kernel blocks projected with D, or,
//     when that is cheaper, X(t, i) = s[iL + t] (the raw signal split into its
//     L polyphase channels) and H(t, c) = (Q_r k_c)[t], the aligned kernel
//     blocks reconstructed from their first r projections.  Both evaluate
//       y[aL] = sum_c sum_t s[(a + c)L + t] sum_l C[t, l] sum_u D[l, u] k[cL + u],
//     grouped as (s C)(D k) or s (C D k); the second needs no projection of
//     the signal and L instead of r channels.
//
// A workgroup (4 waves) owns 512 consecutive rows; lane j of a wave owns rows
// 8j .. 8j + 7 and slides a 16-value window of X along the taps, so every
// pair of 16-byte LDS reads feeds 64 FMAs per phase.  The waves share the
// channels (or, with fewer than 4 channels, the taps) of each staged tile and
// their sums are added in a fixed order at the end.
#include <algorithm>

#include "conv.h"

namespace pj {

namespace {

constexpr int kOPT = 8;            // consecutive output rows per lane
constexpr int kTA = 64 * kOPT;     // output rows per workgroup
constexpr int kCT = 256;           // threads per workgroup
constexpr int kBlockTC = 128;      // taps per staged tile, block rate
constexpr int kBlockCH = 8;        // channels per staged tile, block rate

// Accumulates taps [cb, ce) (multiples of 8) of one channel into the lane's
// kOPT rows for NPH phases.  xw[i] = X(ch, row0 + i) of the staged window
// (the lane's rows start at i = 8 lane), hw[p * hps + c] = H(p, ch, c0 + c).
template <int NPH>
__device__ __forceinline__ void corr_taps(const float* __restrict__ xw, const float* __restrict__ hw, int hps, int cb,
                                          int ce, int lane, float (&acc)[NPH][kOPT])
{
    const float* xl = xw + kOPT * lane;
    f32x4 w0 = *reinterpret_cast<const f32x4*>(xl + cb);
    f32x4 w1 = *reinterpret_cast<const f32x4*>(xl + cb + 4);
    for (int c = cb; c < ce; c += 8) {
        const f32x4 w2 = *reinterpret_cast<const f32x4*>(xl + c + 8);
        const f32x4 w3 = *reinterpret_cast<const f32x4*>(xl + c + 12);
        const float w[16] = {w0[0], w0[1], w0[2], w0[3], w1[0], w1[1], w1[2], w1[3],
                             w2[0], w2[1], w2[2], w2[3], w3[0], w3[1], w3[2], w3[3]};
#pragma unroll
        for (int p = 0; p < NPH; ++p) {
            const f32x4 h0 = *reinterpret_cast<const f32x4*>(hw + p * hps + c);
            const f32x4 h1 = *reinterpret_cast<const f32x4*>(hw + p * hps + c + 4);
            const float h[8] = {h0[0], h0[1], h0[2], h0[3], h1[0], h1[1], h1[2], h1[3]};
#pragma unroll
            for (int e = 0; e < 8; ++e)
#pragma unroll
                for (int o = 0; o < kOPT; ++o) acc[p][o] = fmaf(w[o + e], h[e], acc[p][o]);
        }
        w0 = w2;
        w1 = w3;
    }
}

// The share of a staged tile (nch channels, taps [0, ntc)) that wave w
// contracts: with at least 4 channels the waves take channels w, w + 4, ...
// from the highest down (small high-order terms first), all taps; otherwise
// every wave takes every channel and a quarter of the taps.
struct Share {
    bool by_channel;
    int cb, ce;        // tap range (tap split)
};
__device__ __forceinline__ Share wave_share(int nch, int ntc, int w)
{
    Share s;
    s.by_channel = nch >= 4;
    if (s.by_channel) {
        s.cb = 0;
        s.ce = ntc;
    } else {
        const int q = ((ntc + 31) / 32) * 8;      // quarter, multiple of 8
        s.cb = min(w * q, ntc);
        s.ce = min((w + 1) * q, ntc);
    }
    return s;
}

// Contracts the staged tile: X window rows of length rl per channel (LDS xs),
// taps hs[(p * nch + ch) * tcs + c] (tcs taps per row); optional halo row kTA
// for phase 0 (block rate), accumulated over the same share.
template <int NPH, bool HALO>
__device__ __forceinline__ void corr_tile(const float* __restrict__ xs, int rl, const float* __restrict__ hs, int tcs,
                                          int nch, int ntc, int w, int lane, float (&acc)[NPH][kOPT], float& halo)
{
    const Share sh = wave_share(nch, ntc, w);
    const int hps = nch * tcs;
    if (sh.by_channel) {
        for (int ch = nch - 1 - w; ch >= 0; ch -= 4) {
            corr_taps<NPH>(xs + ch * rl, hs + ch * tcs, hps, 0, ntc, lane, acc);
            if (HALO)
                for (int c = lane; c < ntc; c += 64) halo = fmaf(xs[ch * rl + kTA + c], hs[ch * tcs + c], halo);
        }
    } else {
        for (int ch = nch - 1; ch >= 0; --ch) {
            if (sh.cb < sh.ce) corr_taps<NPH>(xs + ch * rl, hs + ch * tcs, hps, sh.cb, sh.ce, lane, acc);
            if (HALO)
                for (int c = sh.cb + lane; c < sh.ce; c += 64)
                    halo = fmaf(xs[ch * rl + kTA + c], hs[ch * tcs + c], halo);
        }
    }
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// dst(x) = src(x) for x < n over the workgroup's threads, with 8 loads of a
// thread in flight before its first store (a staging loop that stores each
// value before loading the next waits out the memory latency every time).
template <typename Ld, typename St>
__device__ __forceinline__ void stage_copy(int n, Ld ld, St st)
{
    for (int base = threadIdx.x; base < n; base += 8 * kCT) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int x = base + j * kCT;
            v[j] = x < n ? ld(x) : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int x = base + j * kCT;
            if (x < n) st(x, v[j]);
        }
    }
}

// Epilogue shared by both kernels: the four waves' row sums are added in a
// fixed order (wave 3 first), then written as
//   mode 0: y[a0 L + f] = Y for f < kTA NPH (full rate, f = row NPH + p);
//   mode 1: block rate, y[m] for m in [a0 L, (a0 + kTA) L) interpolated
//           between the computed samples (the halo supplies row kTA);
//   mode 2: partial sums part[a] of this channel range (rows a < nd).
template <int NPH>
__device__ __forceinline__ void corr_finish(float* red, const float (&acc)[NPH][kOPT], float halo, int mode,
                                            int64_t a0, int64_t nd, int L, int64_t nout, float* __restrict__ y,
                                            float* __restrict__ part)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    constexpr int NF = kTA * NPH;
    __syncthreads();      // the staged tiles may alias `red`
#pragma unroll
    for (int o = 0; o < kOPT; ++o)
#pragma unroll
        for (int p = 0; p < NPH; ++p) red[w * NF + (kOPT * lane + o) * NPH + p] = acc[p][o];
    float hs = 0.0f;
    if (mode == 1) hs = wave_sum(halo);
    if (mode == 1 && lane == 0) red[4 * NF + w] = hs;
    __syncthreads();
    if (mode == 0) {
        for (int f = tid; f < NF; f += kCT) {
            const int64_t m = a0 * L + f;
            if (m < nout) y[m] = ((red[3 * NF + f] + red[2 * NF + f]) + red[NF + f]) + red[f];
        }
        return;
    }
    if (mode == 2) {
        for (int f = tid; f < kTA; f += kCT) {
            const int64_t a = a0 + f;
            if (a < nd) part[a] = ((red[3 * NF + f] + red[2 * NF + f]) + red[NF + f]) + red[f];
        }
        return;
    }
    // block rate: yd[row] for rows 0 .. kTA (the last from the halo), kept in
    // the wave-0 slice of red after the other slices are added in
    float* yd = red + 5 * NF;
    for (int f = tid; f < kTA; f += kCT) yd[f] = ((red[3 * NF + f] + red[2 * NF + f]) + red[NF + f]) + red[f];
    if (tid == 0) yd[kTA] = ((red[4 * NF + 3] + red[4 * NF + 2]) + red[4 * NF + 1]) + red[4 * NF];
    __syncthreads();
    const int64_t mlo = a0 * L;
    const int nq = (int)((a0 + kTA) * L < nout ? kTA * L : nout - mlo);   // at most kTA L <= 4096
    for (int q = tid; q < nq; q += kCT) {
        const int row = q / L, f = q - row * L;
        float v = yd[row];
        if (f != 0 && a0 + row + 1 < nd) v += ((float)f / (float)L) * (yd[row + 1] - v);
        y[mlo + q] = v;
    }
}

// LDS floats of the epilogue: 4 wave slices, the halo sums and the yd rows.
template <int NPH>
constexpr int finish_floats() { return 5 * kTA * NPH + kTA + 8; }

// ---- blocks of at most 8 samples: everything in one launch ---------------
constexpr int kSmallMaxL = 8;
constexpr int kSmallBudget = 16384;      // LDS floats for a staged tile (64 KiB)

// LDS floats of one staged tile with tc taps: raw signal rows, projected
// channels, kernel segment, taps.
// (the kernel segment is padded to a multiple of 4 floats so that the taps
// after it stay 16-byte aligned for any L)
__host__ __device__ constexpr int small_kseg_floats(int L, int tc) { return (tc * L + 2 * L + 3) / 4 * 4; }
__host__ __device__ constexpr int small_stage_floats(int L, int r, int nph, int tc)
{
    return (kTA + tc + 4) * L + r * (kTA + tc + 4) + small_kseg_floats(L, tc) + nph * r * tc;
}

// dynamic LDS: max(small_stage_floats(L, r, NPH, tc), finish_floats<NPH>())
template <int NPH>
__global__ __launch_bounds__(kCT) void corr_small_kernel(CorrSmallArgs p, int tcmax)
{
    extern __shared__ __align__(16) float lds[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int L = p.L, r = p.r;
    const int rlm = kTA + tcmax + 4;                    // row stride of the staged windows
    float* ss = lds;                                    // [rl * L]   raw signal of the window
    float* xs = ss + rlm * L;                           // [r][rlm]   projected channels
    float* ks = xs + r * rlm;                           // kernel segment
    float* hs = ks + small_kseg_floats(L, tcmax);       // [NPH][r][tcmax] taps
    const int64_t a0 = (int64_t)blockIdx.x * kTA;
    const int64_t ntp = (p.ntap + 7) / 8 * 8;
    const bool halo_on = p.block != 0;

    float acc[NPH][kOPT];
#pragma unroll
    for (int q = 0; q < NPH; ++q)
#pragma unroll
        for (int o = 0; o < kOPT; ++o) acc[q][o] = 0.0f;
    float halo = 0.0f;

    for (int64_t c0 = 0; c0 < ntp; c0 += tcmax) {
        const int tc = (int)(ntp - c0 < tcmax ? ntp - c0 : tcmax);
        const int64_t i0 = a0 + c0;                     // first staged row
        const int rl = kTA + tc + 4;
        __syncthreads();                                // previous tile consumed
        // raw signal samples of rows i0 .. i0 + rl (zero past W, or periodic)
        const int64_t n0 = i0 * L;
        stage_copy(rl * L,
                   [&](int x) {
                       const int64_t n = n0 + x;
                       return p.period > 0 ? p.s[n % p.period] : (n < p.W ? p.s[n] : 0.0f);
                   },
                   [&](int x, float v) { ss[x] = v; });
        // kernel samples k'(c0 L - (L - 1) + x)
        const int64_t k0 = c0 * L - (L - 1);
        stage_copy(tc * L + 2 * L - 1,
                   [&](int x) {
                       const int64_t n = k0 + x;
                       return (n >= 0 && n < p.N) ? (p.reverse ? p.k[p.N - 1 - n] : p.k[n]) : 0.0f;
                   },
                   [&](int x, float v) { ks[x] = v; });
        __syncthreads();
        // channels: X(l, i0 + ii) = sum_t s[(i0 + ii) L + t] C[t, l]
        for (int x = tid; x < r * rl; x += kCT) {
            const int l = x / rl, ii = x - l * rl;
            float v = 0.0f;
            for (int t = 0; t < L; ++t) v = fmaf(ss[ii * L + t], p.C[t * L + l], v);
            xs[l * rlm + ii] = v;
        }
        // taps: H(q, l, c0 + cc) = sum_u D[l, u] k'((c0 + cc) L - q + u), zero past ntap
        for (int x = tid; x < NPH * r * tc; x += kCT) {
            const int cc = x % tc, l = (x / tc) % r, q = x / (tc * r);
            float v = 0.0f;
            if (c0 + cc < p.ntap) {
                const float* kp = ks + cc * L - q + (L - 1);
                for (int u = 0; u < L; ++u) v = fmaf(p.DT[u * L + l], kp[u], v);
            }
            hs[(q * r + l) * tcmax + cc] = v;
        }
        __syncthreads();
        if (halo_on)
            corr_tile<NPH, true>(xs, rlm, hs, tcmax, r, tc, w, lane, acc, halo);
        else
            corr_tile<NPH, false>(xs, rlm, hs, tcmax, r, tc, w, lane, acc, halo);
    }
    corr_finish<NPH>(lds, acc, halo, halo_on ? 1 : 0, a0, p.nrows, L, p.nout, p.y, nullptr);
}

// ---- block rate, longer blocks ----------------------------------------------
constexpr int kBlockRL = kTA + kBlockTC + 4;
constexpr int block_lds_floats()
{
    constexpr int stage = kBlockCH * kBlockRL + kBlockCH * kBlockTC;
    return stage > finish_floats<1>() ? stage : finish_floats<1>();
}

// X(ch, i): SRC 0 = channel rows x[ch * xld + i] (valid i < xn);
//           SRC 1 = polyphase channels of the raw signal x[i * L + ch] (valid i L + ch < xn).
// H(ch, c) = h[ch * hld + c] (zero-padded to hld taps).
// The workgroup walks its staged tiles (channel groups from the highest down,
// then tap tiles); the global loads of tile s + 1 are issued into registers
// before tile s is contracted and parked in LDS after it.
constexpr int kBlockXPT = (kBlockCH * kBlockRL + kCT - 1) / kCT;   // staged X values per thread
constexpr int kBlockHPT = (kBlockCH * kBlockTC + kCT - 1) / kCT;   // staged taps per thread

struct BlockTile {
    int g_lo, nch;     // channels g_lo .. g_lo + nch - 1
    int64_t c0;        // first tap
    int tc, rl;        // taps, staged rows
};

template <int SRC>
__device__ __forceinline__ void block_tile_load(const CorrBlockArgs& p, int64_t a0, const BlockTile& t,
                                                float (&xv)[kBlockXPT], float (&hv)[kBlockHPT])
{
    const int tid = threadIdx.x;
    const int64_t i0 = a0 + t.c0;
#pragma unroll
    for (int j = 0; j < kBlockXPT; ++j) {
        const int x = tid + j * kCT;
        float v = 0.0f;
        if (x < t.nch * t.rl) {
            if (SRC == 0) {
                const int ch = x / t.rl, ii = x - ch * t.rl;
                const int64_t i = i0 + ii;
                if (i < p.xn) v = p.x[(int64_t)(t.g_lo + ch) * p.xld + i];
            } else {   // consecutive threads read consecutive channels of one row
                const int ii = x / t.nch, ch = x - ii * t.nch;
                const int64_t n = (i0 + ii) * p.L + t.g_lo + ch;
                if (n < p.xn) v = p.x[n];
            }
        }
        xv[j] = v;
    }
#pragma unroll
    for (int j = 0; j < kBlockHPT; ++j) {
        const int x = tid + j * kCT;
        float v = 0.0f;
        if (x < t.nch * t.tc) {
            const int ch = x / t.tc, cc = x - ch * t.tc;
            v = p.h[(int64_t)(t.g_lo + ch) * p.hld + t.c0 + cc];
        }
        hv[j] = v;
    }
}

template <int SRC>
__device__ __forceinline__ void block_tile_store(const BlockTile& t, const float (&xv)[kBlockXPT],
                                                 const float (&hv)[kBlockHPT], float* xs, float* hs)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < kBlockXPT; ++j) {
        const int x = tid + j * kCT;
        if (x < t.nch * t.rl) {
            int ch, ii;
            if (SRC == 0) {
                ch = x / t.rl;
                ii = x - ch * t.rl;
            } else {
                ii = x / t.nch;
                ch = x - ii * t.nch;
            }
            xs[ch * kBlockRL + ii] = xv[j];
        }
    }
#pragma unroll
    for (int j = 0; j < kBlockHPT; ++j) {
        const int x = tid + j * kCT;
        if (x < t.nch * t.tc) {
            const int ch = x / t.tc, cc = x - ch * t.tc;
            hs[ch * kBlockTC + cc] = hv[j];
        }
    }
}

template <int SRC>
__global__ __launch_bounds__(kCT) void corr_block_kernel(CorrBlockArgs p)
{
    __shared__ __align__(16) float lds[block_lds_floats()];
    float* xs = lds;                                   // [CH][RL]
    float* hs = xs + kBlockCH * kBlockRL;              // [CH][TC]
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t a0 = (int64_t)blockIdx.x * kTA;
    const int sp = blockIdx.y;
    const int ch_lo = (int)((int64_t)p.nch * sp / p.nsplit), ch_hi = (int)((int64_t)p.nch * (sp + 1) / p.nsplit);
    const int ntt = (int)((p.hld + kBlockTC - 1) / kBlockTC);            // tap tiles per channel group
    const int ngr = (ch_hi - ch_lo + kBlockCH - 1) / kBlockCH;            // channel groups
    auto tile = [&](int s) {
        BlockTile t;
        const int g = s / ntt, q = s - g * ntt;
        const int g_hi = ch_hi - g * kBlockCH;
        t.g_lo = g_hi - kBlockCH > ch_lo ? g_hi - kBlockCH : ch_lo;
        t.nch = g_hi - t.g_lo;
        t.c0 = (int64_t)q * kBlockTC;
        t.tc = (int)(p.hld - t.c0 < kBlockTC ? p.hld - t.c0 : kBlockTC);
        t.rl = kTA + t.tc + 4;
        return t;
    };
    const int nt = ngr * ntt;

    float acc[1][kOPT];
#pragma unroll
    for (int o = 0; o < kOPT; ++o) acc[0][o] = 0.0f;
    float halo = 0.0f;
    float xv[kBlockXPT], hv[kBlockHPT];
    if (nt > 0) {
        block_tile_load<SRC>(p, a0, tile(0), xv, hv);
        block_tile_store<SRC>(tile(0), xv, hv, xs, hs);
    }
    __syncthreads();
    for (int s = 0; s < nt; ++s) {
        const BlockTile t = tile(s);
        if (s + 1 < nt) block_tile_load<SRC>(p, a0, tile(s + 1), xv, hv);     // in flight during the contraction
        corr_tile<1, false>(xs, kBlockRL, hs, kBlockTC, t.nch, t.tc, w, lane, acc, halo);
        __syncthreads();
        if (s + 1 < nt) block_tile_store<SRC>(tile(s + 1), xv, hv, xs, hs);
        __syncthreads();
    }
    corr_finish<1>(lds, acc, halo, 2, a0, p.nd, p.L, p.nout, p.y, p.part + (int64_t)sp * p.nd);
}

// Sum of the channel-range partials (highest range first) for a tile of rows,
// then the block-rate interpolation of every output of those rows:
// y[aL + f] = yd[a] + (f / L)(yd[a + 1] - yd[a]) while a + 1 < nd, else yd[a].
// A workgroup covers kInterpRows(L) rows (about 4096 outputs), so the output
// stream is spread over many workgroups; outputs go out 4 at a time when L is
// a multiple of 4 and y is 16-byte aligned.
constexpr int kInterpOut = 4096;
constexpr int kInterpPart = 4096;      // staged partial sums (nsplit <= 64)
__global__ __launch_bounds__(256) void corr_interp_kernel(const float* __restrict__ part, int nsplit, int64_t nd, int L,
                                                          int rows, int64_t nout, float* __restrict__ y, int vec)
{
    __shared__ float yd[kInterpOut + 1];
    __shared__ float ps[kInterpPart];
    const int tid = threadIdx.x;
    const int64_t a0 = (int64_t)blockIdx.x * rows;
    // the partials of rows a0 .. a0 + rows, all loads in flight at once, then
    // summed per row in a fixed order (highest range first)
    const int nr = rows + 1;
    for (int c0 = 0; c0 < nr; c0 += kInterpPart / nsplit) {
        const int cr = min(kInterpPart / nsplit, nr - c0);
        __syncthreads();
        for (int base = tid; base < cr * nsplit; base += 8 * 256) {
            float v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int x = base + j * 256;
                const int sp = x / cr, i = x - sp * cr;
                const int64_t a = a0 + c0 + i;
                v[j] = (x < cr * nsplit && a < nd) ? part[(int64_t)sp * nd + a] : 0.0f;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int x = base + j * 256;
                if (x < cr * nsplit) ps[x] = v[j];
            }
        }
        __syncthreads();
        for (int i = tid; i < cr; i += 256) {
            float v = ps[(nsplit - 1) * cr + i];
            for (int sp = nsplit - 2; sp >= 0; --sp) v += ps[sp * cr + i];
            yd[c0 + i] = v;
        }
    }
    __syncthreads();
    const int64_t mlo = a0 * L;
    const int nq = (int)(mlo + (int64_t)rows * L < nout ? (int64_t)rows * L : nout - mlo);
    if (vec) {
        for (int q = 4 * tid; q < nq; q += 4 * 256) {
            const int row = q / L, f = q - row * L;
            const float v0 = yd[row];
            const float d = a0 + row + 1 < nd ? yd[row + 1] - v0 : 0.0f;
            f32x4 o;
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = f + e == 0 ? v0 : v0 + ((float)(f + e) / (float)L) * d;
            if (q + 3 < nq) {
                *reinterpret_cast<f32x4*>(y + mlo + q) = o;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (q + e < nq) y[mlo + q + e] = o[e];
            }
        }
    } else {
        for (int q = tid; q < nq; q += 256) {
            const int row = q / L, f = q - row * L;
            float v = yd[row];
            if (f != 0 && a0 + row + 1 < nd) v += ((float)f / (float)L) * (yd[row + 1] - v);
            y[mlo + q] = v;
        }
    }
}

// Kernel-side taps of the block rate, on aligned kernel blocks c < hld (zero
// taps for blocks c >= ncb):
//   kd_kernel:      KD(l, c) = sum_u D[l, u] k'(cL + u), l < r;
//   rebuild_kernel: H(t, c) = sum_{l<r} C[t, l] KD(l, c), highest l first --
//                   the kernel blocks rebuilt from their first r projections
//                   (the raw polyphase grouping, chosen at many projections).
// Both are small contractions (at most L r ncb products each); a workgroup
// owns a 16 x 16 tile of outputs, stages the 16 rows of each operand in LDS
// (zero-padded to a multiple of 4) and gives every thread one dot product,
// read 4 terms at a time into 4 independent partial sums with the loop
// unrolled so that the LDS reads run ahead (a plain loop waits out an LDS
// read latency per step: 64 of them at L = 256), so the work spreads
// over (rows / 16) x (blocks / 16) workgroups instead of queueing behind a few.
constexpr int kTapT = 16;
constexpr int kTapS = 256 + 4;      // LDS row stride (rows of at most 256 values)

// Loads the tile's two operands (n values each, n <= 16 x 256) with every
// load of a thread in flight before its first LDS store: one memory latency
// for the staging instead of one per batch.
template <typename LdA, typename StA, typename LdB, typename StB>
__device__ __forceinline__ void stage_pair(int n, LdA lda, StA sta, LdB ldb, StB stb)
{
    constexpr int PT = kTapT * 256 / kCT;     // values per thread and operand
    float va[PT], vb[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) {
        const int x = threadIdx.x + j * kCT;
        va[j] = x < n ? lda(x) : 0.0f;
        vb[j] = x < n ? ldb(x) : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < PT; ++j) {
        const int x = threadIdx.x + j * kCT;
        if (x < n) {
            sta(x, va[j]);
            stb(x, vb[j]);
        }
    }
}

__global__ __launch_bounds__(256) void kd_kernel(const float* __restrict__ k, int64_t N, int reverse, int L, int r,
                                                 int64_t ncb, const float* __restrict__ DT, float* __restrict__ kd,
                                                 int64_t hld)
{
    __shared__ __align__(16) float ds[kTapT * kTapS];     // ds[i][u] = D[l0 + i, u]
    __shared__ __align__(16) float ks[kTapT * kTapS];     // ks[j][u] = k'((c0 + j) L + u)
    const int tid = threadIdx.x;
    const int l0 = blockIdx.y * kTapT;
    const int64_t c0 = (int64_t)blockIdx.x * kTapT;
    const int L4 = (L + 3) / 4 * 4;
    // D^T rows u hold the l values contiguously: 16 consecutive threads read
    // the tile's 16 rows of D at one u; the kernel blocks are read along u
    stage_pair(kTapT * L4,
               [&](int x) {
                   const int u = x / kTapT, i = x - u * kTapT;
                   return (l0 + i < r && u < L) ? DT[(int64_t)u * L + l0 + i] : 0.0f;
               },
               [&](int x, float v) {
                   const int u = x / kTapT, i = x - u * kTapT;
                   ds[i * kTapS + u] = v;
               },
               [&](int x) {
                   const int j = x / L4, u = x - j * L4;
                   const int64_t c = c0 + j, n = c * L + u;
                   return (c < ncb && u < L && n < N) ? (reverse ? k[N - 1 - n] : k[n]) : 0.0f;
               },
               [&](int x, float v) {
                   const int j = x / L4, u = x - j * L4;
                   ks[j * kTapS + u] = v;
               });
    __syncthreads();
    const int i = tid / kTapT, j = tid - (tid / kTapT) * kTapT;
    const f32x4* dr = reinterpret_cast<const f32x4*>(ds + i * kTapS);
    const f32x4* kr = reinterpret_cast<const f32x4*>(ks + j * kTapS);
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 8
    for (int q = 0; q < L4 / 4; ++q) {
        const f32x4 a = dr[q], b = kr[q];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = fmaf(a[e], b[e], v[e]);
    }
    if (l0 + i < r && c0 + j < hld) kd[(int64_t)(l0 + i) * hld + c0 + j] = (v[0] + v[1]) + (v[2] + v[3]);
}

__global__ __launch_bounds__(256) void rebuild_kernel(int L, int r, const float* __restrict__ CT,
                                                      const float* __restrict__ kd, float* __restrict__ h,
                                                      int64_t hld)
{
    __shared__ __align__(16) float cs[kTapT * kTapS];     // cs[i][l] = C[t0 + i, l]
    __shared__ __align__(16) float qs[kTapT * kTapS];     // qs[j][l] = KD(l, c0 + j)
    const int tid = threadIdx.x;
    const int t0 = blockIdx.y * kTapT;
    const int64_t c0 = (int64_t)blockIdx.x * kTapT;
    const int r4 = (r + 3) / 4 * 4;
    stage_pair(kTapT * r4,
               [&](int x) {
                   const int l = x / kTapT, i = x - l * kTapT;
                   return (t0 + i < L && l < r) ? CT[(int64_t)l * L + t0 + i] : 0.0f;
               },
               [&](int x, float v) {
                   const int l = x / kTapT, i = x - l * kTapT;
                   cs[i * kTapS + l] = v;
               },
               [&](int x) {
                   const int l = x / kTapT, j = x - l * kTapT;
                   return (c0 + j < hld && l < r) ? kd[(int64_t)l * hld + c0 + j] : 0.0f;
               },
               [&](int x, float v) {
                   const int l = x / kTapT, j = x - l * kTapT;
                   qs[j * kTapS + l] = v;
               });
    __syncthreads();
    const int i = tid / kTapT, j = tid - (tid / kTapT) * kTapT;
    const f32x4* cr = reinterpret_cast<const f32x4*>(cs + i * kTapS);
    const f32x4* qr = reinterpret_cast<const f32x4*>(qs + j * kTapS);
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 8
    for (int q = r4 / 4 - 1; q >= 0; --q) {
        const f32x4 a = cr[q], b = qr[q];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = fmaf(a[e], b[e], v[e]);
    }
    if (t0 + i < L && c0 + j < hld) h[(int64_t)(t0 + i) * hld + c0 + j] = (v[3] + v[2]) + (v[1] + v[0]);
}

// The projected kernel blocks alone for the projected grouping (few
// projections, so a 16 x 16 tile of (l, c) would mostly idle): kTapBlocks
// aligned blocks per workgroup of 1024 threads; thread (l, g) sums u over
// range g of ng ranges of at least 16 terms (8 loads of D in flight), and
// the range sums are added in a fixed order (highest range first).
constexpr int kTapBlocks = 4;
constexpr int kTapThreads = 1024;
__global__ __launch_bounds__(kTapThreads) void kd_range_kernel(const float* __restrict__ k, int64_t N, int reverse,
                                                               int L, int r, int64_t ncb, const float* __restrict__ DT,
                                                               float* __restrict__ h, int64_t hld)
{
    __shared__ float kb[kTapBlocks][256];
    __shared__ float part[kTapThreads][kTapBlocks];
    const int tid = threadIdx.x;
    const int64_t cb0 = (int64_t)blockIdx.x * kTapBlocks;
    for (int x = tid; x < kTapBlocks * L; x += kTapThreads) {
        const int j = x / L, u = x - j * L;
        const int64_t n = (cb0 + j) * L + u;
        kb[j][u] = (cb0 + j < ncb && n < N) ? (reverse ? k[N - 1 - n] : k[n]) : 0.0f;
    }
    __syncthreads();
    const int ng = max(1, min(kTapThreads / r, L / 16));
    const int l = tid % r, g = tid / r;
    float v[kTapBlocks] = {};
    if (g < ng) {
        const int ulo = (int)((int64_t)L * g / ng), uhi = (int)((int64_t)L * (g + 1) / ng);
        for (int u0 = ulo; u0 < uhi; u0 += 8) {
            float d[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) d[e] = u0 + e < uhi ? DT[(u0 + e) * L + l] : 0.0f;
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (u0 + e < uhi)
#pragma unroll
                    for (int j = 0; j < kTapBlocks; ++j) v[j] = fmaf(d[e], kb[j][u0 + e], v[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < kTapBlocks; ++j) part[tid][j] = v[j];
    __syncthreads();
    for (int x = tid; x < r * kTapBlocks; x += kTapThreads) {
        const int ll = x / kTapBlocks, j = x - ll * kTapBlocks;
        float sacc = 0.0f;
        for (int gg = ng - 1; gg >= 0; --gg) sacc += part[gg * r + ll][j];
        if (cb0 + j < hld) h[(int64_t)ll * hld + cb0 + j] = sacc;
    }
}

template <int NPH>
int launch_small_t(const CorrSmallArgs& a, hipStream_t s)
{
    // the largest tap tile (a multiple of 32, at most the padded tap count)
    // whose staged tile fits the LDS budget
    const int nph = NPH;
    const int64_t ntp32 = rup(rup(a.ntap, 8), 32);
    const int budget = std::max(kSmallBudget, finish_floats<NPH>());
    int tc = 32;
    while (tc < 2048 && tc < ntp32 && small_stage_floats(a.L, a.r, nph, tc + 32) <= budget) tc += 32;
    const size_t lds = 4 * (size_t)std::max(small_stage_floats(a.L, a.r, nph, tc), finish_floats<NPH>());
    static size_t lds_allowed = 65536;    // per instantiation: raise the dynamic LDS limit when needed
    if (lds > lds_allowed) {
        if (hipFuncSetAttribute((const void*)corr_small_kernel<NPH>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) != hipSuccess)
            return -1;
        lds_allowed = lds;
    }
    hipLaunchKernelGGL(corr_small_kernel<NPH>, dim3((unsigned)cdiv(a.nrows, kTA)), dim3(kCT), lds, s, a, tc);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int corr_rows_per_tile() { return kTA; }
int corr_small_max_L() { return kSmallMaxL; }

int launch_corr_small(const CorrSmallArgs& a, hipStream_t s)
{
    if (a.L < 1 || a.L > kSmallMaxL || a.r < 1 || a.r > a.L) return -2;
    if (a.block) return launch_small_t<1>(a, s);
    switch (a.L) {
    case 1: return launch_small_t<1>(a, s);
    case 2: return launch_small_t<2>(a, s);
    case 3: return launch_small_t<3>(a, s);
    case 4: return launch_small_t<4>(a, s);
    case 5: return launch_small_t<5>(a, s);
    case 6: return launch_small_t<6>(a, s);
    case 7: return launch_small_t<7>(a, s);
    default: return launch_small_t<8>(a, s);
    }
}

int launch_corr_block(const CorrBlockArgs& a, int src, hipStream_t s)
{
    dim3 grid((unsigned)cdiv(a.nd, kTA), (unsigned)a.nsplit);
    if (src == 0) hipLaunchKernelGGL(corr_block_kernel<0>, grid, dim3(kCT), 0, s, a);
    else hipLaunchKernelGGL(corr_block_kernel<1>, grid, dim3(kCT), 0, s, a);
    if (hipGetLastError() != hipSuccess) return -1;
    const int rows = std::max(1, kInterpOut / a.L);
    const int vec = a.L % 4 == 0 && ((uintptr_t)a.y % 16) == 0;
    hipLaunchKernelGGL(corr_interp_kernel, dim3((unsigned)cdiv(a.nd, rows)), dim3(256), 0, s, a.part, a.nsplit, a.nd,
                       a.L, rows, a.nout, a.y, vec);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_ktilde(const float* k, int64_t N, int reverse, int L, int r, int64_t ncb, const float* CT, const float* DT,
                  float* kd, float* h, int64_t hld, hipStream_t s)
{
    if (L > kTapS - 4 || cdiv(hld, kTapT) > 0x7fffffff) return -2;
    hipLaunchKernelGGL(kd_kernel, dim3((unsigned)cdiv(hld, kTapT), (unsigned)cdiv(r, kTapT)), dim3(256), 0, s, k, N,
                       reverse, L, r, ncb, DT, kd, hld);
    if (hipGetLastError() != hipSuccess) return -1;
    hipLaunchKernelGGL(rebuild_kernel, dim3((unsigned)cdiv(hld, kTapT), (unsigned)cdiv(L, kTapT)), dim3(256), 0, s,
                       L, r, CT, (const float*)kd, h, hld);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_kblock_taps(const float* k, int64_t N, int reverse, int L, int r, int64_t ncb, int64_t hld,
                       const float* DT, float* h, hipStream_t s)
{
    if (L > 256 || cdiv(hld, kTapBlocks) > 0x7fffffff) return -2;
    hipLaunchKernelGGL(kd_range_kernel, dim3((unsigned)cdiv(hld, kTapBlocks)), dim3(kTapThreads), 0, s, k, N, reverse,
                       L, r, ncb, DT, h, hld);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace pj
