// fft.hip -- the reduced cross-correlation in the frequency domain (paper
// Sec. III-A: the correlation of the projected signal with the projected
// kernel may be carried out with FFTs; Sec. III-C, eq. (19) and (21): the
// cost model of that realisation).  Same result as the implicit GEMM of
// conv.hip (reading R9, full rate):
//     y[aL + b] = sum_{l<r} sum_{c<T} sc_l[a + c] h_{l,b}[c],   h_{l,b}[c] = kd_l[cL - b],
// i.e. for every output phase b a sum over l of stride-1 correlations of the
// projected signal row sc_l with T taps.  Overlap-save: segment s covers rows
// a in [sP, sP + P) with P = F - T + 1; in the F-point DFT domain
//     Y_{b,s} = sum_{l<r} conj(FFT(h_{l,b})) * FFT(sc_l[sP .. sP + F))
// and the first P samples of IFFT(Y_{b,s}) are the rows of the segment
// (circular correlation without wrap-around there).
//
// Kernels: (1) taps of every (l, b) computed from the kernel and D and
// transformed; (2) every (l, s) signal segment transformed; (3) the bin-wise
// contraction over l; (4) the inverse transform of every (b, s) with the
// rows scattered to y.  Each transform is one workgroup's radix-2 Stockham
// FFT in LDS (natural order in and out), with twiddles computed once in FP64.
#include "conv.h"

namespace pj {

namespace {

constexpr int kFftThreads = 256;
constexpr int kFftMax = 4096;            // largest transform (two LDS buffers of 32 KiB)

struct cf {
    float x, y;
};

// tw[q] = exp(-2 pi i q / F) for q < F / 2, rounded from FP64.
__global__ __launch_bounds__(256) void fft_twiddle_kernel(cf* __restrict__ tw, int F)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= F / 2) return;
    double s, c;
    sincospi(2.0 * (double)q / (double)F, &s, &c);
    tw[q] = cf{(float)c, (float)(-s)};
}

// In-place in the sense of the two LDS buffers: x holds the input, the result
// is in the returned buffer (x or y).  Stage s combines pairs j and j + F/2
// with the twiddle exp(-+2 pi i k / (2 Ns)), k = j mod Ns, Ns = 2^s, and
// writes them to positions (j / Ns) 2 Ns + k and that + Ns (Stockham
// autosort: natural order after the last stage).
template <bool INV>
__device__ cf* fft_lds(cf* x, cf* y, const cf* __restrict__ tw, int F, int logF)
{
    const int half = F >> 1;
    for (int s = 0; s < logF; ++s) {
        const int Ns = 1 << s;
        for (int j = threadIdx.x; j < half; j += kFftThreads) {
            const int k = j & (Ns - 1);
            cf w = tw[k << (logF - 1 - s)];
            if (INV) w.y = -w.y;
            const cf a = x[j], b0 = x[j + half];
            const cf b = {b0.x * w.x - b0.y * w.y, b0.x * w.y + b0.y * w.x};
            const int d = ((j >> s) << (s + 1)) + k;
            y[d] = cf{a.x + b.x, a.y + b.y};
            y[d + Ns] = cf{a.x - b.x, a.y - b.y};
        }
        __syncthreads();
        cf* t = x;
        x = y;
        y = t;
    }
    return x;
}

// (1) Hf[(l L + b) F + f] = FFT_F(h_{l,b}), h_{l,b}[c] = sum_u D[l, u] k'(cL - b + u)
// for c < T (zero-padded to F); one workgroup per (l, b).
__global__ __launch_bounds__(kFftThreads) void fft_taps_kernel(const float* __restrict__ k, int64_t N, int reverse,
                                                               int L, int T, const float* __restrict__ DT,
                                                               const cf* __restrict__ tw, int F, int logF,
                                                               cf* __restrict__ Hf)
{
    __shared__ cf buf[2][kFftMax];
    const int l = blockIdx.x / L, b = blockIdx.x - (blockIdx.x / L) * L;
    for (int c = threadIdx.x; c < F; c += kFftThreads) {
        float v = 0.0f;
        if (c < T) {
            const int64_t n0 = (int64_t)c * L - b;
            for (int u = 0; u < L; ++u) {
                const int64_t n = n0 + u;
                if (n >= 0 && n < N) v = fmaf(DT[u * L + l], reverse ? k[N - 1 - n] : k[n], v);
            }
        }
        buf[0][c] = cf{v, 0.0f};
    }
    __syncthreads();
    const cf* out = fft_lds<false>(buf[0], buf[1], tw, F, logF);
    cf* dst = Hf + (int64_t)blockIdx.x * F;
    for (int f = threadIdx.x; f < F; f += kFftThreads) dst[f] = out[f];
}

// (2) Sf[(l nseg + s) F + f] = FFT_F(sc_l[sP .. sP + F)) (zero past nbp); one
// workgroup per (l, s).
__global__ __launch_bounds__(kFftThreads) void fft_signal_kernel(const float* __restrict__ sc, int64_t nbp,
                                                                 int64_t nseg, int P, const cf* __restrict__ tw,
                                                                 int F, int logF, cf* __restrict__ Sf)
{
    __shared__ cf buf[2][kFftMax];
    const int64_t l = blockIdx.x / nseg, s = blockIdx.x - l * nseg;
    const float* row = sc + l * nbp;
    const int64_t i0 = s * P;
    for (int f = threadIdx.x; f < F; f += kFftThreads) {
        const int64_t i = i0 + f;
        buf[0][f] = cf{i < nbp ? row[i] : 0.0f, 0.0f};
    }
    __syncthreads();
    const cf* out = fft_lds<false>(buf[0], buf[1], tw, F, logF);
    cf* dst = Sf + (int64_t)blockIdx.x * F;
    for (int f = threadIdx.x; f < F; f += kFftThreads) dst[f] = out[f];
}

// (3) Yf[(b nseg + s) F + f] = sum_{l<r} conj(Hf[(l L + b) F + f]) Sf[(l nseg + s) F + f],
// highest l first.  A thread owns one bin f of kSegs segments and kPhases
// phases, so each spectrum value it loads serves several products.
constexpr int kSegs = 2, kPhases = 8;
__global__ __launch_bounds__(256) void fft_contract_kernel(const cf* __restrict__ Hf, const cf* __restrict__ Sf,
                                                           int r, int L, int64_t nseg, int F, cf* __restrict__ Yf)
{
    const int f = blockIdx.x * 256 + threadIdx.x;
    if (f >= F) return;
    const int64_t s0 = (int64_t)blockIdx.y * kSegs;
    const int b0 = blockIdx.z * kPhases;
    cf acc[kSegs][kPhases];
#pragma unroll
    for (int i = 0; i < kSegs; ++i)
#pragma unroll
        for (int j = 0; j < kPhases; ++j) acc[i][j] = cf{0.0f, 0.0f};
    for (int l = r - 1; l >= 0; --l) {
        cf sv[kSegs], hv[kPhases];
#pragma unroll
        for (int i = 0; i < kSegs; ++i)
            sv[i] = s0 + i < nseg ? Sf[((int64_t)l * nseg + s0 + i) * F + f] : cf{0.0f, 0.0f};
#pragma unroll
        for (int j = 0; j < kPhases; ++j)
            hv[j] = b0 + j < L ? Hf[((int64_t)l * L + b0 + j) * F + f] : cf{0.0f, 0.0f};
#pragma unroll
        for (int i = 0; i < kSegs; ++i)
#pragma unroll
            for (int j = 0; j < kPhases; ++j) {     // conj(h) s
                acc[i][j].x = fmaf(hv[j].x, sv[i].x, fmaf(hv[j].y, sv[i].y, acc[i][j].x));
                acc[i][j].y = fmaf(hv[j].x, sv[i].y, fmaf(-hv[j].y, sv[i].x, acc[i][j].y));
            }
    }
#pragma unroll
    for (int i = 0; i < kSegs; ++i)
#pragma unroll
        for (int j = 0; j < kPhases; ++j)
            if (s0 + i < nseg && b0 + j < L) Yf[((int64_t)(b0 + j) * nseg + s0 + i) * F + f] = acc[i][j];
}

// (4) rows a of segment s, phase b: y[(sP + a) L + b] = IFFT_F(Yf[b, s])[a] / F
// for a < P (and inside the output); one workgroup per (b, s).
__global__ __launch_bounds__(kFftThreads) void fft_out_kernel(const cf* __restrict__ Yf, int L, int64_t nseg, int P,
                                                              const cf* __restrict__ tw, int F, int logF,
                                                              int64_t nout, float* __restrict__ y)
{
    __shared__ cf buf[2][kFftMax];
    const int64_t b = blockIdx.x / nseg, s = blockIdx.x - b * nseg;
    const cf* src = Yf + (int64_t)blockIdx.x * F;
    for (int f = threadIdx.x; f < F; f += kFftThreads) buf[0][f] = src[f];
    __syncthreads();
    const cf* out = fft_lds<true>(buf[0], buf[1], tw, F, logF);
    const float scale = 1.0f / (float)F;
    for (int a = threadIdx.x; a < P; a += kFftThreads) {
        const int64_t m = (s * P + a) * L + b;
        if (m < nout) y[m] = out[a].x * scale;
    }
}

}  // namespace

// Transform size: the smallest power of two, at least 512, with at least
// three quarters of it left for outputs (P = F - T + 1 >= 3F / 4), at most
// kFftMax (there a quarter is accepted; longer kernels use the direct path).
ConvFftGeom conv_fft_geom(int64_t W, int64_t N, int L, int r)
{
    ConvFftGeom g;
    g.nout = W - N + 1;
    g.T = (N + L - 2) / L + 1;
    g.rows = cdiv(g.nout, L);
    int F = 512;
    while (F < kFftMax && 4 * (F - g.T + 1) < 3 * F) F *= 2;
    g.F = F;
    g.logF = 0;
    while ((1 << g.logF) < F) ++g.logF;
    g.P = F - g.T + 1;
    g.ok = 4 * g.P >= F;                               // at least a quarter of each transform is output
    g.nseg = g.ok ? cdiv(g.rows, g.P) : 0;
    g.nbp = rup(g.nseg * g.P + F, 128);              // projected rows, zero past the signal
    g.sc_bytes = rup((int64_t)r * g.nbp * 4, 256);
    g.tw_bytes = rup((int64_t)(F / 2) * 8, 256);
    g.hf_bytes = rup((int64_t)r * L * F * 8, 256);
    g.sf_bytes = rup((int64_t)r * g.nseg * F * 8, 256);
    g.yf_bytes = rup((int64_t)L * g.nseg * F * 8, 256);
    g.total = g.sc_bytes + g.tw_bytes + g.hf_bytes + g.sf_bytes + g.yf_bytes;
    return g;
}

// Which realisation proj_conv1d uses: estimated times (fitted to measurements
// on MI355X) of the direct path -- the one-launch vector-ALU kernel for L <= 8
// (W r T products at about 2e13 per second), otherwise the matrix-core
// implicit GEMM over a phase tile of 32, 64, 128 or 256 (the power of two
// covering L, at least 32) after two small launches -- and of the FFT path (six launches; about 0.12 ms + 0.004 ms per
// signal row and phase, r + L, per 2^22 samples, scaled by the share of each
// transform that is output); the FFT path is taken when it is estimated at
// least 20 % faster.
bool conv_prefers_fft(int64_t W, int64_t N, int L, int r)
{
    const ConvFftGeom f = conv_fft_geom(W, N, L, r);
    if (!f.ok || f.T < 16) return false;
    const double scale = (double)W / 4194304.0;
    const double t_fft = 30e-6 + scale * (0.12e-3 + 0.004e-3 * (r + L)) * (3.0 * f.F / (4.0 * f.P));
    double t_direct;
    if (L <= 8) {
        t_direct = 8e-6 + (double)W * r * f.T / 2.0e13;
    } else {
        const double bn = L > 128 ? 256.0 : L > 64 ? 128.0 : L > 32 ? 64.0 : 32.0;   // phase tile
        t_direct = 25e-6 + 2.0 * ((double)W / L) * bn * r * f.T / 1.0e14;
    }
    return t_fft < 0.8 * t_direct;
}

int launch_conv_fft(const ConvArgs& a, hipStream_t st)
{
    const ConvFftGeom g = conv_fft_geom(a.W, a.N, a.L, a.r);
    if (!g.ok) return -2;
    char* w = (char*)a.ws;
    float* sc = (float*)w;
    cf* tw = (cf*)(w + g.sc_bytes);
    cf* Hf = (cf*)(w + g.sc_bytes + g.tw_bytes);
    cf* Sf = (cf*)(w + g.sc_bytes + g.tw_bytes + g.hf_bytes);
    cf* Yf = (cf*)(w + g.sc_bytes + g.tw_bytes + g.hf_bytes + g.sf_bytes);
    if (launch_conv_signal_rows(a, sc, g.nbp, st) != 0) return -1;
    hipLaunchKernelGGL(fft_twiddle_kernel, dim3((unsigned)cdiv(g.F / 2, 256)), dim3(256), 0, st, tw, g.F);
    if (hipGetLastError() != hipSuccess) return -1;
    hipLaunchKernelGGL(fft_taps_kernel, dim3((unsigned)(a.r * a.L)), dim3(kFftThreads), 0, st, a.k, a.N, a.reverse,
                       a.L, (int)g.T, a.DT, tw, g.F, g.logF, Hf);
    if (hipGetLastError() != hipSuccess) return -1;
    hipLaunchKernelGGL(fft_signal_kernel, dim3((unsigned)((int64_t)a.r * g.nseg)), dim3(kFftThreads), 0, st, sc, g.nbp,
                       g.nseg, (int)g.P, tw, g.F, g.logF, Sf);
    if (hipGetLastError() != hipSuccess) return -1;
    dim3 cgrid((unsigned)cdiv(g.F, 256), (unsigned)cdiv(g.nseg, kSegs), (unsigned)cdiv(a.L, kPhases));
    hipLaunchKernelGGL(fft_contract_kernel, cgrid, dim3(256), 0, st, Hf, Sf, a.r, a.L, g.nseg, g.F, Yf);
    if (hipGetLastError() != hipSuccess) return -1;
    hipLaunchKernelGGL(fft_out_kernel, dim3((unsigned)((int64_t)a.L * g.nseg)), dim3(kFftThreads), 0, st, Yf, a.L,
                       g.nseg, (int)g.P, tw, g.F, g.logF, g.nout, a.y);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace pj
