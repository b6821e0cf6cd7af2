// conv.hip -- projected 1-D cross-correlation / convolution (paper Sec. III-A,
// eq. (10)-(14), and Sec. III-B: projection during the blocking of the input
// signal and of the kernel).
//
// The signal s is cut into aligned, non-overlapping blocks of L samples and
// each block is projected onto the first r columns of C:
//     sc_l[i] = sum_{t<L} s[iL + t] c[t, l]                       (step 1)
// The kernel is projected with the rows of D at every one of the L phases an
// output can take relative to the block grid:
//     kd_l[q] = sum_{u<L} d[l, u] k[q + u],  q = cL - b               (step 2)
// and every output sample accumulates the products over the r projections:
//     y[aL + b] = sum_{l<r} sum_c sc_l[a + c] kd_l[cL - b]            (step 3)
// With r = L this is the exact valid cross-correlation (D = C^{-1}); with
// r < L it is the exact cross-correlation of the block-projected signal.
//
// Step 3 is an implicit GEMM Y[a, b] = H[a, (l,c)] K[(l,c), b] whose left
// operand H[a, (l,c)] = sc_l[a + c] is a Hankel matrix: its MFMA fragments are
// read straight from the projected signal (small, cache resident), and the
// right operand K is packed once in the same fragment order as the GEMM's.
#include "common.h"

namespace pj {

namespace {

constexpr int kSigBlocks = 32;   // signal blocks per workgroup in step 1

// ---- step 1: block projection of the signal ---------------------------------
// Thread t handles projection l = t % LR and blocks b = t / LR + k * (256 / LR)
// of the workgroup's kSigBlocks blocks.  The blocks are staged in LDS with a
// padded row (L + 1) so that lanes reading different blocks hit different
// banks.
template <int BPT>
__global__ __launch_bounds__(256) void sig_project_kernel(
    const float* __restrict__ s, int64_t W, int L, int r, int LR, const float* __restrict__ C,
    float* __restrict__ sc, int64_t nbp)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float* lds = reinterpret_cast<float*>(smem_raw);
    const int64_t i0 = (int64_t)blockIdx.x * kSigBlocks;
    const int LP = L + 1;
    for (int idx = threadIdx.x; idx < kSigBlocks * L; idx += 256) {
        const int blk = idx / L, t = idx % L;
        const int64_t n = (i0 + blk) * L + t;
        lds[blk * LP + t] = (n < W) ? s[n] : 0.0f;
    }
    __syncthreads();
    const int l = threadIdx.x % LR;
    const int bg = threadIdx.x / LR, BG = 256 / LR;
    if (l >= r) return;
    float acc[BPT];
#pragma unroll
    for (int k = 0; k < BPT; ++k) acc[k] = 0.0f;
    for (int t = 0; t < L; ++t) {
        const float cf = C[t * L + l];
#pragma unroll
        for (int k = 0; k < BPT; ++k) {
            const int blk = bg + k * BG;
            if (blk < kSigBlocks) acc[k] += lds[blk * LP + t] * cf;
        }
    }
#pragma unroll
    for (int k = 0; k < BPT; ++k) {
        const int blk = bg + k * BG;
        const int64_t i = i0 + blk;
        if (blk < kSigBlocks && i < nbp) sc[(int64_t)l * nbp + i] = acc[k];
    }
}

// ---- step 2: kernel projected at every phase, packed as the right operand ---
// Packed like a GEMM operand (fragment order, FP32 tiles of 32 rows x 8):
// rows are the phases b < L, the contraction index is k = l * ncp + c.
__global__ __launch_bounds__(256) void kmat_pack_kernel(
    const float* __restrict__ k, int N, int reverse, int L, int r, int ncp, const float* __restrict__ DT,
    char* __restrict__ out, int64_t nrb, int64_t nkb)
{
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;   // lane vector index
    const int64_t total = nrb * nkb * 64;
    if (v >= total) return;
    const int lane = (int)(v % 64);
    const int64_t tile = v / 64;
    const int64_t kb = tile % nkb, cb = tile / nkb;
    const int col = lane % 32, g = lane / 32;
    const int b = (int)(cb * 32 + col);
    const int64_t kk = kb * 8 + g * 4;     // first of 4 consecutive contraction indices
    const int l = (int)(kk / ncp);
    const int c0 = (int)(kk % ncp);
    f32x4 w = {0.0f, 0.0f, 0.0f, 0.0f};
    if (b < L && l < r) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t q = (int64_t)(c0 + e) * L - b;
            float acc = 0.0f;
            for (int u = 0; u < L; ++u) {
                const int64_t n = q + u;
                if (n >= 0 && n < N) {
                    const float kv = reverse ? k[N - 1 - n] : k[n];
                    acc += DT[u * L + l] * kv;
                }
            }
            w[e] = acc;
        }
    }
    *reinterpret_cast<f32x4*>(out + v * 16) = w;
}

// ---- step 3: the reduced cross-correlation ------------------------------------
template <int WM, int WN, int WAVES_M, int WAVES_N>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N) void xcorr_kernel(
    const float* __restrict__ sc, int64_t nbp, const char* __restrict__ Kp, int64_t k_nrb, int64_t k_nkb,
    int64_t nkb, int ncp, int L, int64_t nout, float* __restrict__ y, int64_t tiles_m, int64_t ntiles)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave % WAVES_M, wn = wave / WAVES_M;
    const int64_t tile = blockIdx.x;
    const int64_t tm = tile % tiles_m, tn = tile / tiles_m;
    const int64_t rb0 = (tm * WAVES_M + wm) * WM;
    const int64_t cb0 = (tn * WAVES_N + wn) * WN;
    const int row = lane & 31, g = lane >> 5;

    // Projections are visited from the highest l down to l = 0, each into a
    // fresh partial accumulator that is then added to the total: the many
    // small high-order products are summed among themselves before they meet
    // the large low-order ones (blocked summation, no extra memory traffic).
    f32x16 tot[WM][WN], acc[WM][WN];
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b)
#pragma unroll
            for (int j = 0; j < 16; ++j) tot[a][b][j] = acc[a][b][j] = 0.0f;

    const char* kp[WN];
    bool kv[WN];
#pragma unroll
    for (int b = 0; b < WN; ++b) {
        kv[b] = cb0 + b < k_nrb;
        kp[b] = Kp + ((kv[b] ? cb0 + b : 0) * k_nkb * 64 + lane) * 16;
    }

    // k-block visited at step s: projection r-1 - s / kpl, block s % kpl
    const int64_t kpl = ncp / 8;
    const int64_t r = nkb / kpl;
    auto kb_of = [&](int64_t st) { return (r - 1 - st / kpl) * kpl + st % kpl; };

    auto load = [&](int64_t kb, f32x4 (&xf)[WM], f32x4 (&yf)[WN]) {
        const int64_t kk = kb * 8;
        const int64_t l = kk / ncp;
        const int64_t c0 = kk - l * ncp;
        const float* base = sc + l * nbp + c0 + 4 * g + row;
#pragma unroll
        for (int a = 0; a < WM; ++a) {
            const float* p = base + (rb0 + a) * 32;
            xf[a] = f32x4{p[0], p[1], p[2], p[3]};
        }
#pragma unroll
        for (int b = 0; b < WN; ++b)
            yf[b] = kv[b] ? *reinterpret_cast<const f32x4*>(kp[b] + kb * 1024) : f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    };

    f32x4 xc[WM], yc[WN];
    if (nkb > 0) load(kb_of(0), xc, yc);
    for (int64_t st = 0; st < nkb; ++st) {
        f32x4 xn[WM], yn[WN];
        if (st + 1 < nkb) load(kb_of(st + 1), xn, yn);
#pragma unroll
        for (int a = 0; a < WM; ++a)
#pragma unroll
            for (int b = 0; b < WN; ++b) {
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(xc[a][0], yc[b][0], acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(xc[a][1], yc[b][1], acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(xc[a][2], yc[b][2], acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(xc[a][3], yc[b][3], acc[a][b], 0, 0, 0);
            }
        if (st % kpl == kpl - 1) {
#pragma unroll
            for (int a = 0; a < WM; ++a)
#pragma unroll
                for (int b = 0; b < WN; ++b)
#pragma unroll
                    for (int j = 0; j < 16; ++j) {
                        tot[a][b][j] += acc[a][b][j];
                        acc[a][b][j] = 0.0f;
                    }
        }
        if (st + 1 < nkb) {
#pragma unroll
            for (int a = 0; a < WM; ++a) xc[a] = xn[a];
#pragma unroll
            for (int b = 0; b < WN; ++b) yc[b] = yn[b];
        }
    }

#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int64_t ar = (rb0 + a) * 32 + 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
                const int64_t bc = (cb0 + b) * 32 + (lane & 31);
                const int64_t m = ar * L + bc;
                if (bc < L && m < nout) y[m] = tot[a][b][j];
            }
}

constexpr int XW_M = 2, XW_N = 2, XWAVES_M = 2, XWAVES_N = 2;
constexpr int XBM = 32 * XW_M * XWAVES_M;

}  // namespace

// Geometry shared by the workspace query and the launcher.
ConvGeom conv_geom(int64_t W, int64_t N, int L, int r)
{
    ConvGeom g;
    g.nout = W - N + 1;
    g.nc = (N + L - 2) / L + 1;
    g.ncp = rup(g.nc, 8);
    g.rows = cdiv(g.nout, L);                       // output rows a
    g.tiles_m = cdiv(g.rows, XBM);
    g.nbp = rup(g.tiles_m * XBM + g.ncp, 64);       // projected-signal row length
    g.k_nrb = cdiv(L, 32);
    g.k_nkb = (int64_t)r * g.ncp / 8;
    g.sc_bytes = rup((int64_t)r * g.nbp * 4, 256);
    g.k_bytes = g.k_nrb * g.k_nkb * 1024;
    g.total = g.sc_bytes + g.k_bytes;
    return g;
}

int launch_conv(const ConvArgs& a, hipStream_t st)
{
    const ConvGeom g = conv_geom(a.W, a.N, a.L, a.r);
    float* sc = (float*)a.ws;
    char* kp = (char*)a.ws + g.sc_bytes;
    // step 1
    {
        int LR = 1;
        while (LR < a.r) LR *= 2;
        const int BG = 256 / LR;
        const int bpt = (int)cdiv(kSigBlocks, BG);
        dim3 grid((unsigned)cdiv(g.nbp, kSigBlocks));
        const size_t lds = (size_t)kSigBlocks * (a.L + 1) * sizeof(float);
#define SIG_LAUNCH(B)                                                                                        \
    hipLaunchKernelGGL(sig_project_kernel<B>, grid, dim3(256), lds, st, a.s, a.W, a.L, a.r, LR, a.C, sc, g.nbp)
        if (bpt <= 1) SIG_LAUNCH(1);
        else if (bpt <= 2) SIG_LAUNCH(2);
        else if (bpt <= 4) SIG_LAUNCH(4);
        else if (bpt <= 8) SIG_LAUNCH(8);
        else if (bpt <= 16) SIG_LAUNCH(16);
        else SIG_LAUNCH(32);
#undef SIG_LAUNCH
        if (hipGetLastError() != hipSuccess) return -1;
    }
    // step 2
    {
        const int64_t lanes = g.k_nrb * g.k_nkb * 64;
        hipLaunchKernelGGL(kmat_pack_kernel, dim3((unsigned)cdiv(lanes, 256)), dim3(256), 0, st, a.k, (int)a.N,
                           a.reverse, a.L, a.r, (int)g.ncp, a.DT, kp, g.k_nrb, g.k_nkb);
        if (hipGetLastError() != hipSuccess) return -1;
    }
    // step 3
    {
        const int64_t tiles_n = cdiv(g.k_nrb, (int64_t)XWAVES_N * XW_N);
        const int64_t ntiles = g.tiles_m * tiles_n;
        hipLaunchKernelGGL((xcorr_kernel<XW_M, XW_N, XWAVES_M, XWAVES_N>), dim3((unsigned)ntiles),
                           dim3(64 * XWAVES_M * XWAVES_N), 0, st, sc, g.nbp, kp, g.k_nrb, g.k_nkb, g.k_nkb,
                           (int)g.ncp, a.L, g.nout, a.y, g.tiles_m, ntiles);
        if (hipGetLastError() != hipSuccess) return -1;
    }
    return 0;
}

}  // namespace pj
