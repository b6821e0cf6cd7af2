// moments.hip -- block second-moment matrix of training data, the input of
// the data-adaptive (Karhunen-Loeve / principal component) basis that the
// paper names as the alternative to fixed DCT / Haar coefficients (Sec. IV-B
// footnote, Sec. VI):
//     M[t, u] = sum_i sum_j X[i, jL + t] X[i, jL + u]
// over the aligned L-blocks of every row of a row-major FP32 matrix (K
// zero-extended to a multiple of L).
//
// Each workgroup owns a 64 x 64 tile of M and a contiguous chunk of blocks;
// 16 blocks at a time are staged in LDS, and each thread accumulates a 4 x 4
// sub-tile in FP64 (the products of two FP32 values are exact in FP64).  The
// chunk partials are summed afterwards in a fixed order.
#include "moments.h"

namespace pj {

namespace {

constexpr int kMT = 64;      // tile of M
constexpr int kGB = 16;      // blocks staged per step

__global__ __launch_bounds__(256) void moments_kernel(const float* __restrict__ X, int64_t ld, int64_t K, int L,
                                                      int64_t G, int64_t nblk, int64_t chunk, int ntile,
                                                      double* __restrict__ out)
{
    __shared__ __align__(16) float xt[kGB][kMT];
    __shared__ __align__(16) float xu[kGB][kMT];
    const int tid = threadIdx.x;
    const int ti = tid / 16, ui = tid % 16;
    const int tile = blockIdx.x;
    const int t0 = (tile / ntile) * kMT, u0 = (tile % ntile) * kMT;
    const int64_t b0 = (int64_t)blockIdx.y * chunk;
    const int64_t b1 = b0 + chunk < nblk ? b0 + chunk : nblk;

    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;

    for (int64_t g0 = b0; g0 < b1; g0 += kGB) {
        // 2 x 16 x 64 staged values, 8 per thread: (side, block, position)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int idx = tid + q * 256;
            const int side = idx / (kGB * kMT);
            const int bb = (idx / kMT) % kGB, p = idx % kMT;
            const int64_t gb = g0 + bb;
            const int t = (side == 0 ? t0 : u0) + p;
            float v = 0.0f;
            if (gb < b1 && t < L) {
                const int64_t i = gb / G, j = gb - (gb / G) * G;
                const int64_t k = j * L + t;
                if (k < K) v = X[i * ld + k];
            }
            if (side == 0) xt[bb][p] = v;
            else xu[bb][p] = v;
        }
        __syncthreads();
#pragma unroll 4
        for (int bb = 0; bb < kGB; ++bb) {
            const f32x4 a = *reinterpret_cast<const f32x4*>(&xt[bb][4 * ti]);
            const f32x4 b = *reinterpret_cast<const f32x4*>(&xu[bb][4 * ui]);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += (double)a[i] * (double)b[j];
        }
        __syncthreads();
    }
    double* o = out + (int64_t)blockIdx.y * L * L;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int t = t0 + 4 * ti + i, u = u0 + 4 * ui + j;
            if (t < L && u < L) o[(int64_t)t * L + u] = acc[i][j];
        }
}

__global__ __launch_bounds__(256) void moments_sum_kernel(const double* __restrict__ part, int nchunk, int64_t n,
                                                          double* __restrict__ M)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    double v = 0.0;
    for (int c = 0; c < nchunk; ++c) v += part[(int64_t)c * n + e];
    M[e] = v;
}

}  // namespace

MomentsGeom moments_geom(int64_t rows, int64_t K, int L)
{
    MomentsGeom g;
    g.G = cdiv(K, L);
    g.nblk = rows * g.G;
    g.ntile = (int)cdiv(L, kMT);
    const int64_t want = std::max<int64_t>(1, 512 / ((int64_t)g.ntile * g.ntile));
    g.nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(want, cdiv(g.nblk, 256)));
    g.chunk = cdiv(g.nblk, g.nchunk);
    g.ws_bytes = g.nchunk > 1 ? (int64_t)g.nchunk * L * L * 8 : 0;
    return g;
}

int launch_moments(const float* X, int64_t ld, int64_t rows, int64_t K, int L, double* M, void* ws, hipStream_t st)
{
    const MomentsGeom g = moments_geom(rows, K, L);
    double* part = g.nchunk > 1 ? (double*)ws : M;
    dim3 grid((unsigned)(g.ntile * g.ntile), (unsigned)g.nchunk);
    hipLaunchKernelGGL(moments_kernel, grid, dim3(256), 0, st, X, ld, K, L, g.G, g.nblk, g.chunk, g.ntile, part);
    if (hipGetLastError() != hipSuccess) return -1;
    if (g.nchunk > 1) {
        const int64_t n = (int64_t)L * L;
        hipLaunchKernelGGL(moments_sum_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, part, g.nchunk, n, M);
        if (hipGetLastError() != hipSuccess) return -1;
    }
    return 0;
}

}  // namespace pj
