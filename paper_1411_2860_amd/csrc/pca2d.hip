// pca2d.hip -- the non-GEMM steps of 2D-PCA recognition (paper Sec. V-A):
// the training mean image and the centred images (eq. (22)), the symmetric
// part of the scatter matrix handed to the eigensolver (eq. (23): a Gram
// matrix, symmetric up to the rounding of its projected product), and the
// squared Frobenius distances between feature matrices that the nearest-
// neighbour decision of eq. (25)-(26) compares.
#include "pca2d.h"

namespace pj {

namespace {

// mean[e] = (1/J) sum_j X[j, e] (GIVEN = false) or read from mean (GIVEN =
// true); out[j, e] = X[j, e] - mean[e].  One thread per element e of an image
// (consecutive threads: consecutive elements, so every image row is read
// coalesced); the J values of a thread are summed in image order, then
// re-read (from the cache) for the subtraction.
template <bool GIVEN>
__global__ __launch_bounds__(256) void center_kernel(int J, int64_t mn, const float* __restrict__ X,
                                                     float* __restrict__ mean, float* __restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= mn) return;
    float m;
    if constexpr (GIVEN) {
        m = mean[e];
    } else {
        float s = 0.0f;
        for (int j = 0; j < J; ++j) s += X[(int64_t)j * mn + e];
        m = s / (float)J;
        mean[e] = m;
    }
    for (int j = 0; j < J; ++j) out[(int64_t)j * mn + e] = X[(int64_t)j * mn + e] - m;
}

// G <- (G + G^T) / 2 in place: the thread of (t, u), t < u, owns both
// entries; 16 x 16 tiles of the upper triangle, one workgroup each.
__global__ __launch_bounds__(256) void symmetrize_kernel(int n, float* __restrict__ G, int64_t ld)
{
    const int tb = blockIdx.y, ub = blockIdx.x;
    if (ub < tb) return;
    const int t = tb * 16 + threadIdx.x / 16, u = ub * 16 + threadIdx.x % 16;
    if (t >= n || u >= n || u <= t) return;
    const float a = G[(int64_t)t * ld + u], b = G[(int64_t)u * ld + t];
    const float m = 0.5f * (a + b);
    G[(int64_t)t * ld + u] = m;
    G[(int64_t)u * ld + t] = m;
}

// out[i, j] = sum_e (F[i, e] - Y[j, e])^2: one wave per (i, j), lanes along e
// (coalesced rows), partial sums combined across the wave.
__global__ __launch_bounds__(256) void sqdist_kernel(int T, int J, int64_t d, const float* __restrict__ F,
                                                     int64_t ldf, const float* __restrict__ Y, int64_t ldy,
                                                     float* __restrict__ out, int64_t ldo)
{
    const int64_t pair = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pair >= (int64_t)T * J) return;
    const int lane = threadIdx.x & 63;
    const int64_t i = pair / J, j = pair - (pair / J) * J;
    const float* f = F + i * ldf;
    const float* y = Y + j * ldy;
    float s = 0.0f;
    for (int64_t e = lane; e < d; e += 64) {
        const float df = f[e] - y[e];
        s += df * df;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) out[i * ldo + j] = s;
}

}  // namespace

int launch_center(int J, int64_t mn, const float* X, float* mean, float* out, bool given, hipStream_t s)
{
    if (cdiv(mn, 256) > 0x7fffffff) return -2;
    if (given)
        hipLaunchKernelGGL(center_kernel<true>, dim3((unsigned)cdiv(mn, 256)), dim3(256), 0, s, J, mn, X, mean, out);
    else
        hipLaunchKernelGGL(center_kernel<false>, dim3((unsigned)cdiv(mn, 256)), dim3(256), 0, s, J, mn, X, mean,
                           out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_symmetrize(int n, float* G, int64_t ld, hipStream_t s)
{
    const unsigned nb = (unsigned)cdiv(n, 16);
    hipLaunchKernelGGL(symmetrize_kernel, dim3(nb, nb), dim3(256), 0, s, n, G, ld);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_sqdist(int T, int J, int64_t d, const float* F, int64_t ldf, const float* Y, int64_t ldy, float* out,
                  int64_t ldo, hipStream_t s)
{
    const int64_t waves = (int64_t)T * J;
    if (cdiv(waves, 4) > 0x7fffffff) return -2;
    hipLaunchKernelGGL(sqdist_kernel, dim3((unsigned)cdiv(waves, 4)), dim3(256), 0, s, T, J, d, F, ldf, Y, ldy, out,
                       ldo);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace pj
