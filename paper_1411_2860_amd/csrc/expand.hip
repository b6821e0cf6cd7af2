// expand.hip -- synthesis of contraction-index gradients from projected ones
// (the adjoint of the projection in the pack step).  For R = A Q_{r,K} B
// computed as R = (A C_N)(D_N B) truncated to the first r projections, the
// gradient with respect to A is dA = (dR (D_N B)^T) C_N^T restricted to those
// projections, i.e. every projected gradient value is spread back over the L
// indices of its group with the coefficients of C (B side: of D^T):
//
//   out(p, jL + t) = sum_{l<r} in(p, l*Gp + j) * coef[t, l]
//
// One thread per output element; consecutive threads take consecutive
// elements along the output's contiguous dimension.
#include "common.h"

namespace pj {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void expand_kernel(const T* __restrict__ in, int64_t ldi, int in_trans,
                                                     T* __restrict__ out, int64_t ldo, int out_trans, int64_t P,
                                                     int64_t K, int L, int r, int64_t Gp,
                                                     const T* __restrict__ coef)
{
    const int64_t fast = (int64_t)blockIdx.x * 256 + threadIdx.x;   // along the output's contiguous dim
    const int64_t slow = blockIdx.y;
    int64_t p, k;
    if (!out_trans) { p = slow; k = fast; } else { k = slow; p = fast; }
    if (p >= P || k >= K) return;
    const int64_t j = k / L;
    const int t = (int)(k - j * L);
    T acc = 0;
    for (int l = 0; l < r; ++l) {
        const int64_t kk = (int64_t)l * Gp + j;
        const T v = in_trans ? in[kk * ldi + p] : in[p * ldi + kk];
        acc += v * coef[(int64_t)t * L + l];
    }
    if (!out_trans) out[p * ldo + k] = acc;
    else out[k * ldo + p] = acc;
}

template <typename T>
int launch_t(const ExpandArgs& a, hipStream_t s)
{
    const int64_t fast = a.out_trans ? a.P : a.K;
    const int64_t slow = a.out_trans ? a.K : a.P;
    if (cdiv(fast, 256) > 0x7fffffff) return -2;
    // the grid's y dimension is limited: launch in slices of rows if needed
    // (slices of the contraction index start on group boundaries)
    const int64_t step = a.out_trans ? (65535 / a.L) * a.L : 65535;
    for (int64_t y0 = 0; y0 < slow; y0 += step) {
        const int64_t ny = (slow - y0 < step) ? slow - y0 : step;
        ExpandArgs b = a;
        if (!a.out_trans) {
            b.in = (const T*)a.in + (a.in_trans ? y0 : y0 * a.ldi);
            b.out = (T*)a.out + y0 * a.ldo;
            b.P = ny;
        } else {
            // rows of the transposed output are the contraction index k:
            // shift the group/phase bookkeeping by whole groups only
            b.out = (T*)a.out + y0 * a.ldo;
            b.in = (const T*)a.in + (a.in_trans ? (y0 / a.L) * a.ldi : (y0 / a.L));
            b.K = ny;
        }
        hipLaunchKernelGGL(expand_kernel<T>, dim3((unsigned)cdiv(fast, 256), (unsigned)ny), dim3(256), 0, s,
                           (const T*)b.in, b.ldi, b.in_trans, (T*)b.out, b.ldo, b.out_trans, b.P, b.K, b.L, b.r,
                           b.Gp, (const T*)b.coef);
        if (hipGetLastError() != hipSuccess) return -1;
    }
    return 0;
}

}  // namespace

int launch_expand(int is_double, const ExpandArgs& a, hipStream_t s)
{
    return is_double ? launch_t<double>(a, s) : launch_t<float>(a, s);
}

}  // namespace pj
