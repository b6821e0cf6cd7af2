// expand.hip -- synthesis of contraction-index gradients from projected ones
// (the adjoint of the projection in the pack step).  For R = A Q_{r,K} B
// computed as R = (A C_N)(D_N B) truncated to the first r projections, the
// gradient with respect to A is dA = (dR (D_N B)^T) C_N^T restricted to those
// projections, i.e. every projected gradient value is spread back over the L
// indices of its group with the coefficients of C (B side: of D^T):
//
//   out(p, jL + t) = sum_{l<r} in(p, l*Gp + j) * coef[t, l]
//
// One thread per (p, group j) writes the L outputs of its group, 16 at a time:
// for each projection l it loads in(p, l*Gp + j) once and adds it, times the
// 16 coefficients coef[t0 .. t0 + 15, l], to 16 accumulators; the workgroup
// stages those coefficients transposed in LDS, so they arrive as 16-byte
// broadcast reads.  The thread index runs along p when the output is stored
// with p contiguous (each output is then one coalesced store per wave) and
// along (p, j), j fastest, otherwise (the workgroup then parks its groups'
// runs in LDS and 16 consecutive lanes write each run).
#include "common.h"

namespace pj {

namespace {

constexpr int kExpandChunk = 16;          // outputs of a group per pass
constexpr int kExpandMaxR = 256;

template <typename T, bool OUT_T>
__global__ __launch_bounds__(256) void expand_kernel(const T* __restrict__ in, int64_t ldi, int in_trans,
                                                     T* __restrict__ out, int64_t ldo, int64_t P, int64_t K, int L,
                                                     int r, int64_t Gp, const T* __restrict__ coef, int64_t slow0)
{
    __shared__ __align__(16) T cs[kExpandMaxR * kExpandChunk];      // [l][e] = coef[t0 + e, l]
    __shared__ T st[OUT_T ? 1 : 256 * (kExpandChunk + 1)];          // row-major output: runs re-dealt to lanes
    const int64_t fast = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t slow = slow0 + blockIdx.y;
    const int64_t G = (K + L - 1) / L;
    int64_t p, j;
    if (OUT_T) {               // (p fast, one group j per grid row)
        p = fast;
        j = slow;
    } else {                   // (p, j) flattened, j fastest
        p = fast / G;
        j = fast - p * G;
    }
    const bool live = p < P && j < G;
    const int tlim = live ? (int)((K - j * L) < L ? (K - j * L) : L) : 0;   // the last group may be partial
    // the chunk loop runs over [0, L) for every thread (it holds barriers)
    for (int t0 = 0; t0 < L; t0 += kExpandChunk) {
        __syncthreads();
        for (int x = threadIdx.x; x < r * kExpandChunk; x += 256) {
            const int l = x / kExpandChunk, e = x - l * kExpandChunk;
            cs[x] = t0 + e < L ? coef[(int64_t)(t0 + e) * L + l] : T(0);
        }
        __syncthreads();
        T acc[kExpandChunk];
#pragma unroll
        for (int e = 0; e < kExpandChunk; ++e) acc[e] = T(0);
        if (t0 < tlim)
            for (int l = 0; l < r; ++l) {
                const int64_t kk = (int64_t)l * Gp + j;
                const T v = in_trans ? in[kk * ldi + p] : in[p * ldi + kk];
                const T* c = cs + l * kExpandChunk;
#pragma unroll
                for (int e = 0; e < kExpandChunk; ++e) acc[e] += v * c[e];
            }
        if (OUT_T) {
            const int64_t k0 = j * L + t0;
#pragma unroll
            for (int e = 0; e < kExpandChunk; ++e)
                if (t0 + e < tlim) out[(k0 + e) * ldo + p] = acc[e];
        } else {
            // the workgroup's 256 groups (consecutive j, one row p) each hold a
            // run of up to 16 outputs: park them in LDS, then 16 consecutive
            // lanes write each run
#pragma unroll
            for (int e = 0; e < kExpandChunk; ++e) st[threadIdx.x * (kExpandChunk + 1) + e] = acc[e];
            __syncthreads();
            const int64_t fb = (int64_t)blockIdx.x * 256;
            for (int q = threadIdx.x; q < 256 * kExpandChunk; q += 256) {
                const int g = q / kExpandChunk, e = q - g * kExpandChunk;
                const int64_t pg = (fb + g) / G, jg = (fb + g) - pg * G;
                if (pg < P) {
                    const int64_t kq = jg * L + t0 + e;
                    if (t0 + e < L && kq < K) out[pg * ldo + kq] = st[g * (kExpandChunk + 1) + e];
                }
            }
        }
    }
}

template <typename T>
int launch_t(const ExpandArgs& a, hipStream_t s)
{
    if (a.r < 1 || a.r > kExpandMaxR || a.L < 1) return -2;
    const int64_t G = cdiv(a.K, a.L);
    const int64_t fast = a.out_trans ? a.P : a.P * G;
    const int64_t slow = a.out_trans ? G : 1;
    if (cdiv(fast, 256) > 0x7fffffff) return -2;
    // the grid's y dimension is limited: launch in slices
    for (int64_t y0 = 0; y0 < slow; y0 += 65535) {
        const int64_t ny = (slow - y0 < 65535) ? slow - y0 : 65535;
        if (a.out_trans)
            hipLaunchKernelGGL((expand_kernel<T, true>), dim3((unsigned)cdiv(fast, 256), (unsigned)ny), dim3(256), 0,
                               s, (const T*)a.in, a.ldi, a.in_trans, (T*)a.out, a.ldo, a.P, a.K, a.L, a.r, a.Gp,
                               (const T*)a.coef, y0);
        else
            hipLaunchKernelGGL((expand_kernel<T, false>), dim3((unsigned)cdiv(fast, 256), (unsigned)ny), dim3(256), 0,
                               s, (const T*)a.in, a.ldi, a.in_trans, (T*)a.out, a.ldo, a.P, a.K, a.L, a.r, a.Gp,
                               (const T*)a.coef, y0);
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
