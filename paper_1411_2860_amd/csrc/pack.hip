// pack.hip -- projection during block reordering (paper Sec. III-B): the
// rows of a source matrix are cut into groups of L consecutive contraction
// indices, each group is projected onto the first r columns of a coefficient
// matrix, and the results are written straight into the MFMA fragment order
// of the packed operand (see common.h), converted to the operand format.
//
//   out[p, l*Gp + j] = sum_{t<L} X[p, j*L + t] * coef[t, l]
//
// A side: coef = C (A_c = A C_N, eq. (5), (15)).  B side: the source is B^T
// (rows = columns of B) and coef = D^T, i.e. B_d = D_N B.
//
// One workgroup owns RB source rows (one row block of the packed operand) and
// KB consecutive groups j (one k-block per projection), for every projection
// l < r.  The source tile is staged through LDS in chunks of TC indices t;
// lane (row, g) accumulates E consecutive groups for RL projections per
// chunk of work, with the coefficients read as wave-uniform scalars.  Each
// wave writes whole 64-lane tiles, so stores are fully coalesced.
#include "common.h"

namespace pj {

namespace {

constexpr int kPackThreads = 256;
constexpr int kPackLdsBytes = 60 * 1024;

template <typename T>
__device__ inline T ld_src(const T* __restrict__ X, int64_t idx) { return X[idx]; }

// ---- conversion of E accumulated values into one lane vector -------------

template <int PREC, int E, typename TIn>
__device__ inline void store_lane(char* __restrict__ out, int64_t off, int64_t plane_stride,
                                  const TIn (&v)[E])
{
    if constexpr (PREC == P_F64) {
        static_assert(E == 2, "f64 lane vector");
        f64x2 w = {v[0], v[1]};
        *reinterpret_cast<f64x2*>(out + off) = w;
    } else if constexpr (PREC == P_F32) {
        static_assert(E == 4, "f32 lane vector");
        f32x4 w = {(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
        *reinterpret_cast<f32x4*>(out + off) = w;
    } else if constexpr (PREC == P_BF16 || PREC == P_BF16X3) {
        static_assert(E == 8, "bf16 lane vector");
        bf16x8 hi, lo;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            float x = (float)v[e];
            __bf16 h = (__bf16)x;
            hi[e] = h;
            lo[e] = (__bf16)(x - (float)h);
        }
        *reinterpret_cast<bf16x8*>(out + off) = hi;
        if constexpr (PREC == P_BF16X3) *reinterpret_cast<bf16x8*>(out + plane_stride + off) = lo;
    } else if constexpr (PREC == P_F16 || PREC == P_F16X3) {
        static_assert(E == 8, "f16 lane vector");
        f16x8 hi, lo;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            float x = (float)v[e];
            _Float16 h = (_Float16)x;
            hi[e] = h;
            lo[e] = (_Float16)(x - (float)h);
        }
        *reinterpret_cast<f16x8*>(out + off) = hi;
        if constexpr (PREC == P_F16X3) *reinterpret_cast<f16x8*>(out + plane_stride + off) = lo;
    }
}

// ---- the kernel -----------------------------------------------------------
//
// Template parameters: TIn source type, PREC operand format, RL projections
// per register chunk, NCH chunks per wave per pass, TRANS source layout.
// A pass covers 4 * NCH * RL projections; passes repeat until r.
template <typename TIn, int PREC, int RL, int NCH, bool TRANS>
__global__ __launch_bounds__(kPackThreads) void pack_kernel(
    const TIn* __restrict__ X, int64_t ld, int64_t P, int64_t K, int L, int r,
    const TIn* __restrict__ coef, char* __restrict__ out, int64_t nkb, int64_t Gp,
    int64_t plane_stride, int TC, int RS)
{
    constexpr Layout ly = layout_of(PREC);
    constexpr int TR = ly.RB, KB = ly.KB, E = ly.E;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    TIn* lds = reinterpret_cast<TIn*>(smem_raw);

    const int64_t rbi = blockIdx.x;
    const int64_t p0 = rbi * TR;
    const int64_t j0 = (int64_t)blockIdx.y * KB;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int row = lane % TR, g = lane / TR;
    const int ntile = TR * KB * TC;

    for (int lp = 0; lp < r; lp += 4 * NCH * RL) {
        TIn acc[NCH][RL][E];
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int q = 0; q < RL; ++q)
#pragma unroll
                for (int e = 0; e < E; ++e) acc[c][q][e] = (TIn)0;

        for (int t0 = 0; t0 < L; t0 += TC) {
            __syncthreads();
            for (int idx = threadIdx.x; idx < ntile; idx += kPackThreads) {
                int rr, jj, tt;
                if constexpr (!TRANS) {
                    tt = idx % TC;
                    const int q = idx / TC;
                    jj = q % KB;
                    rr = q / KB;
                } else {
                    rr = idx % TR;
                    const int q = idx / TR;
                    tt = q % TC;
                    jj = q / TC;
                }
                const int64_t p = p0 + rr;
                const int64_t k = (j0 + jj) * L + t0 + tt;
                TIn v = (TIn)0;
                if (p < P && k < K) v = TRANS ? ld_src(X, k * ld + p) : ld_src(X, p * ld + k);
                lds[rr * RS + tt * KB + jj] = v;
            }
            __syncthreads();
            for (int tt = 0; tt < TC; ++tt) {
                TIn in[E];
                const TIn* src = lds + row * RS + tt * KB + g * E;
#pragma unroll
                for (int e = 0; e < E; ++e) in[e] = src[e];
                const int64_t crow = (int64_t)(t0 + tt) * L;
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    const int lb = lp + (wave + 4 * c) * RL;
#pragma unroll
                    for (int q = 0; q < RL; ++q) {
                        if (lb + q < r) {
                            const TIn cf = coef[crow + lb + q];
#pragma unroll
                            for (int e = 0; e < E; ++e) acc[c][q][e] += in[e] * cf;
                        }
                    }
                }
            }
        }

#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int lb = lp + (wave + 4 * c) * RL;
#pragma unroll
            for (int q = 0; q < RL; ++q) {
                const int l = lb + q;
                if (l < r) {
                    const int64_t kbi = ((int64_t)l * Gp + j0) / KB;
                    const int64_t off = ((rbi * nkb + kbi) * 64 + lane) * ly.LB;
                    store_lane<PREC, E, TIn>(out, off, plane_stride, acc[c][q]);
                }
            }
        }
    }
}

template <typename TIn, int PREC, int RL, int NCH>
int launch_pack_t(const PackArgs& a, hipStream_t s)
{
    constexpr Layout ly = layout_of(PREC);
    const PackGeom& g = a.geom;
    // chunk of t staged per round: a divisor of L within the LDS budget
    int tcmax = kPackLdsBytes / (int)(ly.RB * ly.KB * sizeof(TIn));
    int TC = a.L;
    if (TC > tcmax) {
        TC = tcmax;
        while (a.L % TC) --TC;
    }
    const int RS = TC * ly.KB + 2 * ly.E;   // row stride of the LDS tile (padded)
    const size_t lds = (size_t)ly.RB * RS * sizeof(TIn);
    dim3 grid((unsigned)g.nrb, (unsigned)(g.Gp / ly.KB));
    const int64_t plane_stride = g.plane_bytes + g.scale_plane;
    if (a.trans)
        hipLaunchKernelGGL((pack_kernel<TIn, PREC, RL, NCH, true>), grid, dim3(kPackThreads), lds, s,
                           (const TIn*)a.X, a.ld, a.P, a.K, a.L, a.r, (const TIn*)a.coef, (char*)a.out,
                           g.nkb, g.Gp, plane_stride, TC, RS);
    else
        hipLaunchKernelGGL((pack_kernel<TIn, PREC, RL, NCH, false>), grid, dim3(kPackThreads), lds, s,
                           (const TIn*)a.X, a.ld, a.P, a.K, a.L, a.r, (const TIn*)a.coef, (char*)a.out,
                           g.nkb, g.Gp, plane_stride, TC, RS);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename TIn, int PREC>
int launch_pack_p(const PackArgs& a, hipStream_t s)
{
    constexpr int E = layout_of(PREC).E;
    if (a.r == 1) return launch_pack_t<TIn, PREC, 1, 1>(a, s);
    if (a.r <= 16 || E > 8) return launch_pack_t<TIn, PREC, 4, 1>(a, s);
    return launch_pack_t<TIn, PREC, 4, 4>(a, s);
}

}  // namespace

int launch_pack(int prec, const PackArgs& a, hipStream_t s)
{
    switch (prec) {
    case P_F64:    return launch_pack_p<double, P_F64>(a, s);
    case P_F32:    return launch_pack_p<float, P_F32>(a, s);
    case P_BF16:   return launch_pack_p<float, P_BF16>(a, s);
    case P_BF16X3: return launch_pack_p<float, P_BF16X3>(a, s);
    case P_F16:    return launch_pack_p<float, P_F16>(a, s);
    case P_F16X3:  return launch_pack_p<float, P_F16X3>(a, s);
    default:       return -2;
    }
}

}  // namespace pj
