// gemm.hip -- the reduced contraction of the projected GEMM (paper Sec. III-B:
// the (l+1) smaller products A_c B_d, summed as in eq. (8)).  Both operands
// are packed (common.h) along the same projection-major contraction
// k = l*Gp + j, so the sum over projections and groups is ONE contraction of
// length r*Gp, accumulated in the matrix-core accumulators:
//
//   R[p, q] = sum_{kb < nkb} sum_{k in kb} X[p, k] * Y[q, k]  (+ beta R[p, q])
//
// Each wave owns WM x WN MFMA blocks of RB x RB outputs and streams its
// operand tiles straight from the packed buffers (one coalesced 16-byte
// access per lane per tile), prefetching the next k-block while the matrix
// cores work on the current one.  Workgroups are mapped XCD-aware: the
// hardware deals workgroups round-robin over the 8 XCDs, so consecutive
// logical tiles are regrouped to land on the same XCD and share its L2.
#include "common.h"

namespace pj {

namespace {

// ---- MFMA operand traits ----------------------------------------------------
template <int PREC> struct MT;

template <> struct MT<P_F32> {
    static constexpr int RB = 32, NACC = 16, PLANES = 1;
    using frag = f32x4;
    using acc = f32x16;
    using out_t = float;
    __device__ static void mma(acc& c, const frag (&a)[PLANES], const frag (&b)[PLANES])
    {
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][0], b[0][0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][1], b[0][1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][2], b[0][2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][3], b[0][3], c, 0, 0, 0);
    }
};

template <> struct MT<P_F64> {
    static constexpr int RB = 16, NACC = 4, PLANES = 1;
    using frag = f64x2;
    using acc = f64x4;
    using out_t = double;
    __device__ static void mma(acc& c, const frag (&a)[PLANES], const frag (&b)[PLANES])
    {
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0][0], b[0][0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0][1], b[0][1], c, 0, 0, 0);
    }
};

template <> struct MT<P_BF16> {
    static constexpr int RB = 32, NACC = 16, PLANES = 1;
    using frag = bf16x8;
    using acc = f32x16;
    using out_t = float;
    __device__ static void mma(acc& c, const frag (&a)[PLANES], const frag (&b)[PLANES])
    {
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[0], c, 0, 0, 0);
    }
};

template <> struct MT<P_BF16X3> {
    static constexpr int RB = 32, NACC = 16, PLANES = 2;
    using frag = bf16x8;
    using acc = f32x16;
    using out_t = float;
    __device__ static void mma(acc& c, const frag (&a)[PLANES], const frag (&b)[PLANES])
    {
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[0], c, 0, 0, 0);
    }
};

template <> struct MT<P_F16> {
    static constexpr int RB = 32, NACC = 16, PLANES = 1;
    using frag = f16x8;
    using acc = f32x16;
    using out_t = float;
    __device__ static void mma(acc& c, const frag (&a)[PLANES], const frag (&b)[PLANES])
    {
        c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[0], b[0], c, 0, 0, 0);
    }
};

template <> struct MT<P_F16X3> {
    static constexpr int RB = 32, NACC = 16, PLANES = 2;
    using frag = f16x8;
    using acc = f32x16;
    using out_t = float;
    __device__ static void mma(acc& c, const frag (&a)[PLANES], const frag (&b)[PLANES])
    {
        c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[1], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[0], b[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[0], b[0], c, 0, 0, 0);
    }
};

// Output position of accumulator element j of `lane` within an RB x RB block.
template <int RB>
__device__ inline void acc_pos(int j, int lane, int& row, int& col)
{
    if constexpr (RB == 32) {
        row = 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3);
        col = lane & 31;
    } else {   // 16 x 16 FP64 block: register j of lane holds row lane/16 + 4 j
        row = (lane >> 4) + 4 * j;
        col = lane & 15;
    }
}

// XCD-aware remap of the hardware workgroup id: the dispatcher hands
// workgroup b to XCD b % 8, so logical tiles [x*n/8, (x+1)*n/8) all run on
// XCD x and share its L2.
__device__ inline int64_t xcd_remap(int64_t b, int64_t n)
{
    const int64_t x = b % 8, i = b / 8;
    const int64_t q = n / 8, rem = n % 8;
    return x * q + (x < rem ? x : rem) + i;
}

template <int PREC, int WM, int WN, int WAVES_M, int WAVES_N>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N) void gemm_kernel(
    const char* __restrict__ X, int64_t x_nrb, int64_t x_nkb, int64_t x_plane,
    const char* __restrict__ Y, int64_t y_nrb, int64_t y_nkb, int64_t y_plane,
    int64_t nkb, int64_t P, int64_t Q, typename MT<PREC>::out_t* __restrict__ R, int64_t ldr,
    float beta, int64_t tiles_m, int64_t ntiles)
{
    using T = MT<PREC>;
    using frag = typename T::frag;
    using acc_t = typename T::acc;
    constexpr int RB = T::RB, PL = T::PLANES;
    constexpr int64_t TB = 64 * 16;   // bytes per tile per plane

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave % WAVES_M, wn = wave / WAVES_M;
    const int64_t tile = xcd_remap(blockIdx.x, ntiles);
    const int64_t tm = tile % tiles_m, tn = tile / tiles_m;
    const int64_t rb0 = (tm * WAVES_M + wm) * WM;
    const int64_t cb0 = (tn * WAVES_N + wn) * WN;

    const char* xp[WM];
    const char* yp[WN];
    bool xv[WM], yv[WN];
#pragma unroll
    for (int a = 0; a < WM; ++a) {
        xv[a] = rb0 + a < x_nrb;
        xp[a] = X + ((xv[a] ? rb0 + a : 0) * x_nkb * 64 + lane) * 16;
    }
#pragma unroll
    for (int b = 0; b < WN; ++b) {
        yv[b] = cb0 + b < y_nrb;
        yp[b] = Y + ((yv[b] ? cb0 + b : 0) * y_nkb * 64 + lane) * 16;
    }

    acc_t acc[WM][WN];
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b)
#pragma unroll
            for (int j = 0; j < T::NACC; ++j) acc[a][b][j] = 0;

    frag xc[WM][PL], yc[WN][PL];
    auto load = [&](int64_t kb, frag (&xf)[WM][PL], frag (&yf)[WN][PL]) {
#pragma unroll
        for (int a = 0; a < WM; ++a)
#pragma unroll
            for (int pl = 0; pl < PL; ++pl)
                xf[a][pl] = xv[a] ? *reinterpret_cast<const frag*>(xp[a] + pl * x_plane + kb * TB) : frag{};
#pragma unroll
        for (int b = 0; b < WN; ++b)
#pragma unroll
            for (int pl = 0; pl < PL; ++pl)
                yf[b][pl] = yv[b] ? *reinterpret_cast<const frag*>(yp[b] + pl * y_plane + kb * TB) : frag{};
    };

    // The contraction runs from the last k-block to the first, i.e. from the
    // highest projection down to l = 0: with an energy-compacting basis the
    // small high-order products are accumulated before the large low-order
    // ones, which keeps the FP32 running sum accurate.
    if (nkb > 0) load(nkb - 1, xc, yc);
    for (int64_t kb = nkb - 1; kb >= 0; --kb) {
        frag xn[WM][PL], yn[WN][PL];
        if (kb > 0) load(kb - 1, xn, yn);
#pragma unroll
        for (int a = 0; a < WM; ++a)
#pragma unroll
            for (int b = 0; b < WN; ++b) T::mma(acc[a][b], xc[a], yc[b]);
        if (kb > 0) {
#pragma unroll
            for (int a = 0; a < WM; ++a)
#pragma unroll
                for (int pl = 0; pl < PL; ++pl) xc[a][pl] = xn[a][pl];
#pragma unroll
            for (int b = 0; b < WN; ++b)
#pragma unroll
                for (int pl = 0; pl < PL; ++pl) yc[b][pl] = yn[b][pl];
        }
    }

#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b)
#pragma unroll
            for (int j = 0; j < T::NACC; ++j) {
                int row, col;
                acc_pos<RB>(j, lane, row, col);
                const int64_t p = (rb0 + a) * RB + row;
                const int64_t q = (cb0 + b) * RB + col;
                if (p < P && q < Q) {
                    typename T::out_t v = (typename T::out_t)acc[a][b][j];
                    if (beta != 0.0f) v += (typename T::out_t)beta * R[p * ldr + q];
                    R[p * ldr + q] = v;
                }
            }
}

template <int PREC, int WM, int WN, int WAVES_M, int WAVES_N>
int launch_gemm_t(const GemmArgs& a, hipStream_t s)
{
    constexpr int RB = MT<PREC>::RB;
    const int64_t tiles_m = cdiv(a.gx.nrb, (int64_t)WAVES_M * WM);
    const int64_t tiles_n = cdiv(a.gy.nrb, (int64_t)WAVES_N * WN);
    const int64_t ntiles = tiles_m * tiles_n;
    (void)RB;
    hipLaunchKernelGGL((gemm_kernel<PREC, WM, WN, WAVES_M, WAVES_N>), dim3((unsigned)ntiles),
                       dim3(64 * WAVES_M * WAVES_N), 0, s,
                       (const char*)a.X, a.gx.nrb, a.gx.nkb, a.gx.plane_bytes + a.gx.scale_plane,
                       (const char*)a.Y, a.gy.nrb, a.gy.nkb, a.gy.plane_bytes + a.gy.scale_plane,
                       a.nkb, a.P, a.Q, (typename MT<PREC>::out_t*)a.R, a.ldr, a.beta, tiles_m, ntiles);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int launch_gemm(int prec, const GemmArgs& a, hipStream_t s)
{
    switch (prec) {
    case P_F64:    return launch_gemm_t<P_F64, 4, 4, 2, 2>(a, s);
    case P_F32:    return launch_gemm_t<P_F32, 2, 2, 2, 2>(a, s);
    case P_BF16:   return launch_gemm_t<P_BF16, 2, 2, 2, 2>(a, s);
    case P_BF16X3: return launch_gemm_t<P_BF16X3, 2, 2, 2, 2>(a, s);
    case P_F16:    return launch_gemm_t<P_F16, 2, 2, 2, 2>(a, s);
    case P_F16X3:  return launch_gemm_t<P_F16X3, 2, 2, 2, 2>(a, s);
    default:       return -2;
    }
}

}  // namespace pj
