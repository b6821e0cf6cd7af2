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
#include <algorithm>

#include "common.h"

namespace pj {

namespace {

// ---- MFMA operand traits ----------------------------------------------------
template <int PREC> struct MT;

// Plain 16-byte lane vectors.
template <typename F>
__device__ __forceinline__ F load_plain(const char* plane, int64_t plane_bytes, int64_t tile, int lane)
{
    (void)plane_bytes;
    return *reinterpret_cast<const F*>(plane + (tile * 64 + lane) * 16);
}

template <> struct MT<P_F32> {
    // NMMA: matrix instructions per mma() (16-byte lane formats, for the
    // LDS ring's instruction schedule)
    static constexpr int RB = 32, NACC = 16, PLANES = 1, NMMA = 4;
    using frag = f32x4;
    using acc = f32x16;
    using out_t = float;
    __device__ __forceinline__ static frag load(const char* pl, int64_t pb, int64_t t, int lane) { return load_plain<frag>(pl, pb, t, lane); }
    __device__ __forceinline__ static void mma(acc& c, const frag (&a)[PLANES], const frag (&b)[PLANES])
    {
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][0], b[0][0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][1], b[0][1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][2], b[0][2], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][3], b[0][3], c, 0, 0, 0);
    }
};

template <> struct MT<P_F64> {
    static constexpr int RB = 16, NACC = 4, PLANES = 1, NMMA = 2;
    using frag = f64x2;
    using acc = f64x4;
    using out_t = double;
    __device__ __forceinline__ static frag load(const char* pl, int64_t pb, int64_t t, int lane) { return load_plain<frag>(pl, pb, t, lane); }
    __device__ __forceinline__ static void mma(acc& c, const frag (&a)[PLANES], const frag (&b)[PLANES])
    {
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0][0], b[0][0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0][1], b[0][1], c, 0, 0, 0);
    }
};

template <> struct MT<P_BF16> {
    static constexpr int RB = 32, NACC = 16, PLANES = 1, NMMA = 1;
    using frag = bf16x8;
    using acc = f32x16;
    using out_t = float;
    __device__ __forceinline__ static frag load(const char* pl, int64_t pb, int64_t t, int lane) { return load_plain<frag>(pl, pb, t, lane); }
    __device__ __forceinline__ static void mma(acc& c, const frag (&a)[PLANES], const frag (&b)[PLANES])
    {
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[0], c, 0, 0, 0);
    }
};

template <> struct MT<P_BF16X3> {
    static constexpr int RB = 32, NACC = 16, PLANES = 2, NMMA = 3;
    using frag = bf16x8;
    using acc = f32x16;
    using out_t = float;
    __device__ __forceinline__ static frag load(const char* pl, int64_t pb, int64_t t, int lane) { return load_plain<frag>(pl, pb, t, lane); }
    __device__ __forceinline__ static void mma(acc& c, const frag (&a)[PLANES], const frag (&b)[PLANES])
    {
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[0], c, 0, 0, 0);
    }
};

template <> struct MT<P_F16> {
    static constexpr int RB = 32, NACC = 16, PLANES = 1, NMMA = 1;
    using frag = f16x8;
    using acc = f32x16;
    using out_t = float;
    __device__ __forceinline__ static frag load(const char* pl, int64_t pb, int64_t t, int lane) { return load_plain<frag>(pl, pb, t, lane); }
    __device__ __forceinline__ static void mma(acc& c, const frag (&a)[PLANES], const frag (&b)[PLANES])
    {
        c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[0], b[0], c, 0, 0, 0);
    }
};

template <> struct MT<P_F16X3> {
    static constexpr int RB = 32, NACC = 16, PLANES = 2, NMMA = 3;
    using frag = f16x8;
    using acc = f32x16;
    using out_t = float;
    __device__ __forceinline__ static frag load(const char* pl, int64_t pb, int64_t t, int lane) { return load_plain<frag>(pl, pb, t, lane); }
    __device__ __forceinline__ static void mma(acc& c, const frag (&a)[PLANES], const frag (&b)[PLANES])
    {
        c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[1], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[0], b[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[0], b[0], c, 0, 0, 0);
    }
};

// FP8: 32-byte lane vectors of OCP e4m3 codes plus one E8M0 scale byte per
// lane (the MX scale of the 32 contraction indices the lane holds), fed to
// the block-scaled 32 x 32 x 64 matrix instruction.
struct Fp8Frag {
    i32x8 v;
    int s;
};

__device__ __forceinline__ Fp8Frag load_fp8(const char* plane, int64_t plane_bytes, int64_t tile, int lane)
{
    Fp8Frag f;
    f.v = *reinterpret_cast<const i32x8*>(plane + (tile * 64 + lane) * 32);
    f.s = (int)(unsigned char)plane[plane_bytes + tile * 64 + lane];
    return f;
}

template <> struct MT<P_FP8> {
    static constexpr int RB = 32, NACC = 16, PLANES = 1;
    using frag = Fp8Frag;
    using acc = f32x16;
    using out_t = float;
    __device__ __forceinline__ static frag load(const char* pl, int64_t pb, int64_t t, int lane) { return load_fp8(pl, pb, t, lane); }
    __device__ __forceinline__ static void mma(acc& c, const frag (&a)[PLANES], const frag (&b)[PLANES])
    {
        c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[0].v, b[0].v, c, 0, 0, 0, a[0].s, 0, b[0].s);
    }
};

template <> struct MT<P_FP8X2> {
    static constexpr int RB = 32, NACC = 16, PLANES = 2;
    using frag = Fp8Frag;
    using acc = f32x16;
    using out_t = float;
    __device__ __forceinline__ static frag load(const char* pl, int64_t pb, int64_t t, int lane) { return load_fp8(pl, pb, t, lane); }
    __device__ __forceinline__ static void mma(acc& c, const frag (&a)[PLANES], const frag (&b)[PLANES])
    {
        c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[1].v, b[0].v, c, 0, 0, 0, a[1].s, 0, b[0].s);
        c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[0].v, b[1].v, c, 0, 0, 0, a[0].s, 0, b[1].s);
        c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[0].v, b[0].v, c, 0, 0, 0, a[0].s, 0, b[0].s);
    }
};

// Output position of accumulator element j of `lane` within an RB x RB block.
template <int RB>
__device__ __forceinline__ void acc_pos(int j, int lane, int& row, int& col)
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
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t n)
{
    const int64_t x = b % 8, i = b / 8;
    const int64_t q = n / 8, rem = n % 8;
    return x * q + (x < rem ? x : rem) + i;
}

// Fragment sets in flight in the direct-load body: enough k-blocks ahead to
// cover the load latency with the matrix work of the wave's own blocks (a
// 16-bit k-block is 4x shorter on the matrix cores than an FP32 one).
template <int PREC, int WM, int WN>
constexpr int gemm_direct_depth()
{
    constexpr int blocks = WM * WN * MT<PREC>::PLANES;
    if constexpr (PREC == P_FP8X2) return 2;           // 32-byte fragments in two planes
    if constexpr (PREC == P_F32 || PREC == P_F64) return blocks >= 4 ? 2 : 4;
    return blocks >= 8 ? 2 : (blocks >= 4 ? 4 : 8);
}

// Writes a wave's WM x WN accumulator blocks (block rows from rb0, block
// columns from cb0) into R, + beta R, inside P x Q.  (Non-temporal stores
// were measured slower here.)
template <int PREC, int WM, int WN>
__device__ __forceinline__ void store_tile(const typename MT<PREC>::acc (&acc)[WM][WN], int lane, int64_t rb0,
                                           int64_t cb0, int64_t P, int64_t Q, typename MT<PREC>::out_t* __restrict__ R,
                                           int64_t ldr, float beta)
{
    using T = MT<PREC>;
    constexpr int RB = T::RB;
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

// One workgroup tile (tm, tn) of R = X Y^T: the body shared by the single
// and the grouped (persistent) launches.  Every wave streams its fragments
// through a ring of DEPTH k-block sets; all loads are unconditional (row
// blocks past the operand read row block 0: their outputs are never stored,
// and loads past the end of the contraction read k-block 0 and are never
// used), so the compiler's wait counts stay exact instead of draining every
// load at each branch.
template <int PREC, int WM, int WN, int WAVES_M, int WAVES_N>
__device__ __forceinline__ void gemm_tile(
    const char* __restrict__ X, int64_t x_nrb, int64_t x_nkb, int64_t x_plane, int64_t x_pb,
    const char* __restrict__ Y, int64_t y_nrb, int64_t y_nkb, int64_t y_plane, int64_t y_pb,
    int64_t nkb, int64_t kb_lo, int64_t P, int64_t Q, typename MT<PREC>::out_t* __restrict__ R, int64_t ldr,
    float beta, int64_t tm, int64_t tn)
{
    using T = MT<PREC>;
    using frag = typename T::frag;
    using acc_t = typename T::acc;
    constexpr int PL = T::PLANES;
    constexpr int DEPTH = gemm_direct_depth<PREC, WM, WN>();

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave % WAVES_M, wn = wave / WAVES_M;
    const int64_t rb0 = (tm * WAVES_M + wm) * WM;
    const int64_t cb0 = (tn * WAVES_N + wn) * WN;

    int64_t xt[WM], yt[WN];   // first tile index of each row block
#pragma unroll
    for (int a = 0; a < WM; ++a) xt[a] = nkb > 0 ? (rb0 + a < x_nrb ? rb0 + a : 0) * x_nkb + kb_lo : 0;
#pragma unroll
    for (int b = 0; b < WN; ++b) yt[b] = nkb > 0 ? (cb0 + b < y_nrb ? cb0 + b : 0) * y_nkb + kb_lo : 0;

    acc_t acc[WM][WN];
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b)
#pragma unroll
            for (int j = 0; j < T::NACC; ++j) acc[a][b][j] = 0;

    // The contraction runs from the last k-block to the first, i.e. from the
    // highest projection down to l = 0: with an energy-compacting basis the
    // small high-order products are accumulated before the large low-order
    // ones, which keeps the FP32 running sum accurate.  Step t contracts
    // k-block nkb - 1 - t with register set t % DEPTH, then loads step
    // t + DEPTH into it.  The loop runs whole trips of DEPTH steps with no
    // branch inside (a branch would merge unequal in-flight load counts and
    // make the compiler drain every load once per trip); the remaining
    // nkb % DEPTH steps follow it.
    const int nk = (int)nkb;                      // 32-bit step arithmetic (scalar); nkb < 2^31
    frag xf[DEPTH][WM][PL], yf[DEPTH][WN][PL];
    auto load = [&](int t, frag (&xd)[WM][PL], frag (&yd)[WN][PL]) {
        const int kb = t < nk ? nk - 1 - t : 0;
#pragma unroll
        for (int a = 0; a < WM; ++a)
#pragma unroll
            for (int pl = 0; pl < PL; ++pl) xd[a][pl] = T::load(X + pl * x_plane, x_pb, xt[a] + kb, lane);
#pragma unroll
        for (int b = 0; b < WN; ++b)
#pragma unroll
            for (int pl = 0; pl < PL; ++pl) yd[b][pl] = T::load(Y + pl * y_plane, y_pb, yt[b] + kb, lane);
    };
    auto mma_set = [&](const frag (&xd)[WM][PL], const frag (&yd)[WN][PL]) {
#pragma unroll
        for (int a = 0; a < WM; ++a)
#pragma unroll
            for (int b = 0; b < WN; ++b) T::mma(acc[a][b], xd[a], yd[b]);
    };
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) load(d, xf[d], yf[d]);
    const int nfull = nk - nk % DEPTH;
    for (int t0 = 0; t0 < nfull; t0 += DEPTH) {
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) {
            mma_set(xf[d], yf[d]);
            load(t0 + d + DEPTH, xf[d], yf[d]);
            // keep each step's loads where they are: left free, the scheduler
            // sinks them towards their use and shortens the prefetch distance
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int d = 0; d + 1 < DEPTH; ++d)
        if (d < nk - nfull) mma_set(xf[d], yf[d]);

    store_tile<PREC, WM, WN>(acc, lane, rb0, cb0, P, Q, R, ldr, beta);
}

// k-blocks staged per step of the LDS-staged tile: two where both stages
// stay within 48 KiB, which halves the barriers per contraction.
template <int PREC, int WM, int WN, int WAVES_M, int WAVES_N>
constexpr int gemm_lds_ks()
{
    return 2 * 2 * (WM * WAVES_M + WN * WAVES_N) * MT<PREC>::PLANES <= 48 ? 2 : 1;
}

// The same workgroup tile with the operands staged through LDS: per step of
// KS k-blocks the workgroup copies its BMB + BNB packed tiles per k-block
// (already in fragment order, 1 KiB per plane, so the copy is a plain
// coalesced 16-byte-per-lane stream) into one of two LDS stages while its
// waves run the matrix instructions on fragments of the other stage.  Each
// tile is fetched from L2 once per workgroup instead of once per wave.  The
// global loads run DEPTH steps ahead through a ring of register sets, all
// unconditional (as in gemm_tile) so that each wait covers exactly the set
// being parked.  16-byte lane formats only (not FP8).
template <int PREC, int WM, int WN, int WAVES_M, int WAVES_N, int DEPTH>
__device__ __forceinline__ void gemm_tile_lds(
    const char* __restrict__ X, int64_t x_nrb, int64_t x_nkb, int64_t x_plane, int64_t x_pb,
    const char* __restrict__ Y, int64_t y_nrb, int64_t y_nkb, int64_t y_plane, int64_t y_pb,
    int64_t nkb, int64_t kb_lo, int64_t P, int64_t Q, typename MT<PREC>::out_t* __restrict__ R, int64_t ldr,
    float beta, int64_t tm, int64_t tn)
{
    using T = MT<PREC>;
    using frag = typename T::frag;
    using acc_t = typename T::acc;
    constexpr int PL = T::PLANES;
    constexpr int NT = 64 * WAVES_M * WAVES_N;
    constexpr int BMB = WM * WAVES_M, BNB = WN * WAVES_N;
    constexpr int NTILE = (BMB + BNB) * PL;        // 1 KiB tiles per k-block
    constexpr int KS = gemm_lds_ks<PREC, WM, WN, WAVES_M, WAVES_N>();   // k-blocks per step
    constexpr int NCH1 = NTILE * 64;               // 16-byte chunks per k-block
    constexpr int NCH = NCH1 * KS;                 // and per step
    constexpr int PER_T = (NCH + NT - 1) / NT;
    static_assert(sizeof(frag) == 16, "LDS path is for 16-byte lane formats");
    static_assert(PER_T <= 32, "validity bits of a register set");
    (void)x_pb;
    (void)y_pb;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    f32x4* lds = reinterpret_cast<f32x4*>(smem_raw);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % WAVES_M, wn = wave / WAVES_M;
    const int64_t rbB = tm * BMB, cbB = tn * BNB;

    // chunk c = tid + i NT of a step belongs to the 1 KiB tile slot
    // u = c / 64 = wave + i NW (the same for the 64 lanes of a wave): k-block
    // kk = u / NTILE of the step, tile ti = u % NTILE = blk * PL + pl.  The
    // per-slot source (row block and plane, first k-block of the range) is
    // wave-uniform; each lane adds its 16 bytes.  Row blocks past the operand
    // read row block 0 (their outputs are never stored); slots past the step
    // read tile 0 and are dropped.
    constexpr int NW = WAVES_M * WAVES_N;
    const char* srcw[PER_T];
    int kk[PER_T];
#pragma unroll
    for (int i = 0; i < PER_T; ++i) {
        const int u = wave + i * NW;
        kk[i] = u / NTILE;
        const int ti = u % NTILE;
        const int blk = ti / PL, pl = ti % PL;
        const int64_t base = nkb > 0 ? kb_lo : 0;
        if (u * 64 >= NCH) {
            srcw[i] = X;
        } else if (blk < BMB) {
            const int64_t rb = rbB + blk;
            srcw[i] = X + pl * x_plane + ((rb < x_nrb ? rb : 0) * x_nkb + base) * 1024;
        } else {
            const int64_t cb = cbB + blk - BMB;
            srcw[i] = Y + pl * y_plane + ((cb < y_nrb ? cb : 0) * y_nkb + base) * 1024;
        }
    }
    // loads of step st: k-blocks nkb - 1 - st KS - kk (bit i of `zero` set
    // where that is below k-block 0: those chunks are parked as zeros; steps
    // past the end read k-block 0 and are never contracted)
    f32x4 stg[DEPTH][PER_T];
    unsigned zero[DEPTH];
    const int nk = (int)nkb;                      // 32-bit step arithmetic (scalar)
    const int nst = (nk + KS - 1) / KS;
    auto gload = [&](int st, f32x4 (&stage)[PER_T], unsigned& z) {
        z = 0;
#pragma unroll
        for (int i = 0; i < PER_T; ++i) {
            const int kb = nk - 1 - st * KS - kk[i];
            z |= (unsigned)(kb < 0) << i;
            stage[i] = *reinterpret_cast<const f32x4*>(srcw[i] + (int64_t)(kb < 0 ? 0 : kb) * 1024 + lane * 16);
        }
    };
    auto swrite = [&](int s, const f32x4 (&stage)[PER_T], unsigned z) {
#pragma unroll
        for (int i = 0; i < PER_T; ++i) {
            const int c = tid + i * NT;
            // zeroing by a mask (not a select, which the compiler may turn
            // into a branch per chunk)
            const int m = (z >> i) & 1 ? 0 : -1;
            if ((i + 1) * NT <= NCH || c < NCH)
                lds[s * NCH + c] = __builtin_bit_cast(f32x4, __builtin_bit_cast(i32x4, stage[i]) & m);
        }
    };

    acc_t acc[WM][WN];
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b)
#pragma unroll
            for (int j = 0; j < T::NACC; ++j) acc[a][b][j] = 0;

    // highest projection first (see gemm_tile): step st contracts k-blocks
    // nkb - 1 - st KS down to nkb - st KS - KS (a zero block past the end
    // adds exact zeros)
    auto contract = [&](int s) {
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            frag fa[WM][PL], fb[WN][PL];
            const f32x4* base = lds + s * NCH + k * NCH1;
#pragma unroll
            for (int a = 0; a < WM; ++a)
#pragma unroll
                for (int pl = 0; pl < PL; ++pl)
                    fa[a][pl] = *reinterpret_cast<const frag*>(&base[((wm * WM + a) * PL + pl) * 64 + lane]);
#pragma unroll
            for (int b = 0; b < WN; ++b)
#pragma unroll
                for (int pl = 0; pl < PL; ++pl)
                    fb[b][pl] = *reinterpret_cast<const frag*>(&base[((BMB + wn * WN + b) * PL + pl) * 64 + lane]);
#pragma unroll
            for (int a = 0; a < WM; ++a)
#pragma unroll
                for (int b = 0; b < WN; ++b) T::mma(acc[a][b], fa[a], fb[b]);
        }
    };
    // step t (LDS buffer t & 1): issue the loads of step t + DEPTH into the
    // register set that held step t (parked in LDS during step t - 1),
    // contract, then park step t + 1 in the other LDS buffer.  As in
    // gemm_tile, whole trips of DEPTH steps run without a branch (DEPTH is
    // even, so the buffer of step t0 + d is d & 1; the last trip may park a
    // step past the end, which nothing reads), then the remaining nst % DEPTH
    // steps.
    static_assert(DEPTH % 2 == 0, "LDS buffer parity per trip position");
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) gload(d, stg[d], zero[d]);
    if (nst > 0) swrite(0, stg[0], zero[0]);
    __syncthreads();
    const int nfull = nst - nst % DEPTH;
    for (int t0 = 0; t0 < nfull; t0 += DEPTH) {
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) {
            gload(t0 + d + DEPTH, stg[d], zero[d]);
            __builtin_amdgcn_sched_barrier(0);     // the loads go out before the step's matrix work
            contract(d & 1);
            swrite((d + 1) & 1, stg[(d + 1) % DEPTH], zero[(d + 1) % DEPTH]);
            __syncthreads();
        }
    }
#pragma unroll
    for (int d = 0; d + 1 < DEPTH; ++d) {
        if (d < nst - nfull) {
            contract(d & 1);
            if (d + 1 < nst - nfull) swrite((d + 1) & 1, stg[d + 1], zero[d + 1]);
            __syncthreads();
        }
    }

    const int64_t rb0 = rbB + wm * WM, cb0 = cbB + wn * WN;
    store_tile<PREC, WM, WN>(acc, lane, rb0, cb0, P, Q, R, ldr, beta);
}

// The LDS-staged tile with the copies done by the memory pipeline itself:
// each wave instruction moves one 1 KiB packed tile from global memory
// straight into a slot of the LDS ring (no registers, no LDS store
// instructions).  NS stages of KS k-blocks; the copies of step t + NS - 1 are
// issued at step t, so each has NS - 2 steps of matrix work to land behind.
// A wave waits for its own copies of the step by count, then the barrier
// makes every wave's copies visible.  Copies past the end read k-block 0 of
// their tile and are never contracted; slots below k-block 0 (the last step of
// a contraction that is not a multiple of KS) are overwritten with zeros once
// their copy has landed.
template <int PREC, int WM, int WN, int WAVES_M, int WAVES_N, int NS>
__device__ __forceinline__ void gemm_tile_dma(
    const char* __restrict__ X, int64_t x_nrb, int64_t x_nkb, int64_t x_plane, int64_t x_pb,
    const char* __restrict__ Y, int64_t y_nrb, int64_t y_nkb, int64_t y_plane, int64_t y_pb,
    int64_t nkb, int64_t kb_lo, int64_t P, int64_t Q, typename MT<PREC>::out_t* __restrict__ R, int64_t ldr,
    float beta, int64_t tm, int64_t tn)
{
    using T = MT<PREC>;
    using frag = typename T::frag;
    using acc_t = typename T::acc;
    constexpr int PL = T::PLANES;
    constexpr int NW = WAVES_M * WAVES_N;
    constexpr int BMB = WM * WAVES_M, BNB = WN * WAVES_N;
    constexpr int NTILE = (BMB + BNB) * PL;        // 1 KiB tiles per k-block
    constexpr int KS = gemm_lds_ks<PREC, WM, WN, WAVES_M, WAVES_N>();
    constexpr int NSLOT = NTILE * KS;              // tiles per step
    constexpr int PER_W = (NSLOT + NW - 1) / NW;   // copies per wave per step
    constexpr int NCH = NSLOT * 64;                // 16-byte chunks per stage
    static_assert(sizeof(frag) == 16, "LDS path is for 16-byte lane formats");
    static_assert(NSLOT % NW == 0, "every wave issues the same number of copies");
    (void)x_pb;
    (void)y_pb;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    f32x4* lds = reinterpret_cast<f32x4*>(smem_raw);

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave % WAVES_M, wn = wave / WAVES_M;
    const int64_t rbB = tm * BMB, cbB = tn * BNB;
    const char* srcw[PER_W];
    int kk[PER_W], slot[PER_W];
#pragma unroll
    for (int i = 0; i < PER_W; ++i) {
        const int u = wave + i * NW;
        slot[i] = u;
        kk[i] = u / NTILE;
        const int ti = u % NTILE;
        const int blk = ti / PL, pl = ti % PL;
        const int64_t base = nkb > 0 ? kb_lo : 0;
        if (blk < BMB) {
            const int64_t rb = rbB + blk;
            srcw[i] = X + pl * x_plane + ((rb < x_nrb ? rb : 0) * x_nkb + base) * 1024;
        } else {
            const int64_t cb = cbB + blk - BMB;
            srcw[i] = Y + pl * y_plane + ((cb < y_nrb ? cb : 0) * y_nkb + base) * 1024;
        }
    }
    const int nk = (int)nkb;
    const int nst = (nk + KS - 1) / KS;
    auto copy = [&](int st, int stage) {
#pragma unroll
        for (int i = 0; i < PER_W; ++i) {
            const int kb = nk - 1 - st * KS - kk[i];
            const char* src = srcw[i] + (int64_t)(kb < 0 ? 0 : kb) * 1024 + lane * 16;
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src),
                                             reinterpret_cast<void*>(lds + stage * NCH + slot[i] * 64), 16, 0, 0);
        }
    };
    // after the copies of step st have landed: zero the slots below k-block 0
    auto fix = [&](int st, int stage) {
#pragma unroll
        for (int i = 0; i < PER_W; ++i)
            if (nk - 1 - st * KS - kk[i] < 0) lds[stage * NCH + slot[i] * 64 + lane] = f32x4{0.f, 0.f, 0.f, 0.f};
    };

    acc_t acc[WM][WN];
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b)
#pragma unroll
            for (int j = 0; j < T::NACC; ++j) acc[a][b][j] = 0;
    auto contract = [&](int s) {
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            frag fa[WM][PL], fb[WN][PL];
            const f32x4* base = lds + s * NCH + k * NTILE * 64;
#pragma unroll
            for (int a = 0; a < WM; ++a)
#pragma unroll
                for (int pl = 0; pl < PL; ++pl)
                    fa[a][pl] = *reinterpret_cast<const frag*>(&base[((wm * WM + a) * PL + pl) * 64 + lane]);
#pragma unroll
            for (int b = 0; b < WN; ++b)
#pragma unroll
                for (int pl = 0; pl < PL; ++pl)
                    fb[b][pl] = *reinterpret_cast<const frag*>(&base[((BMB + wn * WN + b) * PL + pl) * 64 + lane]);
#pragma unroll
            for (int a = 0; a < WM; ++a)
#pragma unroll
                for (int b = 0; b < WN; ++b) T::mma(acc[a][b], fa[a], fb[b]);
        }
    };
    // step t uses stage t % NS; whole trips of NS steps (stage indices fixed
    // per trip position), then the remaining steps; every step issues its
    // NS - 1 ahead copies (clamped past the end) so the wait count is fixed
    constexpr int AHEAD = (NS - 2) * PER_W;     // copies issued after those of the step waited for
    static_assert(AHEAD < 64, "in-flight copy count");
#pragma unroll
    for (int d = 0; d + 1 < NS; ++d) copy(d, d);
    auto step = [&](int t, int d) {
        asm volatile("s_waitcnt vmcnt(%0)" ::"n"(AHEAD) : "memory");
        fix(t, d);
        // the barrier without the workgroup fence of __syncthreads(), whose
        // release would wait for every copy in flight (vmcnt(0)): ordering
        // here is explicit (own copies counted above, LDS accesses drained)
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        copy(t + NS - 1, (d + NS - 1) % NS);
        contract(d);
    };
    const int nfull = nst - nst % NS;
    for (int t0 = 0; t0 < nfull; t0 += NS) {
#pragma unroll
        for (int d = 0; d < NS; ++d) step(t0 + d, d);
    }
#pragma unroll
    for (int d = 0; d + 1 < NS; ++d)
        if (d < nst - nfull) step(nfull + d, d);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // no copy outlives the workgroup's LDS

    const int64_t rb0 = rbB + wm * WM, cb0 = cbB + wn * WN;
    store_tile<PREC, WM, WN>(acc, lane, rb0, cb0, P, Q, R, ldr, beta);
}

// The same copy ring with the fragments read one step ahead.  Without it,
// each step starts with every wave of the workgroup at the barrier and then
// waits for its LDS fragment reads before the first matrix instruction, so
// the matrix pipe idles for a read latency per step.  Here the barrier of
// step t makes stage t + 1 visible, its fragments are read into the second
// register set right away, and the matrix instructions of step t (on the
// set read during step t - 1) run while those reads are in flight.  A slot
// is refilled right after the barrier that follows its last read, so the
// copies still run NS - 2 stages ahead of the stage being waited for.
template <int PREC, int WM, int WN, int WAVES_M, int WAVES_N, int NS, int KS, bool ILV = false>
__device__ __forceinline__ void gemm_tile_dma_ra(
    const char* __restrict__ X, int64_t x_nrb, int64_t x_nkb, int64_t x_plane,
    const char* __restrict__ Y, int64_t y_nrb, int64_t y_nkb, int64_t y_plane,
    int64_t nkb, int64_t kb_lo, int64_t P, int64_t Q, typename MT<PREC>::out_t* __restrict__ R, int64_t ldr,
    float beta, int64_t tm, int64_t tn)
{
    using T = MT<PREC>;
    using frag = typename T::frag;
    using acc_t = typename T::acc;
    constexpr int PL = T::PLANES;
    constexpr int NW = WAVES_M * WAVES_N;
    constexpr int BMB = WM * WAVES_M, BNB = WN * WAVES_N;
    constexpr int NTILE = (BMB + BNB) * PL;
    constexpr int NSLOT = NTILE * KS;
    constexpr int PER_W = (NSLOT + NW - 1) / NW;
    constexpr int NCH = NSLOT * 64;
    static_assert(sizeof(frag) == 16, "LDS path is for 16-byte lane formats");
    static_assert(NSLOT % NW == 0, "every wave issues the same number of copies");
    static_assert(NS % 2 == 0, "register sets alternate with the step parity");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    f32x4* lds = reinterpret_cast<f32x4*>(smem_raw);

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wm = wave % WAVES_M, wn = wave / WAVES_M;
    const int64_t rbB = tm * BMB, cbB = tn * BNB;
    const char* srcw[PER_W];
    int kk[PER_W], slot[PER_W];
#pragma unroll
    for (int i = 0; i < PER_W; ++i) {
        const int u = wave + i * NW;
        slot[i] = u;
        kk[i] = u / NTILE;
        const int ti = u % NTILE;
        const int blk = ti / PL, pl = ti % PL;
        const int64_t base = nkb > 0 ? kb_lo : 0;
        if (blk < BMB) {
            const int64_t rb = rbB + blk;
            srcw[i] = X + pl * x_plane + ((rb < x_nrb ? rb : 0) * x_nkb + base) * 1024;
        } else {
            const int64_t cb = cbB + blk - BMB;
            srcw[i] = Y + pl * y_plane + ((cb < y_nrb ? cb : 0) * y_nkb + base) * 1024;
        }
    }
    const int nk = (int)nkb;
    const int nst = (nk + KS - 1) / KS;
    // stage st holds k-blocks nk - 1 - st KS - kk (highest first); copies past
    // k-block 0 read k-block 0 and are zeroed by fix once they have landed
    auto copy = [&](int st, int stage) {
#pragma unroll
        for (int i = 0; i < PER_W; ++i) {
            const int kb = nk - 1 - st * KS - kk[i];
            const char* src = srcw[i] + (int64_t)(kb < 0 ? 0 : kb) * 1024 + lane * 16;
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src),
                                             reinterpret_cast<void*>(lds + stage * NCH + slot[i] * 64), 16, 0, 0);
        }
    };
    auto fix = [&](int st, int stage) {
#pragma unroll
        for (int i = 0; i < PER_W; ++i)
            if (nk - 1 - st * KS - kk[i] < 0) lds[stage * NCH + slot[i] * 64 + lane] = f32x4{0.f, 0.f, 0.f, 0.f};
    };

    acc_t acc[WM][WN];
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b)
#pragma unroll
            for (int j = 0; j < T::NACC; ++j) acc[a][b][j] = 0;
    frag fa[2][KS][WM][PL], fb[2][KS][WN][PL];
    auto read = [&](int s, int set) {
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const f32x4* base = lds + s * NCH + k * NTILE * 64;
#pragma unroll
            for (int a = 0; a < WM; ++a)
#pragma unroll
                for (int pl = 0; pl < PL; ++pl)
                    fa[set][k][a][pl] = *reinterpret_cast<const frag*>(&base[((wm * WM + a) * PL + pl) * 64 + lane]);
#pragma unroll
            for (int b = 0; b < WN; ++b)
#pragma unroll
                for (int pl = 0; pl < PL; ++pl)
                    fb[set][k][b][pl] =
                        *reinterpret_cast<const frag*>(&base[((BMB + wn * WN + b) * PL + pl) * 64 + lane]);
        }
    };
    auto mmas = [&](int set) {
#pragma unroll
        for (int k = 0; k < KS; ++k)
#pragma unroll
            for (int a = 0; a < WM; ++a)
#pragma unroll
                for (int b = 0; b < WN; ++b) T::mma(acc[a][b], fa[set][k][a], fb[set][k][b]);
    };
    constexpr int AHEAD = (NS - 2) * PER_W;     // copies issued after those of the stage waited for
    static_assert((NS - 1) * PER_W < 64, "in-flight copy count");
#pragma unroll
    for (int d = 0; d < NS; ++d) copy(d, d);
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"((NS - 1) * PER_W) : "memory");
    fix(0, 0);
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    read(0, 0);
    // step t = trip start + d: slot d, register set d & 1 holding stage t
    auto step = [&](int t, int d) {
        asm volatile("s_waitcnt vmcnt(%0)" ::"n"(AHEAD) : "memory");   // own copies of stage t + 1
        fix(t + 1, (d + 1) % NS);
        // every wave's copies of stage t + 1 are in, every read of slot d is done
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        copy(t + NS, d);
        read((d + 1) % NS, (d + 1) & 1);
        mmas(d & 1);
        if constexpr (ILV) {
            constexpr int NR = KS * (WM + WN) * PL;
            constexpr int NM = KS * WM * WN * T::NMMA;
            __builtin_amdgcn_sched_group_barrier(0x020, PER_W, 0);
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, NM / NR, 0);
            }
            if constexpr (NM % NR != 0) __builtin_amdgcn_sched_group_barrier(0x008, NM % NR, 0);
        }
    };
    const int nfull = nst - nst % NS;
    for (int t0 = 0; t0 < nfull; t0 += NS) {
#pragma unroll
        for (int d = 0; d < NS; ++d) step(t0 + d, d);
    }
#pragma unroll
    for (int d = 0; d + 1 < NS; ++d)
        if (d < nst - nfull) step(nfull + d, d);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // no copy outlives the workgroup's LDS

    const int64_t rb0 = rbB + wm * WM, cb0 = cbB + wn * WN;
    store_tile<PREC, WM, WN>(acc, lane, rb0, cb0, P, Q, R, ldr, beta);
}

// Kernel body selector: KIND 0 = direct fragment loads, 1 = LDS-staged with
// loads two steps ahead, 2 = LDS-staged with loads four steps ahead, 3 = LDS
// ring filled by direct global-to-LDS copies, 4 = the same ring with the
// fragments read one step ahead, 5 = kind 4 with the step's copies issued
// first and its fragment reads interleaved one by one with its matrix
// instructions (scheduling groups), so that the LDS command queue never
// holds a whole step's reads in front of the matrix pipe.
template <int KIND, int PREC, int WM, int WN, int WAVES_M, int WAVES_N>
__device__ __forceinline__ void gemm_any(
    const char* __restrict__ X, int64_t x_nrb, int64_t x_nkb, int64_t x_plane, int64_t x_pb,
    const char* __restrict__ Y, int64_t y_nrb, int64_t y_nkb, int64_t y_plane, int64_t y_pb,
    int64_t nkb, int64_t kb_lo, int64_t P, int64_t Q, typename MT<PREC>::out_t* __restrict__ R, int64_t ldr,
    float beta, int64_t tm, int64_t tn)
{
    if constexpr (KIND == 5 && sizeof(typename MT<PREC>::frag) == 16)
        gemm_tile_dma_ra<PREC, WM, WN, WAVES_M, WAVES_N, 4, gemm_lds_ks<PREC, WM, WN, WAVES_M, WAVES_N>(), true>(
            X, x_nrb, x_nkb, x_plane, Y, y_nrb, y_nkb, y_plane, nkb, kb_lo, P, Q, R, ldr, beta, tm, tn);
    else if constexpr (KIND == 4 && sizeof(typename MT<PREC>::frag) == 16)
        gemm_tile_dma_ra<PREC, WM, WN, WAVES_M, WAVES_N, 4, gemm_lds_ks<PREC, WM, WN, WAVES_M, WAVES_N>()>(
            X, x_nrb, x_nkb, x_plane, Y, y_nrb, y_nkb, y_plane, nkb, kb_lo, P, Q, R, ldr, beta, tm, tn);
    else if constexpr (KIND == 3 && sizeof(typename MT<PREC>::frag) == 16)
        gemm_tile_dma<PREC, WM, WN, WAVES_M, WAVES_N, 4>(X, x_nrb, x_nkb, x_plane, x_pb, Y, y_nrb, y_nkb, y_plane,
                                                         y_pb, nkb, kb_lo, P, Q, R, ldr, beta, tm, tn);
    else if constexpr (KIND >= 1 && sizeof(typename MT<PREC>::frag) == 16)
        gemm_tile_lds<PREC, WM, WN, WAVES_M, WAVES_N, KIND == 2 ? 4 : 2>(X, x_nrb, x_nkb, x_plane, x_pb, Y, y_nrb,
                                                                         y_nkb, y_plane, y_pb, nkb, kb_lo, P, Q, R,
                                                                         ldr, beta, tm, tn);
    else
        gemm_tile<PREC, WM, WN, WAVES_M, WAVES_N>(X, x_nrb, x_nkb, x_plane, x_pb, Y, y_nrb, y_nkb, y_plane, y_pb,
                                                  nkb, kb_lo, P, Q, R, ldr, beta, tm, tn);
}

template <int KIND, int PREC, int WM, int WN, int WAVES_M, int WAVES_N>
constexpr size_t gemm_lds_bytes()
{
    if constexpr (KIND >= 3 && sizeof(typename MT<PREC>::frag) == 16)
        return 4ull * gemm_lds_ks<PREC, WM, WN, WAVES_M, WAVES_N>() * (WM * WAVES_M + WN * WAVES_N) *
               MT<PREC>::PLANES * 1024;
    else if constexpr (KIND >= 1 && sizeof(typename MT<PREC>::frag) == 16)
        return 2ull * gemm_lds_ks<PREC, WM, WN, WAVES_M, WAVES_N>() * (WM * WAVES_M + WN * WAVES_N) *
               MT<PREC>::PLANES * 1024;
    return 0;
}

// OCC = minimum resident workgroups per CU the register allocation must allow.
// The two-plane FP8 fragments (two 32-byte planes plus scales, double
// buffered) do not fit the 256 registers per lane of two resident waves per
// SIMD, so that format always gets the whole register file.
template <int PREC, int OCC>
constexpr int gemm_occ() { return PREC == P_FP8X2 ? 1 : OCC; }
#define PJ_GEMM_BOUNDS __launch_bounds__(64 * WAVES_M * WAVES_N, (gemm_occ<PREC, OCC>()))

template <int KIND, int PREC, int WM, int WN, int WAVES_M, int WAVES_N, int OCC>
__global__ PJ_GEMM_BOUNDS void gemm_kernel(
    const char* __restrict__ X, int64_t x_nrb, int64_t x_nkb, int64_t x_plane, int64_t x_pb,
    const char* __restrict__ Y, int64_t y_nrb, int64_t y_nkb, int64_t y_plane, int64_t y_pb,
    int64_t nkb, int64_t P, int64_t Q, typename MT<PREC>::out_t* __restrict__ R, int64_t ldr,
    float beta, int64_t tiles_m, int64_t ntiles, int nsplit, typename MT<PREC>::out_t* __restrict__ part)
{
    // grid.y = contiguous k-block ranges; with more than one, each range
    // writes its own P x Q partial and gemm_split_sum_kernel adds them
    const int64_t tile = xcd_remap(blockIdx.x, ntiles);
    const int sp = blockIdx.y;
    const int64_t lo = nkb * sp / nsplit, hi = nkb * (sp + 1) / nsplit;
    typename MT<PREC>::out_t* dst = nsplit == 1 ? R : part + (int64_t)sp * P * Q;
    gemm_any<KIND, PREC, WM, WN, WAVES_M, WAVES_N>(X, x_nrb, x_nkb, x_plane, x_pb, Y, y_nrb, y_nkb, y_plane, y_pb,
                                                   hi - lo, lo, P, Q, dst, nsplit == 1 ? ldr : Q,
                                                   nsplit == 1 ? beta : 0.0f, tile % tiles_m, tile / tiles_m);
}

// Sum of the k-range partials, highest range (highest projections) first,
// then beta R.
template <typename OT>
__global__ __launch_bounds__(256) void gemm_split_sum_kernel(const OT* __restrict__ part, int nsplit, int64_t P,
                                                             int64_t Q, OT* __restrict__ R, int64_t ldr, float beta)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= P * Q) return;
    const int64_t n = P * Q;
    OT v = part[(int64_t)(nsplit - 1) * n + e];
    for (int sp = nsplit - 2; sp >= 0; --sp) v += part[(int64_t)sp * n + e];
    const int64_t p = e / Q, q = e - p * Q;
    if (beta != 0.0f) v += (OT)beta * R[p * ldr + q];
    R[p * ldr + q] = v;
}

// Persistent grouped launch: workgroup b processes items b, b + grid, ... of
// a list of (problem, tile) items sorted by decreasing contraction length, so
// the longest tiles start first and the tail is made of short ones.  Each
// item names its body: the configuration's tile, or the small tile of one
// MFMA block per wave on the same waves (for problems whose sides the large
// tile would mostly pad).
template <int KIND, int PREC, int WM, int WN, int WAVES_M, int WAVES_N, int OCC>
__global__ PJ_GEMM_BOUNDS void gemm_grouped_kernel(
    const GroupedProblem* __restrict__ probs, const GroupedItem* __restrict__ items, int64_t nitems)
{
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const GroupedItem w = items[it];
        const GroupedProblem& p = probs[w.prob];
        if (w.body == 0)
            gemm_any<KIND, PREC, WM, WN, WAVES_M, WAVES_N>(
                (const char*)p.X, p.x_nrb, p.x_nkb, p.x_plane, p.x_pb, (const char*)p.Y, p.y_nrb, p.y_nkb,
                p.y_plane, p.y_pb, p.nkb, 0, p.P, p.Q, (typename MT<PREC>::out_t*)p.R, p.ldr, p.beta, w.tm, w.tn);
        else
            gemm_any<0, PREC, 1, 1, WAVES_M, WAVES_N>(
                (const char*)p.X, p.x_nrb, p.x_nkb, p.x_plane, p.x_pb, (const char*)p.Y, p.y_nrb, p.y_nkb,
                p.y_plane, p.y_pb, p.nkb, 0, p.P, p.Q, (typename MT<PREC>::out_t*)p.R, p.ldr, p.beta, w.tm, w.tn);
    }
}

// Dynamic LDS above the default 64 KiB has to be allowed per kernel first.
inline int raise_lds_limit(const void* kernel, size_t lds)
{
    if (lds <= 65536) return 0;
    return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) == hipSuccess ? 0 : -1;
}

template <int KIND, int PREC, int WM, int WN, int WAVES_M, int WAVES_N, int OCC>
int launch_gemm_t(const GemmArgs& a, hipStream_t s)
{
    constexpr int RB = MT<PREC>::RB;
    const int64_t tiles_m = cdiv(a.gx.nrb, (int64_t)WAVES_M * WM);
    const int64_t tiles_n = cdiv(a.gy.nrb, (int64_t)WAVES_N * WN);
    const int64_t ntiles = tiles_m * tiles_n;
    (void)RB;
    constexpr size_t lds = gemm_lds_bytes<KIND, PREC, WM, WN, WAVES_M, WAVES_N>();
    using OT = typename MT<PREC>::out_t;
    const int ns = a.nsplit > 1 && a.part ? a.nsplit : 1;
    if (raise_lds_limit((const void*)gemm_kernel<KIND, PREC, WM, WN, WAVES_M, WAVES_N, OCC>, lds) != 0) return -1;
    hipLaunchKernelGGL((gemm_kernel<KIND, PREC, WM, WN, WAVES_M, WAVES_N, OCC>), dim3((unsigned)ntiles, (unsigned)ns),
                       dim3(64 * WAVES_M * WAVES_N), lds, s,
                       (const char*)a.X, a.gx.nrb, a.gx.nkb, a.gx.plane_bytes + a.gx.scale_plane, a.gx.plane_bytes,
                       (const char*)a.Y, a.gy.nrb, a.gy.nkb, a.gy.plane_bytes + a.gy.scale_plane, a.gy.plane_bytes,
                       a.nkb, a.P, a.Q, (OT*)a.R, a.ldr, a.beta, tiles_m, ntiles, ns, (OT*)a.part);
    if (hipGetLastError() != hipSuccess) return -1;
    if (ns > 1) {
        hipLaunchKernelGGL(gemm_split_sum_kernel<OT>, dim3((unsigned)cdiv(a.P * a.Q, 256)), dim3(256), 0, s,
                           (const OT*)a.part, ns, a.P, a.Q, (OT*)a.R, a.ldr, a.beta);
        if (hipGetLastError() != hipSuccess) return -1;
    }
    return 0;
}

}  // namespace

// Tile configurations: (kind: 0 direct fragment loads, 1 - 5 LDS-staged; MFMA
// blocks per wave along M, along N; waves along M, along N; minimum resident
// workgroups per CU).  The workgroup tile is RB*WM*WAVES_M x RB*WN*WAVES_N.
// FP8 runs the LDS kinds as direct.
#define PJ_GEMM_CONFIGS(X)   \
    X(0, 0, 2, 2, 2, 2, 2)   \
    X(1, 0, 4, 2, 2, 2, 1)   \
    X(2, 0, 2, 4, 2, 2, 1)   \
    X(3, 3, 2, 4, 2, 2, 1)   \
    X(4, 0, 2, 2, 1, 1, 2)   \
    X(5, 0, 1, 1, 2, 2, 2)   \
    X(6, 1, 2, 2, 2, 2, 2)   \
    X(7, 1, 2, 4, 2, 2, 1)   \
    X(8, 1, 4, 2, 2, 2, 1)   \
    X(9, 1, 2, 2, 2, 4, 1)   \
    X(10, 1, 2, 2, 4, 2, 1)  \
    X(11, 2, 2, 2, 2, 2, 2)  \
    X(12, 3, 2, 2, 4, 2, 1)  \
    X(13, 3, 2, 2, 2, 2, 2)  \
    X(14, 3, 4, 2, 2, 2, 1)  \
    X(15, 2, 2, 2, 4, 2, 1)  \
    X(16, 4, 2, 2, 4, 2, 1)  \
    X(17, 4, 2, 2, 2, 2, 2)  \
    X(18, 5, 2, 2, 4, 2, 1)

namespace {
struct TileCfg { int wm, wn, wavm, wavn; };
constexpr TileCfg kTileCfgs[] = {
#define PJ_CFG_ROW(i, k, a, b, c, d, o) {a, b, c, d},
    PJ_GEMM_CONFIGS(PJ_CFG_ROW)
#undef PJ_CFG_ROW
};
constexpr int kNumTileCfgs = (int)(sizeof(kTileCfgs) / sizeof(kTileCfgs[0]));

template <int KIND, int PREC, int WM, int WN, int WAVES_M, int WAVES_N, int OCC>
int launch_grouped_t(const GroupedProblem* probs, const GroupedItem* items, int64_t nitems, int64_t cus,
                     hipStream_t s)
{
    constexpr size_t lds = gemm_lds_bytes<KIND, PREC, WM, WN, WAVES_M, WAVES_N>();
    const void* kern = (const void*)gemm_grouped_kernel<KIND, PREC, WM, WN, WAVES_M, WAVES_N, OCC>;
    if (raise_lds_limit(kern, lds) != 0) return -1;
    // as many persistent workgroups as the CUs hold at once (registers, LDS)
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * WAVES_M * WAVES_N, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int64_t grid = std::min<int64_t>(nitems, (int64_t)per_cu * cus);
    hipLaunchKernelGGL((gemm_grouped_kernel<KIND, PREC, WM, WN, WAVES_M, WAVES_N, OCC>), dim3((unsigned)grid),
                       dim3(64 * WAVES_M * WAVES_N), lds, s, probs, items, nitems);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int PREC>
int launch_grouped_cfg(const GroupedProblem* probs, const GroupedItem* items, int64_t nitems, int64_t cus, int cfg,
                       hipStream_t s)
{
    switch (cfg) {
#define PJ_CFG_CASE(i, k_, a_, b_, c_, d_, o_) \
    case i: return launch_grouped_t<k_, PREC, a_, b_, c_, d_, o_>(probs, items, nitems, cus, s);
        PJ_GEMM_CONFIGS(PJ_CFG_CASE)
#undef PJ_CFG_CASE
    default: return -2;
    }
}

template <int PREC>
int launch_cfg(const GemmArgs& a, int cfg, hipStream_t s)
{
    switch (cfg) {
#define PJ_CFG_CASE(i, k_, a_, b_, c_, d_, o_) \
    case i: return launch_gemm_t<k_, PREC, a_, b_, c_, d_, o_>(a, s);
        PJ_GEMM_CONFIGS(PJ_CFG_CASE)
#undef PJ_CFG_CASE
    default: return -2;
    }
}
}  // namespace

int gemm_num_configs() { return kNumTileCfgs; }

int launch_gemm_grouped(int prec, const GroupedProblem* probs, const GroupedItem* items, int64_t nitems,
                        int64_t cus, int cfg, hipStream_t s)
{
    switch (prec) {
    case P_F64:    return launch_grouped_cfg<P_F64>(probs, items, nitems, cus, cfg, s);
    case P_F32:    return launch_grouped_cfg<P_F32>(probs, items, nitems, cus, cfg, s);
    case P_BF16:   return launch_grouped_cfg<P_BF16>(probs, items, nitems, cus, cfg, s);
    case P_BF16X3: return launch_grouped_cfg<P_BF16X3>(probs, items, nitems, cus, cfg, s);
    case P_F16:    return launch_grouped_cfg<P_F16>(probs, items, nitems, cus, cfg, s);
    case P_F16X3:  return launch_grouped_cfg<P_F16X3>(probs, items, nitems, cus, cfg, s);
    case P_FP8:    return launch_grouped_cfg<P_FP8>(probs, items, nitems, cus, cfg, s);
    case P_FP8X2:  return launch_grouped_cfg<P_FP8X2>(probs, items, nitems, cus, cfg, s);
    default:       return -2;
    }
}

int gemm_config_tile(int prec, int cfg, int* tile_m, int* tile_n)
{
    if (cfg < 0 || cfg >= kNumTileCfgs) return -1;
    const int rb = layout_of(prec).RB;
    *tile_m = rb * kTileCfgs[cfg].wm * kTileCfgs[cfg].wavm;
    *tile_n = rb * kTileCfgs[cfg].wn * kTileCfgs[cfg].wavn;
    return 0;
}

int gemm_config_small_tile(int prec, int cfg, int* tile_m, int* tile_n)
{
    if (cfg < 0 || cfg >= kNumTileCfgs) return -1;
    const int rb = layout_of(prec).RB;
    *tile_m = rb * kTileCfgs[cfg].wavm;
    *tile_n = rb * kTileCfgs[cfg].wavn;
    return 0;
}

int gemm_default_config(int prec, int64_t P, int64_t Q, int64_t nkb)
{
    // small problems: smaller tiles so that the grid still covers the chip
    const int64_t tiles128 = cdiv(P, 128) * cdiv(Q, 128);
    if (tiles128 < 256) return 5;
    // (measured on the recognition and backward shapes, one timing per config)
    const bool fill256 = cdiv(P, 256) * cdiv(Q, 128) >= 256;   // 256 x 128 tiles still cover the chip
    switch (prec) {
    case P_F64: return 10;                                 // LDS, 8 waves, 128 x 64 (16 x 16 blocks)
    case P_F32:
        if (!fill256) return 0;
        return nkb >= 16 ? 18 : 10;                        // copy ring read ahead, interleaved; very short: LDS 8 waves
    case P_FP8:
    case P_FP8X2: return 9;                                // 128 x 256, 8 waves, fragments direct
    case P_BF16X3:
    case P_F16X3:
    default:                                               // BF16, FP16 and their x3 splits
        if (!fill256) return 0;                            // direct 128 x 128
        // copy ring read ahead, 256 x 128: from 64 k-blocks, or from 16 when
        // those tiles are one round on the chip (with more rounds the shorter
        // prologue of the LDS-staged 128 x 256 tile wins below 64)
        return (nkb >= 64 || (nkb >= 16 && cdiv(P, 256) * cdiv(Q, 128) <= 256)) ? 16 : 9;
    }
}

// Contiguous k-block ranges for a contraction whose tile grid alone would
// under-fill the chip (skinny outputs with a long contraction: scatter and
// Gram matrices): about 256 workgroups, at least 32 k-blocks per range.
int gemm_split_count(int prec, int64_t P, int64_t Q, int64_t nkb, int cfg)
{
    if (cfg < 0) cfg = gemm_default_config(prec, P, Q, nkb);
    int tm = 0, tn = 0;
    if (gemm_config_tile(prec, cfg, &tm, &tn) != 0) return 1;
    const int64_t tiles = cdiv(P, tm) * cdiv(Q, tn);
    if (tiles >= 128 || nkb < 64) return 1;
    int64_t ns = std::min<int64_t>(cdiv(256, tiles), nkb / 32);
    ns = std::min<int64_t>(ns, 64);
    return (int)std::max<int64_t>(ns, 1);
}

int launch_gemm(int prec, const GemmArgs& a, int cfg, hipStream_t s)
{
    if (cfg < 0) cfg = gemm_default_config(prec, a.P, a.Q, a.nkb);
    switch (prec) {
    case P_F64:    return launch_cfg<P_F64>(a, cfg, s);
    case P_F32:    return launch_cfg<P_F32>(a, cfg, s);
    case P_BF16:   return launch_cfg<P_BF16>(a, cfg, s);
    case P_BF16X3: return launch_cfg<P_BF16X3>(a, cfg, s);
    case P_F16:    return launch_cfg<P_F16>(a, cfg, s);
    case P_F16X3:  return launch_cfg<P_F16X3>(a, cfg, s);
    case P_FP8:    return launch_cfg<P_FP8>(a, cfg, s);
    case P_FP8X2:  return launch_cfg<P_FP8X2>(a, cfg, s);
    default:       return -2;
    }
}

}  // namespace pj
