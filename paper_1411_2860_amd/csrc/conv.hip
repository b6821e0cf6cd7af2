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
#include <algorithm>

#include "conv.h"

namespace pj {

namespace {

constexpr int kMaxConvL = 256;   // largest block length the library accepts

// Steps 1 and 2 are small dense contractions over the L samples of a block
// (resp. the L taps of a phase) and run on the FP32 matrix cores: one wave
// computes a 32 x 32 tile (32 projections x 32 blocks, resp. 32 lags) with
// 32x32x2 MFMAs, 8 contraction indices per lane step (lane half g takes
// indices 4g .. 4g + 3 of each group of 8, element e in MFMA number e).

// Copies the 32 columns l0 .. l0 + 31 of an L x L row-major FP32 matrix into
// LDS as [row][32] (rows up to the next multiple of 8 of L, zeros past L and
// past column r), with every load of a thread issued before its first store.
template <int NT>
__device__ __forceinline__ void stage_slice(const float* __restrict__ M, int L, int r, int l0, float* __restrict__ S)
{
    constexpr int SPT = kMaxConvL * 32 / NT;
    const int tid = threadIdx.x;
    const int lim = ((L + 7) / 8) * 8 * 32;
    float v[SPT];
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int idx = tid + j * NT;
        const int t = idx / 32, l = idx % 32;
        v[j] = (t < L && l0 + l < r) ? M[(int64_t)t * L + l0 + l] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int idx = tid + j * NT;
        if (idx < lim) S[idx] = v[j];
    }
}

// ---- step 1: block projection of the signal ---------------------------------
// sc_l[i] = sum_t C[t, l] s[iL + t]: A = C^T (32 projections from the LDS copy
// of C[:, l0 : l0 + 32]), B = the blocks (lane = block; its samples stream
// through a 4-deep register ring, 16 bytes at a time when aligned).
// Accumulator register j of a lane holds projection 8 (j / 4) + 4 g + (j % 4)
// of block lane % 32, so each register writes 32 consecutive entries of one
// row sc_l[.].
template <bool VEC>
__device__ __forceinline__ f32x4 sig_chunk(const float* __restrict__ s, int64_t W, int L, int64_t nb, int ch, int g)
{
    f32x4 v = {0.0f, 0.0f, 0.0f, 0.0f};
    const int t = 8 * ch + 4 * g;
    const int64_t n = nb + t;
    if (VEC && t + 3 < L && n + 3 < W) {
        v = *reinterpret_cast<const f32x4*>(s + n);
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (t + e < L && n + e < W) ? s[n + e] : 0.0f;
    }
    return v;
}

// The same projection for a few projections (r <= 4; at 8 the shuffles cost
// more than the strided tile below) and L a power of two
// in 4 .. 256: one 16-byte chunk per lane covers 256 consecutive samples per
// wave step, i.e. 256 / L whole blocks; lane j holds samples (4j mod L) ..
// +3 of its block, multiplies them with its 4 x R coefficients (the same in
// every step, loaded once), and the L / 4 lanes of a block combine their
// partial sums with xor shuffles.  Each wave takes steps wave, wave + nwaves,
// ... with the loads PD steps ahead; every load is unconditional (past the
// signal: a valid address, the values masked), so the wait counts stay
// exact.  The chunk that straddles the end of a signal whose length is not a
// multiple of 4 is read as zeros here; sig_tail_kernel recomputes that block.
constexpr int kFewPD = 4;
// (body of workgroup bx of nblk; a launch of its own or the first part of
// project_pair_kernel)
template <int R>
__device__ __forceinline__ void sig_few_body(const float* __restrict__ s, int64_t W, int L, int r,
                                             const float* __restrict__ C, float* __restrict__ sc, int64_t nbp,
                                             int64_t nstep, int64_t bx, int64_t nblk)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = bx * 4 + (threadIdx.x >> 6);
    const int64_t nwaves = nblk * 4;
    const int t = (4 * lane) & (L - 1);
    const int lg = L / 4;                        // lanes per block
    const int bpi = 256 / L;                     // blocks per step
    float c[4][R];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int l = 0; l < R; ++l) c[q][l] = l < r ? C[(int64_t)(t + q) * L + l] : 0.0f;
    const int64_t nk = wave < nstep ? (nstep - wave + nwaves - 1) / nwaves : 0;   // this wave's steps
    auto load = [&](int64_t k) -> f32x4 {
        const int64_t e = (wave + k * nwaves) * 256 + 4 * lane;
        const bool full = k < nk && e + 3 < W;
        const f32x4 v = *reinterpret_cast<const f32x4*>(s + (full ? e : 0));
        return full ? v : f32x4{0.f, 0.f, 0.f, 0.f};
    };
    f32x4 ring[kFewPD];
#pragma unroll
    for (int d = 0; d < kFewPD; ++d) ring[d] = load(d);
    for (int64_t k0 = 0; k0 < nk; k0 += kFewPD) {
#pragma unroll
        for (int d = 0; d < kFewPD; ++d) {
            const int64_t k = k0 + d;
            const f32x4 x = ring[d];
            ring[d] = load(k + kFewPD);
            float p[R];
#pragma unroll
            for (int l = 0; l < R; ++l) p[l] = x[0] * c[0][l] + x[1] * c[1][l] + x[2] * c[2][l] + x[3] * c[3][l];
            for (int off = lg / 2; off > 0; off >>= 1)
#pragma unroll
                for (int l = 0; l < R; ++l) p[l] += __shfl_xor(p[l], off, 64);
            const int64_t blk = (wave + k * nwaves) * bpi + lane / lg;
            if (k < nk && (lane & (lg - 1)) == 0 && blk < nbp) {
#pragma unroll
                for (int l = 0; l < R; ++l)
                    if (l < r) sc[(int64_t)l * nbp + blk] = p[l];
            }
        }
    }
}

template <int R>
__global__ __launch_bounds__(256) void sig_project_few_kernel(const float* __restrict__ s, int64_t W, int L, int r,
                                                              const float* __restrict__ C, float* __restrict__ sc,
                                                              int64_t nbp, int64_t nstep)
{
    sig_few_body<R>(s, W, L, r, C, sc, nbp, nstep, blockIdx.x, gridDim.x);
}

// Block (W - 1) / L recomputed from all its samples (zeros past W), for a
// signal whose last 16-byte chunk sig_project_few_kernel read as zeros.
__global__ __launch_bounds__(64) void sig_tail_kernel(const float* __restrict__ s, int64_t W, int L, int r,
                                                      const float* __restrict__ C, float* __restrict__ sc,
                                                      int64_t nbp)
{
    const int64_t blk = (W - 1) / L;
    const int l = threadIdx.x;
    if (l >= r || blk >= nbp) return;
    float acc = 0.0f;
    for (int t = 0; t < L; ++t) {
        const int64_t n = blk * L + t;
        if (n < W) acc += s[n] * C[(int64_t)t * L + l];
    }
    sc[(int64_t)l * nbp + blk] = acc;
}

// The NW = 4 waves of a workgroup share its 32 blocks and split the
// contraction over t: wave w takes chunks [w ncw, (w + 1) ncw) of 8 samples
// (4 per lane half), issues every load of its range before its first matrix
// instruction (one memory latency, and a chain of at most L / 8 matrix
// instructions instead of L / 2), and the four partial tiles are added in LDS
// in a fixed order (highest wave first); wave q then writes accumulator
// registers 4q .. 4q + 3.
constexpr int kSplitNW = 4;
__device__ __forceinline__ f32x16 split_sum(f32x4 (*red)[4][64], const f32x16& acc, int wave, int lane)
{
    __syncthreads();      // the previous tile's sums have been read
#pragma unroll
    for (int q = 0; q < 4; ++q)
        red[wave][q][lane] = f32x4{acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]};
    __syncthreads();
    f32x4 v = red[kSplitNW - 1][wave][lane];
#pragma unroll
    for (int w = kSplitNW - 2; w >= 0; --w) v += red[w][wave][lane];
    f32x16 out;
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e] = v[e];
    return out;     // registers 4 wave .. 4 wave + 3 of the summed tile, in out[0 .. 3]
}

// With fewer than four chunks per block (L <= 24) the split would idle waves:
// SPLIT = false gives each wave its own 32 blocks and the whole contraction.
template <bool VEC, bool SPLIT>
__global__ __launch_bounds__(64 * kSplitNW) void sig_project_kernel(
    const float* __restrict__ s, int64_t W, int L, int r, const float* __restrict__ C,
    float* __restrict__ sc, int64_t nbp)
{
    constexpr int MAXC = kMaxConvL / 8 / kSplitNW;   // chunks per wave
    __shared__ float Cs[kMaxConvL * 32];              // [t][l - l0]
    __shared__ f32x4 red[kSplitNW][4][64];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row = lane & 31, g = lane >> 5;
    const int l0 = blockIdx.y * 32;
    const int64_t i0 = ((int64_t)blockIdx.x * (SPLIT ? 1 : kSplitNW) + (SPLIT ? 0 : wave)) * 32;
    const int nch = (L + 7) / 8;
    const int ncw = SPLIT ? (nch + kSplitNW - 1) / kSplitNW : nch;
    const int cb = SPLIT ? wave * ncw : 0;
    const int64_t nb = (i0 + row) * L;
    static_assert(SPLIT || 3 <= MAXC, "unsplit blocks have at most 3 chunks");

    f32x4 x[MAXC];
#pragma unroll
    for (int j = 0; j < MAXC; ++j)
        x[j] = (j < ncw && cb + j < nch) ? sig_chunk<VEC>(s, W, L, nb, cb + j, g) : f32x4{0.f, 0.f, 0.f, 0.f};
    stage_slice<64 * kSplitNW>(C, L, r, l0, Cs);
    __syncthreads();

    f32x16 acc;
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = 0.0f;
#pragma unroll
    for (int j = 0; j < MAXC; ++j) {
        if (j < ncw && cb + j < nch) {
            const float* cp = &Cs[(8 * (cb + j) + 4 * g) * 32 + row];
#pragma unroll
            for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(cp[32 * e], x[j][e], acc, 0, 0, 0);
        }
    }
    const int64_t i = i0 + row;
    if constexpr (SPLIT) {
        const f32x16 sum = split_sum(red, acc, wave, lane);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int jj = 4 * wave + e;
            const int l = l0 + 8 * (jj >> 2) + 4 * g + (jj & 3);
            if (l < r && i < nbp) sc[(int64_t)l * nbp + i] = sum[e];
        }
    } else {
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
            const int l = l0 + 8 * (jj >> 2) + 4 * g + (jj & 3);
            if (l < r && i < nbp) sc[(int64_t)l * nbp + i] = acc[jj];
        }
    }
}

// ---- step 2: kernel projected at every phase, packed as the right operand ---
// kd_l[q] = sum_u D[l, u] k'(q + u) for the lags q = e - (L - 1), e < ncp L:
// A = D (32 projections from the LDS copy of D^T[:, l0 : l0 + 32]), B = the
// Hankel matrix of k' (lane = lag, its 4 taps read from the LDS window of
// k').  Lag q is phase b = L - 1 - (e mod L) of kernel block c = e / L; the
// result goes straight to the packed right operand (fragment order, FP32
// tiles of 32 rows x 8): row b, contraction index l * ncp + c.
// NT x 32 lags per workgroup on independent accumulators (NT = 4 with more
// than 32 projections, where the grid has several projection tiles already
// and the staged slice of D then serves 128 lags); its four waves split the
// contraction over u as the signal projection above does.
// LC = columns of D staged: 32 (a whole projection tile), or 4 when r <= 4
// (the matrix rows l >= 4 then read zeros from registers, and the LDS of the
// workgroup shrinks from 50 KB to 22 KB).
template <int NT, int LC>
__device__ __forceinline__ void kphase_body(const float* __restrict__ k, int64_t N, int reverse, int L, int r,
                                            int64_t ncp, const float* __restrict__ DT, char* __restrict__ out,
                                            int64_t k_nkb, int64_t bx, int by)
{
    constexpr int KS = 32 * NT + kMaxConvL + 8;
    constexpr int KPT = (KS + 64 * kSplitNW - 1) / (64 * kSplitNW);
    static_assert(LC == 32 || LC == 4, "staged columns of D");
    __shared__ float Ds[kMaxConvL * LC];          // [u][l - l0], l - l0 < LC
    __shared__ float Ks[KS];                      // k'(qlo + x)
    __shared__ f32x4 red[kSplitNW][4][64];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int row = lane & 31, g = lane >> 5;
    const int l0 = by * 32;
    const int64_t e0 = bx * 32 * NT;
    const int64_t qlo = e0 - (L - 1);
    const int nch = (L + 7) / 8;
    const int ncw = (nch + kSplitNW - 1) / kSplitNW;
    const int cb = wave * ncw;

    float kv[KPT];
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
        const int idx = tid + j * 64 * kSplitNW;
        const int64_t n = qlo + idx;
        kv[j] = (idx < 32 * NT + nch * 8 && n >= 0 && n < N) ? (reverse ? k[N - 1 - n] : k[n]) : 0.0f;
    }
    if constexpr (LC == 32) {
        stage_slice<64 * kSplitNW>(DT, L, r, l0, Ds);
    } else {
        constexpr int SPT = kMaxConvL * LC / (64 * kSplitNW);
        float v[SPT];
#pragma unroll
        for (int j = 0; j < SPT; ++j) {
            const int idx = tid + j * 64 * kSplitNW;
            const int t = idx / LC, l = idx % LC;
            v[j] = (t < L && l0 + l < r) ? DT[(int64_t)t * L + l0 + l] : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < SPT; ++j) {
            const int idx = tid + j * 64 * kSplitNW;
            if (idx < nch * 8 * LC) Ds[idx] = v[j];
        }
    }
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
        const int idx = tid + j * 64 * kSplitNW;
        if (idx < 32 * NT + nch * 8) Ks[idx] = kv[j];
    }
    __syncthreads();

    f32x16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int j = 0; j < 16; ++j) acc[t][j] = 0.0f;
    for (int ch = cb; ch < cb + ncw && ch < nch; ++ch) {
        const float* dp = &Ds[(8 * ch + 4 * g) * LC + (LC == 32 ? row : (row & (LC - 1)))];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float a = (LC == 32 || row < LC) ? dp[LC * e] : 0.0f;
#pragma unroll
            for (int t = 0; t < NT; ++t)   // lane's lag of tile t, tap 8 ch + 4 g + e
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, Ks[32 * t + row + 8 * ch + 4 * g + e], acc[t], 0,
                                                              0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const f32x16 sum = split_sum(red, acc[t], wave, lane);
        const int64_t e = e0 + 32 * t + row;
        if (e >= ncp * L) continue;
        const int64_t c = e / L;
        const int b = L - 1 - (int)(e - c * L);
        const int64_t cbk = b / 32;
        const int bl = b % 32;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int jj = 4 * wave + q;
            const int l = l0 + 8 * (jj >> 2) + 4 * g + (jj & 3);
            if (l >= r) continue;
            const int64_t kk = (int64_t)l * ncp + c;
            const int ln = bl + 32 * (int)((kk % 8) / 4);
            const int64_t off = ((cbk * k_nkb + kk / 8) * 64 + ln) * 16 + (kk % 4) * 4;
            *reinterpret_cast<float*>(out + off) = sum[q];
        }
    }
}

template <int NT>
__global__ __launch_bounds__(64 * kSplitNW) void kphase_kernel(
    const float* __restrict__ k, int64_t N, int reverse, int L, int r, int64_t ncp, const float* __restrict__ DT,
    char* __restrict__ out, int64_t k_nkb)
{
    kphase_body<NT, 32>(k, N, reverse, L, r, ncp, DT, out, k_nkb, blockIdx.x, blockIdx.y);
}

// Both projections of a full-rate call with few projections in one launch:
// workgroups [0, nsig) run the signal pass (sig_few_body), the others one
// 32-lag tile of kernel phases each.  The two are independent and each alone
// leaves most of the chip idle; a second stream joined by events would cost
// more than either.
template <int R>
__global__ __launch_bounds__(256) void project_pair_kernel(const float* __restrict__ s, int64_t W, int L, int r,
                                                           const float* __restrict__ C, float* __restrict__ sc,
                                                           int64_t nbp, int64_t nstep, int64_t nsig,
                                                           const float* __restrict__ k, int64_t N, int reverse,
                                                           int64_t ncp, const float* __restrict__ DT,
                                                           char* __restrict__ out, int64_t k_nkb)
{
    if ((int64_t)blockIdx.x < nsig)
        sig_few_body<R>(s, W, L, r, C, sc, nbp, nstep, blockIdx.x, nsig);
    else
        kphase_body<1, 4>(k, N, reverse, L, r, ncp, DT, out, k_nkb, (int64_t)blockIdx.x - nsig, 0);
}

// Zero fill (16-byte stores) of the packed kernel operand, needed when L is
// not a multiple of 32 and the last row tile has padding rows b >= L.
__global__ __launch_bounds__(256) void zero16_kernel(f32x4* __restrict__ p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
}

// ---- step 3: the reduced cross-correlation ------------------------------------
// Workgroup tile: BM output rows a x BN phases b, for one contiguous range of
// k-blocks (the split; several splits raise the number of workgroups when
// the tiles alone do not fill the chip).  The contraction
// index is kk = l ncp + c (ncp a multiple of 4), in k-blocks of 8: each half
// (4 consecutive kernel blocks c0 .. c0 + 3 of one projection l) has its own
// Hankel window sc_l[a0 + c0 .. a0 + c0 + BM + 4) in LDS, next to the BN x 8
// slice of the packed kernel operand, double buffered, one barrier per
// k-block.  A lane's A fragment is sc_l[a + c0 + e], e < 4, from the window
// of its half g = lane / 32 (rows a = lane % 32 of the block), matching the
// packed B lanes.
template <int WM, int WN, int WAVES_M, int WAVES_N>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N) void xcorr_kernel(
    const float* __restrict__ sc, int64_t nbp, const char* __restrict__ Kp, int64_t k_nrb, int64_t k_nkb,
    int64_t ncp, int r, int nsplit, int L, int64_t nout, float* __restrict__ y, float* __restrict__ part,
    int64_t tiles_m)
{
    constexpr int NT = 64 * WAVES_M * WAVES_N;
    constexpr int BMB = WM * WAVES_M, BNB = WN * WAVES_N;
    constexpr int BM = 32 * BMB;
    constexpr int AW = BM + 4;                      // window of one half k-block
    constexpr int NCH = BNB * 64;
    constexpr int B_PER_T = (NCH + NT - 1) / NT;
    constexpr int A_PER_T = (2 * AW + NT - 1) / NT;
    __shared__ __align__(16) f32x4 Bs[2][NCH];
    __shared__ float As[2][2 * AW];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave % WAVES_M, wn = wave / WAVES_M;
    const int64_t tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
    const int sp = blockIdx.y;
    const int64_t kkt = (int64_t)r * ncp;                  // valid contraction indices
    const int64_t kb_lo = k_nkb * sp / nsplit, kb_hi = k_nkb * (sp + 1) / nsplit;
    const int64_t nst = kb_hi - kb_lo;
    const int64_t a0 = tm * BM;
    const int row = lane & 31, g = lane >> 5;

    // B chunk sources (k-block offset added per step)
    const char* bsrc[B_PER_T];
    bool bok[B_PER_T];
#pragma unroll
    for (int i = 0; i < B_PER_T; ++i) {
        const int c = tid + i * NT;
        const int blk = c / 64, lc = c % 64;
        const int64_t cb = tn * BNB + blk;
        bok[i] = c < NCH && cb < k_nrb;
        bsrc[i] = Kp + ((bok[i] ? cb : 0) * k_nkb * 64 + lc) * 16;
    }
    // two register sets: the loads of step st + 2 are issued while step st is
    // contracted (two k-blocks of work to hide each global load behind)
    f32x4 bst0[B_PER_T], bst1[B_PER_T];
    float ast0[A_PER_T], ast1[A_PER_T];
    // step st: k-block kb = kb_hi - 1 - st (highest projections first); half
    // g holds indices kk = 8 kb + 4 g .. + 3 (zeros past r ncp).  The steps
    // are loaded in order, so each staged value tracks its (l, c0) by
    // stepping kk down by 8.
    int64_t tkk[A_PER_T], tl[A_PER_T], tc[A_PER_T];
#pragma unroll
    for (int i = 0; i < A_PER_T; ++i) {
        const int x = tid + i * NT;
        tkk[i] = 8 * (kb_hi - 1) + 4 * (x >= AW ? 1 : 0);
        tl[i] = tkk[i] >= 0 ? tkk[i] / ncp : 0;
        tc[i] = tkk[i] - tl[i] * ncp;
    }
    auto gload = [&](int64_t st, float (&ast)[A_PER_T], f32x4 (&bst)[B_PER_T]) {
        const int64_t kb = kb_hi - 1 - st;
#pragma unroll
        for (int i = 0; i < A_PER_T; ++i) {
            const int x = tid + i * NT;
            const int xi = x >= AW ? x - AW : x;
            ast[i] = x < 2 * AW && tkk[i] < kkt ? sc[tl[i] * nbp + a0 + tc[i] + xi] : 0.0f;
            tkk[i] -= 8;
            tc[i] -= 8;
            while (tc[i] < 0 && tl[i] > 0) {
                tc[i] += ncp;
                --tl[i];
            }
        }
#pragma unroll
        for (int i = 0; i < B_PER_T; ++i)
            bst[i] = bok[i] ? *reinterpret_cast<const f32x4*>(bsrc[i] + kb * 1024) : f32x4{0.f, 0.f, 0.f, 0.f};
    };
    auto swrite = [&](int s, const float (&ast)[A_PER_T], const f32x4 (&bst)[B_PER_T]) {
#pragma unroll
        for (int i = 0; i < A_PER_T; ++i) {
            const int x = tid + i * NT;
            if (x < 2 * AW) As[s][x] = ast[i];
        }
#pragma unroll
        for (int i = 0; i < B_PER_T; ++i) {
            const int c = tid + i * NT;
            if (c < NCH) Bs[s][c] = bst[i];
        }
    };

    // One FP32 accumulator per output over the whole contraction, highest
    // projection first: with an energy-compacting basis the small high-order
    // products are summed before the large low-order ones.
    f32x16 acc[WM][WN];
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b)
#pragma unroll
            for (int j = 0; j < 16; ++j) acc[a][b][j] = 0.0f;

    auto step = [&](int64_t st, float (&la)[A_PER_T], f32x4 (&lb)[B_PER_T], const float (&sa)[A_PER_T],
                    const f32x4 (&sb)[B_PER_T]) {
        const int s = (int)(st & 1);
        if (st + 2 < nst) gload(st + 2, la, lb);
        f32x4 xf[WM], yf[WN];
#pragma unroll
        for (int a = 0; a < WM; ++a) {
            const float* p = &As[s][g * AW + (wm * WM + a) * 32 + row];
            xf[a] = f32x4{p[0], p[1], p[2], p[3]};
        }
#pragma unroll
        for (int b = 0; b < WN; ++b) yf[b] = Bs[s][(wn * WN + b) * 64 + lane];
#pragma unroll
        for (int a = 0; a < WM; ++a)
#pragma unroll
            for (int b = 0; b < WN; ++b) {
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(xf[a][0], yf[b][0], acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(xf[a][1], yf[b][1], acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(xf[a][2], yf[b][2], acc[a][b], 0, 0, 0);
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(xf[a][3], yf[b][3], acc[a][b], 0, 0, 0);
            }
        if (st + 1 < nst) swrite(s ^ 1, sa, sb);
        __syncthreads();
    };
    if (nst > 0) {
        gload(0, ast0, bst0);
        swrite(0, ast0, bst0);
    }
    if (nst > 1) gload(1, ast1, bst1);
    __syncthreads();
    for (int64_t st = 0; st < nst; st += 2) {
        step(st, ast0, bst0, ast1, bst1);
        if (st + 1 < nst) step(st + 1, ast1, bst1, ast0, bst0);
    }

    float* dst = nsplit == 1 ? y : part + (int64_t)sp * nout;
#pragma unroll
    for (int a = 0; a < WM; ++a)
#pragma unroll
        for (int b = 0; b < WN; ++b)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int64_t ar = a0 + (wm * WM + a) * 32 + 8 * (j >> 2) + 4 * g + (j & 3);
                const int64_t bc = (tn * BNB + wn * WN + b) * 32 + row;
                const int64_t m = ar * L + bc;
                if (bc < L && m < nout) dst[m] = acc[a][b][j];
            }
}

// Circular mode: the projected blocks of a periodic signal repeat, so the
// rows are completed by copying: sc_l[i] = sc_l[i mod nb0] for nb0 <= i < nbp.
__global__ __launch_bounds__(256) void wrap_kernel(float* __restrict__ sc, int64_t nbp, int64_t nb0, int r)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t span = nbp - nb0;
    if (e >= (int64_t)r * span) return;
    const int64_t l = e / span, i = nb0 + e % span;
    sc[l * nbp + i] = sc[l * nbp + i % nb0];
}

// Blocks of at most kSmallL samples use the vector-ALU path of corr.hip (a
// 32-phase matrix-core tile would be mostly padding there).
constexpr int kSmallL = 8;

// Sum of the split partials, highest projection range first.
__global__ __launch_bounds__(256) void split_sum_kernel(const float* __restrict__ part, int nsplit, int64_t nout,
                                                        float* __restrict__ y)
{
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (m >= nout) return;
    float v = part[(int64_t)(nsplit - 1) * nout + m];
    for (int s = nsplit - 2; s >= 0; --s) v += part[(int64_t)s * nout + m];
    y[m] = v;
}

// Tile shapes by block length, so that the phase tile covers the L phases
// with at most half of it padding: 128 rows x 256 phases (8 waves) for
// L > 128, 128 x 128 for L > 64, 128 x 64 for L > 32 and 256 x 32 for L <= 32
// (4 waves each).
constexpr int xcorr_bm(int L) { return L <= 32 ? 256 : 128; }
constexpr int xcorr_bnb(int L) { return L > 128 ? 8 : L > 64 ? 4 : L > 32 ? 2 : 1; }
// Splits of the contraction: enough for one workgroup per CU (256) with at
// least 32 k-blocks each, and up to 512 workgroups with at least 64 each
// (more splits cost a pass over their partial outputs).
constexpr int kXcorrFillWG = 256, kXcorrFillSteps = 32;
constexpr int kXcorrTargetWG = 512, kXcorrMinSteps = 64;

}  // namespace

// Geometry shared by the workspace query and the launcher.
ConvGeom conv_geom(int64_t W, int64_t N, int L, int r)
{
    ConvGeom g;
    g.nout = W - N + 1;
    g.nc = (N + L - 2) / L + 1;
    g.ncp = rup(g.nc, 4);
    g.rows = cdiv(g.nout, L);                       // output rows a
    g.k_nrb = cdiv(L, 32);
    g.k_nkb = cdiv((int64_t)r * g.ncp, 8);
    g.tiles_n = cdiv(g.k_nrb, xcorr_bnb(L));
    g.small = L <= kSmallL;
    // row tile: halved when the grid (tiles x contraction ranges) would not
    // give every CU a workgroup (few projections: short contractions, no split)
    auto split_of = [&](int64_t tiles) {
        const int64_t t1 = std::max<int64_t>(1, tiles);
        const int64_t fill = std::min<int64_t>(cdiv(kXcorrFillWG, t1), g.k_nkb / kXcorrFillSteps);
        const int64_t more = std::min<int64_t>(kXcorrTargetWG / t1, g.k_nkb / kXcorrMinSteps);
        return std::min<int64_t>(std::max<int64_t>(1, std::max(fill, more)), r);
    };
    int bm = xcorr_bm(L);
    g.half_m = cdiv(g.rows, bm) * g.tiles_n * split_of(cdiv(g.rows, bm) * g.tiles_n) < 256;
    if (g.half_m) bm /= 2;
    g.tiles_m = cdiv(g.rows, bm);
    g.nbp = rup(g.tiles_m * bm + g.ncp, 64);        // projected-signal row length
    const int64_t ns = split_of(g.tiles_m * g.tiles_n);
    g.nsplit = g.small ? 1 : (int)ns;
    if (g.small) {       // everything happens inside the workgroups (corr.hip)
        g.sc_bytes = g.k_bytes = g.part_bytes = 0;
        g.total = 256;
        return g;
    }
    g.sc_bytes = rup((int64_t)r * g.nbp * 4, 256);
    g.k_bytes = g.k_nrb * g.k_nkb * 1024;
    g.part_bytes = g.nsplit > 1 ? rup((int64_t)g.nsplit * g.nout * 4, 256) : 0;
    g.total = g.sc_bytes + g.k_bytes + g.part_bytes;
    return g;
}

// Step 1 for both rates: sc_l[i] for l < r, i < nbp.
static int launch_sig_project(const ConvArgs& a, float* sc, int64_t nbp, hipStream_t st);
int launch_conv_signal_rows(const ConvArgs& a, float* sc, int64_t nbp, hipStream_t st)
{
    return launch_sig_project(a, sc, nbp, st);
}
// The signal pass of few projections (sig_project_few_kernel) applies: r <= 4,
// L a power of two >= 4, a 16-byte aligned signal.
static bool few_signal_pass(const ConvArgs& a)
{
    return a.L <= kMaxConvL && a.L % 4 == 0 && ((uintptr_t)a.s % 16) == 0 && a.r <= 4 && a.L >= 4 &&
           (a.L & (a.L - 1)) == 0;
}

static int launch_sig_project(const ConvArgs& a, float* sc, int64_t nbp, hipStream_t st)
{
    if (a.L > kMaxConvL) return -2;
    const bool vec = a.L % 4 == 0 && ((uintptr_t)a.s % 16) == 0;
    if (few_signal_pass(a)) {
        // few projections: coalesced 16-byte chunks, partial sums combined
        // across the lanes of a block (the 32 x 32 MFMA tile below reads the
        // blocks strided and leaves most of the chip idle at this size)
        const int64_t nstep = cdiv(nbp * a.L, 256);
        const int64_t grid = std::max<int64_t>(1, cdiv(nstep, 4 * kFewPD));
        if (grid > 0x7fffffff) return -2;
#define PJ_FEW(R_)                                                                                              \
    hipLaunchKernelGGL((sig_project_few_kernel<R_>), dim3((unsigned)grid), dim3(256), 0, st, a.s, a.W, a.L, a.r, \
                       a.C, sc, nbp, nstep)
        if (a.r == 1) PJ_FEW(1);
        else if (a.r == 2) PJ_FEW(2);
        else PJ_FEW(4);
#undef PJ_FEW
        if (hipGetLastError() != hipSuccess) return -1;
        if (a.W % 4 != 0) {
            hipLaunchKernelGGL(sig_tail_kernel, dim3(1), dim3(64), 0, st, a.s, a.W, a.L, a.r, a.C, sc, nbp);
            if (hipGetLastError() != hipSuccess) return -1;
        }
        return 0;
    }
    const bool split = (a.L + 7) / 8 >= kSplitNW;
    dim3 grid((unsigned)cdiv(nbp, split ? 32 : 32 * kSplitNW), (unsigned)cdiv(a.r, 32));
#define PJ_SP(V, S) hipLaunchKernelGGL((sig_project_kernel<V, S>), grid, dim3(256), 0, st, a.s, a.W, a.L, a.r, a.C, sc, nbp)
    if (vec) { if (split) PJ_SP(true, true); else PJ_SP(true, false); }
    else { if (split) PJ_SP(false, true); else PJ_SP(false, false); }
#undef PJ_SP
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_conv(const ConvArgs& a, hipStream_t st)
{
    const ConvGeom g = conv_geom(a.W, a.N, a.L, a.r);
    if (g.small) {
        CorrSmallArgs c;
        c.s = a.s; c.W = a.W; c.period = a.period;
        c.k = a.k; c.N = a.N; c.reverse = a.reverse;
        c.L = a.L; c.r = a.r; c.C = a.C; c.DT = a.DT;
        c.nrows = g.rows; c.ntap = g.nc; c.nout = g.nout;
        c.y = a.y; c.block = 0;
        return launch_corr_small(c, st);
    }
    float* sc = (float*)a.ws;
    char* kp = (char*)a.ws + g.sc_bytes;
    const bool pad_kp = a.L % 32 != 0 || ((int64_t)a.r * g.ncp) % 8 != 0;
    if (a.period == 0 && few_signal_pass(a)) {
        // steps 1 and 2 in one launch (project_pair_kernel)
        if (pad_kp) {
            const int64_t n16 = g.k_nrb * g.k_nkb * 64;
            hipLaunchKernelGGL(zero16_kernel, dim3((unsigned)cdiv(n16, 256)), dim3(256), 0, st, (f32x4*)kp, n16);
            if (hipGetLastError() != hipSuccess) return -1;
        }
        const int64_t nstep = cdiv(g.nbp * a.L, 256);
        const int64_t nsig = std::max<int64_t>(1, cdiv(nstep, 4 * kFewPD));
        const int64_t nkph = cdiv(g.ncp * a.L, 32);
        if (nsig + nkph > 0x7fffffff) return -2;
#define PJ_PAIR(R_)                                                                                                  \
    hipLaunchKernelGGL((project_pair_kernel<R_>), dim3((unsigned)(nsig + nkph)), dim3(256), 0, st, a.s, a.W, a.L, a.r, \
                       a.C, sc, g.nbp, nstep, nsig, a.k, a.N, a.reverse, g.ncp, a.DT, kp, g.k_nkb)
        if (a.r == 1) PJ_PAIR(1);
        else if (a.r == 2) PJ_PAIR(2);
        else PJ_PAIR(4);
#undef PJ_PAIR
        if (hipGetLastError() != hipSuccess) return -1;
        if (a.W % 4 != 0) {
            hipLaunchKernelGGL(sig_tail_kernel, dim3(1), dim3(64), 0, st, a.s, a.W, a.L, a.r, a.C, sc, g.nbp);
            if (hipGetLastError() != hipSuccess) return -1;
        }
    } else {
        // step 1
        if (a.period > 0) {
            // periodic signal: project its W / L blocks once, then repeat them
            ConvArgs p = a;
            p.W = a.period;
            const int64_t nb0 = a.period / a.L;
            if (launch_sig_project(p, sc, g.nbp, st) != 0) return -1;
            const int64_t n = (int64_t)a.r * (g.nbp - nb0);
            if (n > 0) {
                hipLaunchKernelGGL(wrap_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, sc, g.nbp, nb0, a.r);
                if (hipGetLastError() != hipSuccess) return -1;
            }
        } else if (launch_sig_project(a, sc, g.nbp, st) != 0) {
            return -1;
        }
        // step 2
        {
            if (pad_kp) {
                // padding rows b >= L, or the unused half of the last k-block
                const int64_t n16 = g.k_nrb * g.k_nkb * 64;
                hipLaunchKernelGGL(zero16_kernel, dim3((unsigned)cdiv(n16, 256)), dim3(256), 0, st, (f32x4*)kp,
                                   n16);
                if (hipGetLastError() != hipSuccess) return -1;
            }
            // more than 32 projections: four lag tiles per workgroup share its staged slice of D
            const int nt = a.r > 32 ? 4 : 1;
            dim3 grid((unsigned)cdiv(g.ncp * a.L, 32 * nt), (unsigned)cdiv(a.r, 32));
            if (nt == 4)
                hipLaunchKernelGGL(kphase_kernel<4>, grid, dim3(256), 0, st, a.k, a.N, a.reverse, a.L, a.r, g.ncp,
                                   a.DT, kp, g.k_nkb);
            else
                hipLaunchKernelGGL(kphase_kernel<1>, grid, dim3(256), 0, st, a.k, a.N, a.reverse, a.L, a.r, g.ncp,
                                   a.DT, kp, g.k_nkb);
            if (hipGetLastError() != hipSuccess) return -1;
        }
    }
    // step 3
    {
        float* part = (float*)((char*)a.ws + g.sc_bytes + g.k_bytes);
        dim3 grid((unsigned)(g.tiles_m * g.tiles_n), (unsigned)g.nsplit);
#define PJ_XC(WM_, WN_, WA_, WB_)                                                                                 \
    hipLaunchKernelGGL((xcorr_kernel<WM_, WN_, WA_, WB_>), grid, dim3(64 * WA_ * WB_), 0, st, sc, g.nbp, kp,      \
                       g.k_nrb, g.k_nkb, g.ncp, a.r, g.nsplit, a.L, g.nout, a.y, part, g.tiles_m)
        if (a.L > 128) { if (g.half_m) PJ_XC(1, 2, 2, 4); else PJ_XC(2, 2, 2, 4); }
        else if (a.L > 64) { if (g.half_m) PJ_XC(1, 2, 2, 2); else PJ_XC(2, 2, 2, 2); }
        else if (a.L > 32) { if (g.half_m) PJ_XC(1, 1, 2, 2); else PJ_XC(2, 1, 2, 2); }
        else { if (g.half_m) PJ_XC(1, 1, 4, 1); else PJ_XC(2, 1, 4, 1); }
#undef PJ_XC
        if (hipGetLastError() != hipSuccess) return -1;
        if (g.nsplit > 1) {
            hipLaunchKernelGGL(split_sum_kernel, dim3((unsigned)cdiv(g.nout, 256)), dim3(256), 0, st, part, g.nsplit,
                               g.nout, a.y);
            if (hipGetLastError() != hipSuccess) return -1;
        }
    }
    return 0;
}

// Block rate.  Blocks of at most kSmallL samples: one launch (corr.hip).
// Longer blocks: the computed samples are
//   yd[a] = sum_c sum_t s[(a + c)L + t] sum_{l<r} C[t, l] sum_u D[l, u] k'(cL + u),
// contracted either as (s C)(D k) -- the projected signal rows against the
// projected kernel blocks, r channels -- or as s (C D k) -- the raw signal's
// L polyphase rows against the kernel blocks reconstructed from their first r
// projections, L channels and no projection of the signal.  The second is
// used when it costs fewer operations, counting the signal projection (on the
// matrix cores) at half the cost per product of the vector ALUs.
ConvBlockGeom conv_block_geom(int64_t W, int64_t N, int L, int r)
{
    ConvBlockGeom g;
    g.nout = W - N + 1;
    g.nd = (g.nout - 1) / L + 1;
    g.ncb = cdiv(N, L);
    g.ntp = rup(g.ncb, 8);
    g.nbp = rup(g.nd + g.ncb, 128);
    g.sc_bytes = g.h_bytes = g.part_bytes = 0;
    g.nsplit = 1;
    if (L <= kSmallL) {
        g.form = BF_SMALL;
        g.nch = r;
        g.total = 256;
        return g;
    }
    const bool direct = (int64_t)r * (2 * g.ncb + L) >= 2 * (int64_t)L * g.ncb;
    g.form = direct ? BF_DIRECT : BF_PROJECTED;
    g.nch = direct ? L : r;
    // enough channel ranges for about four workgroups per CU, at least 8
    // channels (two per wave) each
    const int64_t tiles = cdiv(g.nd, corr_rows_per_tile());
    int64_t ns = std::min<int64_t>(cdiv(1024, tiles), g.nch / 8);
    g.nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(ns, 64));
    // projected form: the projected signal rows; direct form: the projected
    // kernel blocks the taps are rebuilt from
    g.sc_bytes = direct ? rup((int64_t)r * g.ntp * 4, 256) : rup((int64_t)r * g.nbp * 4, 256);
    g.h_bytes = rup((int64_t)g.nch * g.ntp * 4, 256);
    g.part_bytes = rup((int64_t)g.nsplit * g.nd * 4, 256);     // per-range sums of the computed samples
    g.total = g.sc_bytes + g.h_bytes + g.part_bytes;
    return g;
}

int launch_conv_block(const ConvArgs& a, hipStream_t st)
{
    const ConvBlockGeom g = conv_block_geom(a.W, a.N, a.L, a.r);
    if (g.form == BF_SMALL) {
        CorrSmallArgs c;
        c.s = a.s; c.W = a.W; c.period = 0;
        c.k = a.k; c.N = a.N; c.reverse = a.reverse;
        c.L = a.L; c.r = a.r; c.C = a.C; c.DT = a.DT;
        c.nrows = g.nd; c.ntap = g.ncb; c.nout = g.nout;
        c.y = a.y; c.block = 1;
        return launch_corr_small(c, st);
    }
    float* sc = (float*)a.ws;
    float* h = (float*)((char*)a.ws + g.sc_bytes);
    float* part = (float*)((char*)a.ws + g.sc_bytes + g.h_bytes);
    CorrBlockArgs c;
    c.L = a.L;
    c.nch = g.nch;
    c.h = h;
    c.hld = g.ntp;
    c.nd = g.nd;
    c.nout = g.nout;
    c.nsplit = g.nsplit;
    c.part = part;
    c.y = a.y;
    if (g.form == BF_PROJECTED) {
        if (launch_sig_project(a, sc, g.nbp, st) != 0) return -1;
        if (launch_kblock_taps(a.k, a.N, a.reverse, a.L, a.r, g.ncb, g.ntp, a.DT, h, st) != 0) return -1;
        c.x = sc; c.xld = g.nbp; c.xn = g.nbp;
        return launch_corr_block(c, 0, st);
    }
    if (launch_ktilde(a.k, a.N, a.reverse, a.L, a.r, g.ncb, a.CT, a.DT, sc, h, g.ntp, st) != 0) return -1;
    c.x = a.s; c.xld = 0; c.xn = a.W;
    return launch_corr_block(c, 1, st);
}

}  // namespace pj
