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
// One workgroup owns TRc source rows and KB consecutive groups j (one k-block
// per projection), for every projection l < r.  The source tile is staged
// through LDS in rounds of TC indices t, in one of three round layouts:
//   0  [row][group][t] with padded strides, filled through registers
//      (16-byte or element loads);
//   1  swizzled and unpadded, filled by direct global-to-LDS loads (16 bytes
//      per lane for aligned rows, else one value per lane);
//   2  transposed ([group][t][row], rows padded), filled by single-value
//      direct loads from a transposed source.
// FP32-input tiles of 32 rows project on the FP32 matrix cores (16 x 16 x 4),
// 16 projections per pass, and return the results to the store layout
// through LDS; otherwise lane (row, g) accumulates the E consecutive groups
// of its lane vector for RL projections at a time with vector FMAs, the
// coefficients being wave-uniform scalars.  Every wave writes whole 64-lane
// tiles, so stores are fully coalesced.
//
// Both operands of a GEMM are packed by one launch (two jobs over one grid,
// so the small A side overlaps with the large B side) when they use the same
// round layout, else by one launch each.
#include <vector>

#include <algorithm>
#include <type_traits>

#include "common.h"

namespace pj {

namespace {

constexpr int kPackThreads = 256;
constexpr int kPackLdsBytes = 48 * 1024;
constexpr int kPackSwzLdsBytes = 64 * 1024;

template <typename TIn>
struct PackJob {
    const TIn* X;
    int64_t ld;
    int trans;       // 0: (p, k) at X[p*ld + k]; 1: at X[k*ld + p]
    int vec4;        // 16-byte loads allowed (k-contiguous and aligned)
    int64_t P, K;
    int L, r;
    const TIn* coef; // L x L, element (t, l)
    char* out;
    int64_t nkb, Gp, plane_stride, plane_bytes, plain_ld;
    int64_t nrb, ngt;   // row blocks, group tiles (Gp / KB)
    int64_t nrt;        // row tiles of the compute mapping
    int TC, TCp, JS, RS;
    // Swizzled round layout (FP32 input, TC / 4 a power of two): row rr of
    // the tile holds NC = KB * TC / 4 chunks of 4 values without padding,
    // chunk c = group * TC / 4 + t / 4 at slot c ^ (rr & SM), so that the
    // 16 rows read by one matrix-core step fall in distinct banks.
    int swz, lnc, ltc4, sm;
    int dma4;        // direct loads of single values (rows not 16-byte aligned)
    // Transposed round layout (FP32 transposed source): element (rr, group
    // jj, t) at (jj * TCp + t) * RT + rr, filled by single-value direct loads
    // along the contiguous rows of the source.
    int tdma, RT;
    TIn* keep;          // plain copy of the projections (nullptr: none)
    int64_t keep_ld;
};

// ---- OCP FP8 E4M3 (1 sign, 4 exponent bits with bias 7, 3 mantissa bits,
// largest finite 448, no infinities) with round-to-nearest-even; |v| <= 448.
__device__ __forceinline__ unsigned fp8_e4m3_rne(float v)
{
    const unsigned sign = (__float_as_uint(v) >> 24) & 0x80u;
    const float a = fabsf(v);
    unsigned code;
    if (a < 0.015625f) {                       // below 2^-6: subnormal steps of 2^-9
        code = (unsigned)__float2uint_rn(a * 512.0f);   // 0 .. 8 (8 = smallest normal)
    } else {
        unsigned b = __float_as_uint(a);
        b += 0x7FFFFu + ((b >> 20) & 1u);      // round the 23-bit mantissa to 3 bits
        code = ((((b >> 23) & 0xFFu) - 120u) << 3) | ((b >> 20) & 7u);
    }
    return sign | code;
}

// ---- conversion of E accumulated values into one lane vector -------------

template <int PREC, int E, typename TIn>
__device__ __forceinline__ void store_lane(char* __restrict__ out, int64_t off, int64_t plane_stride, int64_t plane_bytes,
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

// 16 bytes per lane from global memory straight into LDS: lane i writes
// dst + 4 i (dst is the same for the whole wave).
__device__ __forceinline__ void lds_direct16(const float* src, float* dst)
{
    __builtin_amdgcn_global_load_lds(src, dst, 16, 0, 0);
}

// 4 bytes per lane: lane i writes dst + i.
__device__ __forceinline__ void lds_direct4(const float* src, float* dst)
{
    __builtin_amdgcn_global_load_lds(src, dst, 4, 0, 0);
}

template <typename TIn> struct Vec4;
template <> struct Vec4<float> { using type = f32x4; };
template <> struct Vec4<double> { using type = f64x4; };

// ---- the kernel -----------------------------------------------------------
// Thread mapping of the projection: each wave covers TRc rows x KB groups,
// lane (row, g) computing Ec consecutive groups; 4 waves split the
// projections.  For FP8 a lane computes one eighth of a 64-group tile row so
// that the 4 lanes of an MX block are adjacent (their maximum is combined
// with lane shuffles).
template <int PREC> struct Cmap {
    static constexpr Layout ly = layout_of(PREC);
    static constexpr int Ec = (ly.E > 8) ? 8 : ly.E;
    static constexpr int NGc = ly.KB / Ec;
    static constexpr int TRc = 64 / NGc;
};

// The projection runs on the FP32 matrix cores (16 x 16 x 4 MFMA: 16 rows x
// 16 projections per instruction) for FP32 input, 32-row tiles and passes of
// 16 projections (as many passes as r needs); otherwise (a single
// projection, FP8's 8-row tiles, FP64) as vector FMAs.
template <typename TIn, int PREC, int RL, int NCH>
constexpr bool pack_mfma()
{
    return std::is_same<TIn, float>::value && Cmap<PREC>::TRc == 32 && 4 * NCH * RL == 16 &&
           (PREC == P_F32 || PREC == P_BF16 || PREC == P_BF16X3 || PREC == P_F16 || PREC == P_F16X3);
}

// LDS floats per projection of the transpose that returns the matrix-core
// results to the lane layout of the stores: 32 rows x KB groups, padded.
template <int PREC>
constexpr int pack_mfma_ds() { return 32 * layout_of(PREC).KB + 4; }

__device__ __forceinline__ unsigned fp8_exp_byte(float amax, float& inv, float& sc)
{
    int ex = -127;
    if (amax > 0.0f) {
        int f;
        const float m = frexpf(amax / 448.0f, &f);   // amax / 448 = m 2^f, m in [0.5, 1)
        ex = (m == 0.5f) ? f - 1 : f;                  // ceil(log2(amax / 448))
        ex = ex < -127 ? -127 : (ex > 127 ? 127 : ex);
    }
    inv = ldexpf(1.0f, -ex);
    sc = ldexpf(1.0f, ex);
    return (unsigned)(ex + 127);
}

__device__ __forceinline__ float fp8_decode(unsigned c)
{
    const unsigned mag = c & 0x7Fu;
    const float val = (mag < 8u) ? (float)mag * 0.001953125f
                                 : ldexpf(1.0f + (float)(mag & 7u) * 0.125f, (int)(mag >> 3) - 7);
    return (c & 0x80u) ? -val : val;
}

// 8 values of one MX block quarter: codes (2 words) with the block's scale;
// optionally the dequantised values.
__device__ __forceinline__ void fp8_encode8(const float* v, float inv, float sc, unsigned& w0, unsigned& w1, float* deq)
{
    w0 = w1 = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const float x = fminf(fmaxf(v[e] * inv, -448.0f), 448.0f);
        const unsigned c = fp8_e4m3_rne(x);
        if (e < 4) w0 |= c << (8 * e);
        else w1 |= c << (8 * (e - 4));
        if (deq) deq[e] = fp8_decode(c) * sc;
    }
}

__device__ __forceinline__ float quad_max(float a)
{
    a = fmaxf(a, __shfl_xor(a, 1));
    a = fmaxf(a, __shfl_xor(a, 2));
    return a;
}

// One FP8 (x2) lane quarter: lane (row, g) of the compute mapping holds
// indices 8g .. 8g+7 of a 64-index tile row, i.e. quarter g % 4 of MX block
// g / 4.  The instruction reads block h of row `row` as bytes 16h..16h+15 of
// lane row (indices 32h..32h+15) and of lane 32 + row (32h+16..32h+31).
template <int PREC>
__device__ __forceinline__ void store_fp8_quarter(char* __restrict__ out, int64_t tile, int rib, int g, int64_t plane_stride,
                                         int64_t plane_bytes, const float (&v)[8])
{
    const int h = g / 4, sub = g % 4;
    const int lane_dst = (sub < 2) ? rib : 32 + rib;
    const int64_t off = (tile * 64 + lane_dst) * 32 + 16 * h + 8 * (sub % 2);
    float amax = 0.0f;
#pragma unroll
    for (int e = 0; e < 8; ++e) amax = fmaxf(amax, fabsf(v[e]));
    amax = quad_max(amax);
    float inv, sc;
    const unsigned s = fp8_exp_byte(amax, inv, sc);
    unsigned w0, w1;
    float deq[8];
    fp8_encode8(v, inv, sc, w0, w1, PREC == P_FP8X2 ? deq : nullptr);
    *reinterpret_cast<uint2*>(out + off) = make_uint2(w0, w1);
    if (sub == 0) out[plane_bytes + tile * 64 + 32 * h + rib] = (char)s;
    if constexpr (PREC == P_FP8X2) {
        float res[8];
        float rmax = 0.0f;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            res[e] = v[e] - deq[e];
            rmax = fmaxf(rmax, fabsf(res[e]));
        }
        rmax = quad_max(rmax);
        const unsigned s2 = fp8_exp_byte(rmax, inv, sc);
        fp8_encode8(res, inv, sc, w0, w1, nullptr);
        *reinterpret_cast<uint2*>(out + plane_stride + off) = make_uint2(w0, w1);
        if (sub == 0) out[plane_stride + plane_bytes + tile * 64 + 32 * h + rib] = (char)s2;
    }
}

// LAY: round layout in LDS -- 0 padded rows (register staging), 1 swizzled
// (direct loads, rows contiguous along k), 2 transposed (direct loads from a
// transposed source).
template <typename TIn, int PREC, int RL, int NCH, int LAY>
__device__ __forceinline__ void pack_tile(const PackJob<TIn>& J, int64_t tix)
{
    constexpr Layout ly = layout_of(PREC);
    constexpr int KB = ly.KB, RB = ly.RB;
    constexpr int Ec = Cmap<PREC>::Ec, NGc = Cmap<PREC>::NGc, TRc = Cmap<PREC>::TRc;
    using V4 = typename Vec4<TIn>::type;
    // staged values per thread never exceed the LDS budget's: 16-byte groups
    // of 4 values (contiguous path) and 4 x 4 blocks (strided path)
    constexpr int kMaxV4 = kPackLdsBytes / (4 * (int)sizeof(TIn) * kPackThreads);
    constexpr int kMaxV16 = kPackLdsBytes / (16 * (int)sizeof(TIn) * kPackThreads);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    TIn* lds = reinterpret_cast<TIn*>(smem_raw);

    // tile order: along the groups of a row tile for row-contiguous sources;
    // along the rows of a group tile for a transposed source, so that the
    // workgroups in flight read neighbouring segments of the same k rows
    const int64_t rti = J.trans ? tix % J.nrt : tix / J.ngt;          // row tile of TRc rows
    const int64_t j0 = (J.trans ? tix / J.nrt : tix % J.ngt) * KB;
    const int64_t p0 = rti * TRc;
    const int64_t rbi = p0 / RB;                   // row block of the packed operand
    const int rib0 = (int)(p0 % RB);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int row = lane / NGc, g = lane % NGc;
    const int L = J.L, r = J.r, TC = J.TC, TCp = J.TCp, JS = J.JS, RS = J.RS;
    const TIn* __restrict__ X = J.X;
    using ConstTIn = const __attribute__((address_space(4))) TIn;
    ConstTIn* coefc = (ConstTIn*)(J.coef);

    // LDS element index of (row rr, group jj, index t of the round): the
    // swizzled layout with direct loads, else rows of RS with padding
    const int lnc = J.lnc, ltc4 = J.ltc4, sm = J.sm;
    auto loff = [&](int rr, int jj, int t) -> int {
        if constexpr (LAY == 1) return ((rr << lnc) + (((jj << ltc4) + (t >> 2)) ^ (rr & sm))) * 4 + (t & 3);
        else if constexpr (LAY == 2) return (jj * TCp + t) * J.RT + rr;
        else return rr * RS + jj * JS + t;
    };

    // staging of one round: t0 .. t0 + TC of every group of the tile into LDS
    auto stage = [&](int t0) {
        if constexpr (LAY == 2) {
            // transposed layout filled by single-value direct loads: 64
            // consecutive floats per wave instruction, i.e. consecutive rows
            // p of one source row k (coalesced); padding columns rr >= TRc
            // and values outside the operand (p >= P, k >= K, t >= TC) are
            // read from X itself and then overwritten with zeros
            const int RT = J.RT;
            const int tot = KB * TCp * RT;
            const int per_wave = (tot + kPackThreads - 1) / kPackThreads;
            const bool interior = p0 + TRc <= J.P && (j0 + KB - 1) * L + t0 + TC <= J.K && TC == TCp;
            auto src_of = [&](int f, bool& ok) -> const TIn* {
                const int q = f / RT, rr = f - q * RT;
                const int jj = q / TCp, t = q - jj * TCp;
                const int64_t p = p0 + rr;
                const int64_t k = (j0 + jj) * L + t0 + t;
                ok = rr < TRc && (interior || (t < TC && p < J.P && k < J.K));
                return ok ? X + k * J.ld + p : X;
            };
            for (int i = 0; i < per_wave; ++i) {
                const int f0 = (wave * per_wave + i) * 64;
                const int f = f0 + lane;
                if (f0 < tot) {
                    bool ok;
                    const TIn* src = src_of(f < tot ? f : tot - 1, ok);
                    if (f < tot) lds_direct4(src, lds + f0);
                }
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            if (!interior) {
                for (int i = 0; i < per_wave; ++i) {
                    const int f = (wave * per_wave + i) * 64 + lane;
                    if (f < tot) {
                        bool ok;
                        src_of(f, ok);
                        if (!ok) lds[f] = (TIn)0;
                    }
                }
            }
            return;
        }
        if constexpr (LAY == 1) {
            // swizzled layout filled by direct loads: the 16-byte chunks go
            // from memory straight into LDS (no registers), each wave
            // instruction filling 64 consecutive slots.  Chunks outside the
            // operand (rows >= P, indices >= K; K is a multiple of 4 here)
            // are read from X itself and then overwritten with zeros.
            const bool interior = p0 + TRc <= J.P && (j0 + KB - 1) * L + t0 + TC <= J.K;
            const TIn* __restrict__ base = X + p0 * J.ld + j0 * L + t0;
            if (J.dma4) {
                // rows not 16-byte aligned: one value per lane, 64 consecutive
                // floats of the layout per wave instruction (value e of chunk
                // slot s at float 4 s + e), validity per value
                const int per_wave4 = (TRc << lnc) * 4 / kPackThreads;
                for (int i = 0; i < per_wave4; ++i) {
                    const int f0 = (wave * per_wave4 + i) * 64;
                    const int f = f0 + lane;
                    const int rr = f >> (lnc + 2);
                    const int c = ((f >> 2) & ((1 << lnc) - 1)) ^ (rr & sm);
                    const int64_t ko = (c >> ltc4) * L + 4 * (c & ((1 << ltc4) - 1)) + (f & 3);
                    const TIn* src = base + rr * J.ld + ko;
                    if (!interior && (p0 + rr >= J.P || j0 * L + t0 + ko >= J.K)) src = X;
                    lds_direct4(src, lds + f0);
                }
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                if (!interior) {
                    for (int i = 0; i < per_wave4; ++i) {
                        const int f = (wave * per_wave4 + i) * 64 + lane;
                        const int rr = f >> (lnc + 2);
                        const int c = ((f >> 2) & ((1 << lnc) - 1)) ^ (rr & sm);
                        const int64_t ko = (c >> ltc4) * L + 4 * (c & ((1 << ltc4) - 1)) + (f & 3);
                        if (p0 + rr >= J.P || j0 * L + t0 + ko >= J.K) lds[f] = (TIn)0;
                    }
                }
                return;
            }
            const int per_wave = (TRc << lnc) / kPackThreads;
            unsigned outside = 0;
            for (int i = 0; i < per_wave; ++i) {
                const int slot0 = (wave * per_wave + i) * 64;
                const int gsl = slot0 + lane;
                const int rr = gsl >> lnc;
                const int c = (gsl & ((1 << lnc) - 1)) ^ (rr & sm);
                const int64_t ko = (c >> ltc4) * L + 4 * (c & ((1 << ltc4) - 1));
                const TIn* src = base + rr * J.ld + ko;
                if (!interior && (p0 + rr >= J.P || j0 * L + t0 + ko >= J.K)) {
                    src = X;
                    outside |= 1u << i;
                }
                lds_direct16(src, lds + slot0 * 4);
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            if (!interior) {
                for (int i = 0; i < per_wave; ++i)
                    if (outside & (1u << i))
                        *reinterpret_cast<V4*>(lds + ((wave * per_wave + i) * 64 + lane) * 4) = V4{0, 0, 0, 0};
            }
            return;
        }
        if (J.vec4 && !J.trans) {
            // 16-byte loads along the contiguous contraction index; every
            // load of a thread is issued before its first LDS store
            const int n4 = TRc * KB * (TC / 4);
            V4 buf[kMaxV4];
#pragma unroll
            for (int i = 0; i < kMaxV4; ++i) {
                const int idx = threadIdx.x + i * kPackThreads;
                buf[i] = V4{0, 0, 0, 0};
                if (idx < n4) {
                    const int tt4 = idx % (TC / 4);
                    const int q = idx / (TC / 4);
                    const int jj = q % KB, rr = q / KB;
                    const int64_t p = p0 + rr;
                    const int64_t k = (j0 + jj) * L + t0 + 4 * tt4;
                    if (p < J.P && k < J.K) buf[i] = *reinterpret_cast<const V4*>(X + p * J.ld + k);
                }
            }
#pragma unroll
            for (int i = 0; i < kMaxV4; ++i) {
                const int idx = threadIdx.x + i * kPackThreads;
                if (idx < n4) {
                    const int tt4 = idx % (TC / 4);
                    const int q = idx / (TC / 4);
                    const int jj = q % KB, rr = q / KB;
                    *reinterpret_cast<V4*>(lds + loff(rr, jj, 4 * tt4)) = buf[i];
                }
            }
        } else if (J.vec4) {
            // strided source: 4 rows x 4 indices per thread, 16-byte loads
            // along the rows, transposed in registers (all loads first)
            const int n16 = (TRc / 4) * KB * (TC / 4);
            V4 col[kMaxV16][4];
#pragma unroll
            for (int s = 0; s < kMaxV16; ++s) {
                const int idx = threadIdx.x + s * kPackThreads;
#pragma unroll
                for (int i = 0; i < 4; ++i) col[s][i] = V4{0, 0, 0, 0};
                if (idx < n16) {
                    const int rr4 = idx % (TRc / 4);
                    const int q = idx / (TRc / 4);
                    const int tt4 = q % (TC / 4), jj = q / (TC / 4);
                    const int64_t p = p0 + 4 * rr4;
                    const int64_t k = (j0 + jj) * L + t0 + 4 * tt4;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        if (k + i < J.K) {
                            if (p + 3 < J.P) {
                                col[s][i] = *reinterpret_cast<const V4*>(X + (k + i) * J.ld + p);
                            } else {
#pragma unroll
                                for (int u = 0; u < 4; ++u)
                                    if (p + u < J.P) col[s][i][u] = X[(k + i) * J.ld + p + u];
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int s = 0; s < kMaxV16; ++s) {
                const int idx = threadIdx.x + s * kPackThreads;
                if (idx < n16) {
                    const int rr4 = idx % (TRc / 4);
                    const int q = idx / (TRc / 4);
                    const int tt4 = q % (TC / 4), jj = q / (TC / 4);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const V4 w = {col[s][0][u], col[s][1][u], col[s][2][u], col[s][3][u]};
                        *reinterpret_cast<V4*>(lds + loff(4 * rr4 + u, jj, 4 * tt4)) = w;
                    }
                }
            }
        } else {
            // element loads (unaligned rows), kB per thread in flight before
            // their LDS stores
            const int n1 = TRc * KB * TCp;
            constexpr int kB = 64 / (int)sizeof(TIn);
            auto where = [&](int idx, int& rr, int& jj, int& tt) {
                if (!J.trans) {
                    tt = idx % TCp;
                    const int q = idx / TCp;
                    jj = q % KB;
                    rr = q / KB;
                } else {
                    rr = idx % TRc;
                    const int q = idx / TRc;
                    tt = q % TCp;
                    jj = q / TCp;
                }
            };
            for (int base = 0; base < n1; base += kB * kPackThreads) {
                TIn v[kB];
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    const int idx = base + u * kPackThreads + (int)threadIdx.x;
                    v[u] = (TIn)0;
                    if (idx < n1) {
                        int rr, jj, tt;
                        where(idx, rr, jj, tt);
                        const int64_t p = p0 + rr;
                        const int64_t k = (j0 + jj) * L + t0 + tt;
                        if (tt < TC && p < J.P && k < J.K) v[u] = J.trans ? X[k * J.ld + p] : X[p * J.ld + k];
                    }
                }
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    const int idx = base + u * kPackThreads + (int)threadIdx.x;
                    if (idx < n1) {
                        int rr, jj, tt;
                        where(idx, rr, jj, tt);
                        lds[loff(rr, jj, tt)] = v[u];
                    }
                }
            }
        }
    };

    for (int lp = 0; lp < r; lp += 4 * NCH * RL) {
        TIn acc[NCH][RL][Ec];
#pragma unroll
        for (int c = 0; c < NCH; ++c)
#pragma unroll
            for (int q = 0; q < RL; ++q)
#pragma unroll
                for (int e = 0; e < Ec; ++e) acc[c][q][e] = (TIn)0;

        if constexpr (pack_mfma<TIn, PREC, RL, NCH>()) {
            // Matrix cores: wave w contracts groups w * GPW .. w * GPW + GPW - 1
            // of the tile for the 16 projections lp .. lp + 15, two 16-row
            // halves each; lane (i, kq) supplies data row i / coefficient
            // column i.  The contraction runs over quads of 4 chunks: in
            // quad q lane kq reads its chunk 4 q + kq (4 indices, one 16-byte
            // LDS read) and feeds its 4 values to 4 consecutive products, so
            // step 4 q + e pairs lane kq with index 4 (4 q + kq) + e.
            constexpr int GPW = KB / 4;
            constexpr int kMaxQ = 4;           // TCp / 4 <= 16 chunks per group
            const int i16 = lane & 15, kq = lane >> 4;
            const int tc4 = TCp / 4, nq = (tc4 + 3) / 4;
            f32x4 macc[GPW][2];
#pragma unroll
            for (int gi = 0; gi < GPW; ++gi)
#pragma unroll
                for (int h = 0; h < 2; ++h) macc[gi][h] = f32x4{0.f, 0.f, 0.f, 0.f};
            // chunk 4 q + kq of group gi, row half h: ab[gi][h] + 4 (ay[gi] ^ 4 q);
            // the swizzle flips chunk bits, the padded layout has ay = kq
            const TIn* ab[GPW][2];
            int ay[GPW];
#pragma unroll
            for (int gi = 0; gi < GPW; ++gi) {
                const int jj = wave * GPW + gi;
                ay[gi] = LAY == 1 ? (((jj << ltc4) ^ (i16 & sm)) ^ kq) : kq;
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    ab[gi][h] = LAY == 1   ? lds + (((h * 16 + i16) << lnc) << 2)
                                : LAY == 2 ? lds + (jj * TCp + 4 * kq) * J.RT + h * 16 + i16
                                           : lds + (h * 16 + i16) * RS + jj * JS;
            }
            const int lcol = min(lp + i16, L - 1);     // columns >= r are never stored
            for (int t0 = 0; t0 < L; t0 += TC) {
                float cB[4 * kMaxQ];
#pragma unroll
                for (int q = 0; q < kMaxQ; ++q)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int ch = 4 * q + kq;
                        cB[4 * q + e] = q < nq && ch < tc4
                                            ? (float)J.coef[(int64_t)min(t0 + 4 * ch + e, L - 1) * L + lcol] : 0.0f;
                    }
                __syncthreads();
                stage(t0);
                __syncthreads();
                // quads fully unrolled; the reads of quad q + 1 are issued
                // before the products of quad q
                f32x4 av[2][GPW][2];
                auto rdq = [&](int q, f32x4 (&d)[GPW][2]) {
                    const bool ok = 4 * q + kq < tc4;
#pragma unroll
                    for (int gi = 0; gi < GPW; ++gi)
#pragma unroll
                        for (int h = 0; h < 2; ++h)
                            if constexpr (LAY == 2) {
                                // the 4 indices of the chunk are rows RT apart
                                const TIn* pp = ab[gi][h] + 16 * q * J.RT;
                                d[gi][h] = ok ? f32x4{pp[0], pp[J.RT], pp[2 * J.RT], pp[3 * J.RT]}
                                              : f32x4{0.f, 0.f, 0.f, 0.f};
                            } else {
                                d[gi][h] = ok ? *reinterpret_cast<const f32x4*>(ab[gi][h] + 4 * (ay[gi] ^ (4 * q)))
                                              : f32x4{0.f, 0.f, 0.f, 0.f};
                            }
                };
                rdq(0, av[0]);
#pragma unroll
                for (int q = 0; q < kMaxQ; ++q) {
                    if (q < nq) {
                        if (q + 1 < nq) rdq(q + 1, av[(q + 1) & 1]);
#pragma unroll
                        for (int e = 0; e < 4; ++e)
#pragma unroll
                            for (int gi = 0; gi < GPW; ++gi)
#pragma unroll
                                for (int h = 0; h < 2; ++h)
                                    macc[gi][h] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                        av[q & 1][gi][h][e], cB[4 * q + e], macc[gi][h], 0, 0, 0);
                    }
                }
            }
            // back to the lane layout of the stores through LDS:
            // Dt[ll][row][group], ll = projection - lp
            constexpr int DS = pack_mfma_ds<PREC>();
            float* Dt = reinterpret_cast<float*>(lds);
            __syncthreads();
#pragma unroll
            for (int gi = 0; gi < GPW; ++gi)
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        Dt[i16 * DS + (h * 16 + 4 * kq + j) * KB + wave * GPW + gi] = macc[gi][h][j];
            __syncthreads();
#pragma unroll
            for (int c = 0; c < NCH; ++c)
#pragma unroll
                for (int q = 0; q < RL; ++q) {
                    const int ll = (wave + 4 * c) * RL + q;
#pragma unroll
                    for (int e = 0; e < Ec; ++e) acc[c][q][e] = (TIn)Dt[ll * DS + row * KB + g * Ec + e];
                }
        } else {
            for (int t0 = 0; t0 < L; t0 += TC) {
                __syncthreads();
                stage(t0);
                __syncthreads();
                for (int tt4 = 0; tt4 < TCp / 4; ++tt4) {
                    const int tb = t0 + 4 * tt4;
                    // wave-uniform coefficients through the constant address space
                    // (scalar loads).  Indices are clamped into the L x L matrix: a
                    // clamped t only meets zero data (t >= t0 + TC is zero-padded in
                    // LDS) and a clamped projection l >= r is never stored.
                    TIn cf[NCH][4][RL];
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        const int lb = lp + (wave + 4 * c) * RL;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int t = min(tb + i, L - 1);
#pragma unroll
                            for (int q = 0; q < RL; ++q) cf[c][i][q] = coefc[(int64_t)t * L + min(lb + q, L - 1)];
                        }
                    }
#pragma unroll
                    for (int e = 0; e < Ec; ++e) {
                        V4 v;
                        if constexpr (LAY == 2) {
                            const TIn* pp = lds + loff(row, g * Ec + e, 4 * tt4);
                            v = V4{pp[0], pp[J.RT], pp[2 * J.RT], pp[3 * J.RT]};
                        } else {
                            v = *reinterpret_cast<const V4*>(lds + loff(row, g * Ec + e, 4 * tt4));
                        }
#pragma unroll
                        for (int c = 0; c < NCH; ++c)
#pragma unroll
                            for (int q = 0; q < RL; ++q) {
                                acc[c][q][e] += v[0] * cf[c][0][q];
                                acc[c][q][e] += v[1] * cf[c][1][q];
                                acc[c][q][e] += v[2] * cf[c][2][q];
                                acc[c][q][e] += v[3] * cf[c][3][q];
                            }
                    }
                }
            }
        }
        const int rib = rib0 + row;   // row within the packed row block
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int lb = lp + (wave + 4 * c) * RL;
#pragma unroll
            for (int q = 0; q < RL; ++q) {
                const int l = lb + q;
                if (l >= r) continue;   // wave-uniform
                if constexpr (PREC == P_PLAIN32 || PREC == P_PLAIN64) {
                    const int64_t p = p0 + row;
                    if (p < J.P) {
                        TIn* dst = reinterpret_cast<TIn*>(J.out) + p * J.plain_ld + (int64_t)l * J.Gp + j0 + g * Ec;
#pragma unroll
                        for (int e = 0; e < Ec; ++e) dst[e] = acc[c][q][e];
                    }
                } else {
                    if (J.keep) {
                        const int64_t p = p0 + row;
                        if (p < J.P) {
                            TIn* dst = J.keep + p * J.keep_ld + (int64_t)l * J.Gp + j0 + g * Ec;
#pragma unroll
                            for (int e = 0; e < Ec; ++e) dst[e] = acc[c][q][e];
                        }
                    }
                    const int64_t kbi = ((int64_t)l * J.Gp + j0) / KB;
                    const int64_t tile = rbi * J.nkb + kbi;
                    if constexpr (PREC == P_FP8 || PREC == P_FP8X2) {
                        float v8[8];
#pragma unroll
                        for (int e = 0; e < 8; ++e) v8[e] = (float)acc[c][q][e];
                        store_fp8_quarter<PREC>(J.out, tile, rib, g, J.plane_stride, J.plane_bytes, v8);
                    } else {
                        const int64_t off = (tile * 64 + g * RB + rib) * ly.LB;
                        store_lane<PREC, Ec, TIn>(J.out, off, J.plane_stride, J.plane_bytes, acc[c][q]);
                    }
                }
            }
        }
    }
}

// Two jobs passed by value (one GEMM's A and B sides).
// Waves per SIMD the register allocation must allow for the matrix-core
// variants: with direct loads (rounds of at most 48 KB) 4 for FP32 output and
// 3 for the 16-bit outputs, whose conversions need more registers (2 for the
// two-job launch of a transposed source, which needs more still); with
// register staging 2; else the compiler's choice.
template <typename TIn, int PREC, int RL, int NCH, int LAY, bool GROUPED>
constexpr int pack_waves_per_eu()
{
    if constexpr (pack_mfma<TIn, PREC, RL, NCH>()) {
        if constexpr (LAY == 0) return 2;
        if constexpr (PREC == P_F32) return 4;
        return LAY == 2 && !GROUPED ? 2 : 3;
    }
    return 1;
}

template <typename TIn, int PREC, int RL, int NCH, int LAY>
__global__ __launch_bounds__(kPackThreads)
__attribute__((amdgpu_waves_per_eu(pack_waves_per_eu<TIn, PREC, RL, NCH, LAY, false>()))) void pack_kernel(PackJob<TIn> ja, PackJob<TIn> jb, int64_t nblk_a)
{
    if ((int64_t)blockIdx.x < nblk_a) pack_tile<TIn, PREC, RL, NCH, LAY>(ja, (int64_t)blockIdx.x);
    else pack_tile<TIn, PREC, RL, NCH, LAY>(jb, (int64_t)blockIdx.x - nblk_a);
}

// Any number of jobs from a device table; prefix[i] is the first workgroup
// of job i (prefix[njobs] = grid size).
template <typename TIn, int PREC, int RL, int NCH, int LAY>
__global__ __launch_bounds__(kPackThreads)
__attribute__((amdgpu_waves_per_eu(pack_waves_per_eu<TIn, PREC, RL, NCH, LAY, true>()))) void pack_grouped_kernel(const PackJob<TIn>* __restrict__ jobs,
                                                                    const int64_t* __restrict__ prefix, int njobs)
{
    const int64_t b = blockIdx.x;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {                 // last job whose first workgroup is <= b
        const int mid = (lo + hi + 1) / 2;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    pack_tile<TIn, PREC, RL, NCH, LAY>(jobs[lo], b - prefix[lo]);
}

template <typename TIn, int PREC>
PackJob<TIn> make_job(const PackArgs& a)
{
    constexpr Layout ly = layout_of(PREC);
    const PackGeom& g = a.geom;
    PackJob<TIn> j;
    j.X = (const TIn*)a.X;
    j.ld = a.ld;
    j.trans = a.trans;
    // 16-byte loads: along k (contiguous source) or along the rows (strided)
    j.vec4 = a.L % 4 == 0 && a.ld % 4 == 0 && ((uintptr_t)a.X % (4 * sizeof(TIn))) == 0 &&
             (a.trans ? true : a.K % 4 == 0);
    j.P = a.P;
    j.K = a.K;
    j.L = a.L;
    j.r = a.r;
    j.coef = (const TIn*)a.coef;
    j.out = (char*)a.out;
    j.nkb = g.nkb;
    j.Gp = g.Gp;
    j.plane_stride = g.plane_bytes + g.scale_plane;
    j.plane_bytes = g.plane_bytes;
    j.plain_ld = a.plain_ld;
    j.keep = (TIn*)a.keep;
    j.keep_ld = a.keep_ld;
    j.nrb = g.nrb;
    j.ngt = g.Gp / ly.KB;
    // whole row blocks, so that padding rows are written (as zeros) too
    j.nrt = g.nrb * (ly.RB / Cmap<PREC>::TRc);
    // chunk of t staged per round: the largest divisor of L whose padded tile
    // fits the LDS budget (a multiple of 4 when 16-byte loads are used)
    auto lds_of = [&](int tc) {
        const int tcp = (tc + 3) / 4 * 4;
        return (size_t)Cmap<PREC>::TRc * ((size_t)ly.KB * (tcp + 4) + 4) * sizeof(TIn);
    };
    int TC = a.L;
    while (TC > 1 && (lds_of(TC) > (size_t)kPackLdsBytes || a.L % TC != 0 || (j.vec4 && TC % 4 != 0))) --TC;
    if (std::is_same<TIn, float>::value && !a.trans && Cmap<PREC>::TRc == 32 && (ly.KB == 16 || a.r > 16)) {
        // rows streamed into the unpadded swizzled layout: a larger budget
        // (fewer rounds) for the 16-bit outputs and for passes over more
        // than 16 projections; FP32 at r <= 16 keeps more workgroups per CU
        int tc = 4;
        while (tc * 2 <= a.L && a.L % (tc * 2) == 0 &&
               (size_t)Cmap<PREC>::TRc * ly.KB * (tc * 2) * sizeof(TIn) <= (size_t)kPackSwzLdsBytes)
            tc *= 2;
        if (a.L % tc == 0 && tc > TC) TC = tc;
    }
    if (j.vec4 && TC % 4 != 0) j.vec4 = 0;
    j.TC = TC;
    j.TCp = (TC + 3) / 4 * 4;
    j.JS = j.TCp + 4;
    j.RS = ly.KB * j.JS + 4;
    // direct loads into the swizzled layout: FP32 rows contiguous along k,
    // TC / 4 a power of two, the tile's chunks filling whole 64-slot wave
    // instructions (at most 32 per wave); 16 bytes per lane when the rows are
    // 16-byte aligned, else one value per lane
    const int tc4 = TC / 4;
    const int nc = ly.KB * tc4;
    j.swz = std::is_same<TIn, float>::value && !j.trans && TC % 4 == 0 && tc4 > 0 && (tc4 & (tc4 - 1)) == 0 &&
            (Cmap<PREC>::TRc * nc) % kPackThreads == 0 && Cmap<PREC>::TRc * nc <= 32 * kPackThreads;
    j.dma4 = j.swz && !j.vec4;
    j.lnc = j.ltc4 = j.sm = 0;
    if (j.swz) {
        while ((1 << j.lnc) < nc) ++j.lnc;
        while ((1 << j.ltc4) < tc4) ++j.ltc4;
        j.sm = (nc < 16 ? nc : 16) - 1;
    }
    // transposed FP32 sources whose rows are not 16-byte aligned (aligned
    // ones are faster with 16-byte register staging), 32-row tiles: direct
    // loads into the transposed layout when its round (columns padded to
    // TRc + 4) fits the LDS budget
    j.RT = Cmap<PREC>::TRc + 4;
    j.tdma = std::is_same<TIn, float>::value && j.trans && !j.vec4 && Cmap<PREC>::TRc == 32 &&
             (size_t)ly.KB * j.TCp * j.RT * sizeof(TIn) <= (size_t)kPackLdsBytes;
    return j;
}

// Round layout of a job (the LAY of pack_tile) and its LDS elements.
template <typename TIn>
int job_layout(const PackJob<TIn>& j) { return j.swz ? 1 : (j.tdma ? 2 : 0); }

template <typename TIn, int PREC>
size_t round_lds_elems(const PackJob<TIn>& j, int lay)
{
    if (lay == 1) return (size_t)Cmap<PREC>::TRc * ((size_t)4 << j.lnc);
    if (lay == 2) return (size_t)layout_of(PREC).KB * j.TCp * j.RT;
    return (size_t)Cmap<PREC>::TRc * j.RS;
}

// Launch of pack_kernel (one or two jobs) or pack_grouped_kernel with the
// round layout chosen at run time.
template <typename TIn, int PREC, int RL, int NCH, bool GROUPED, int LAY, typename... Args>
void launch_one(dim3 grid, size_t lds, hipStream_t s, Args... args)
{
    if constexpr (GROUPED)
        hipLaunchKernelGGL((pack_grouped_kernel<TIn, PREC, RL, NCH, LAY>), grid, dim3(kPackThreads), lds, s, args...);
    else
        hipLaunchKernelGGL((pack_kernel<TIn, PREC, RL, NCH, LAY>), grid, dim3(kPackThreads), lds, s, args...);
}

template <typename TIn, int PREC, int RL, int NCH, bool GROUPED, typename... Args>
int launch_lay(int lay, dim3 grid, size_t lds, hipStream_t s, Args... args)
{
    if constexpr (std::is_same<TIn, float>::value) {
        if (lay == 1) launch_one<TIn, PREC, RL, NCH, GROUPED, 1>(grid, lds, s, args...);
        else if (lay == 2) launch_one<TIn, PREC, RL, NCH, GROUPED, 2>(grid, lds, s, args...);
        else launch_one<TIn, PREC, RL, NCH, GROUPED, 0>(grid, lds, s, args...);
    } else {
        (void)lay;
        launch_one<TIn, PREC, RL, NCH, GROUPED, 0>(grid, lds, s, args...);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename TIn, int PREC, int RL, int NCH>
int launch_t(const PackArgs* a, int n, hipStream_t s)
{
    PackJob<TIn> ja = make_job<TIn, PREC>(a[0]);
    PackJob<TIn> jb = n > 1 ? make_job<TIn, PREC>(a[1]) : ja;
    const int lay = job_layout(ja);
    if (n > 1 && job_layout(jb) != lay) {
        // the two sides stage differently: one launch each
        const int e = launch_t<TIn, PREC, RL, NCH>(a, 1, s);
        return e != 0 ? e : launch_t<TIn, PREC, RL, NCH>(a + 1, 1, s);
    }
    const int64_t na = ja.nrt * ja.ngt;
    const int64_t nb = n > 1 ? jb.nrt * jb.ngt : 0;
    size_t lds = std::max(round_lds_elems<TIn, PREC>(ja, lay), round_lds_elems<TIn, PREC>(jb, lay)) * sizeof(TIn);
    if constexpr (pack_mfma<TIn, PREC, RL, NCH>())
        lds = std::max(lds, (size_t)16 * pack_mfma_ds<PREC>() * sizeof(float));
    if (na + nb > 0x7fffffff) return -2;
    return launch_lay<TIn, PREC, RL, NCH, false>(lay, dim3((unsigned)(na + nb)), lds, s, ja, jb, na);
}

template <typename TIn, int PREC>
int launch_p(const PackArgs* a, int n, hipStream_t s)
{
    int r = a[0].r;
    if (n > 1 && a[1].r > r) r = a[1].r;
    if (r == 1) return launch_t<TIn, PREC, 1, 1>(a, n, s);
    if constexpr (layout_of(PREC).E > 8) {
        return launch_t<TIn, PREC, 2, 1>(a, n, s);       // FP8: r <= 8
    } else {
        // 16-projection passes on the matrix cores where they apply (every r,
        // so that a pack at any r sums in the same order), else 64 per pass
        if (r <= 16 || pack_mfma<TIn, PREC, 4, 1>()) return launch_t<TIn, PREC, 4, 1>(a, n, s);
        return launch_t<TIn, PREC, 4, 4>(a, n, s);
    }
}


// ---- transposed sources, column-wise -----------------------------------------
// A source stored with the contraction index along its rows (X[k * ld + p]:
// the B side of a GEMM whose B is K x W) is projected one column p per
// thread: each group of L consecutive source rows is read as L coalesced row
// segments (256 columns, any alignment) and combined into RL projections at
// a time with vector FMAs, the coefficients broadcast from LDS; a thread
// keeps the E consecutive groups of one lane vector and writes it, so the 32
// threads of a row block write one contiguous half-tile.  Workgroup = 256
// columns x one k-block of groups, for every projection.
constexpr int kColW = 256;
constexpr int kColRL = 16;
constexpr int kColMaxL = 256;   // the library's largest projection size

template <typename TIn>
struct ColJob {
    const TIn* X; int64_t ld;
    int64_t P, K;
    int L, r;
    const TIn* coef;        // L x L, element (t, l)
    char* out;
    int64_t nkb, Gp, plane_stride;
    int64_t ncol;           // column tiles
    TIn* keep; int64_t keep_ld;
};

template <typename TIn, int PREC>
__device__ __forceinline__ void colpack_tile(const ColJob<TIn>& J, int64_t tix)
{
    constexpr Layout ly = layout_of(PREC);
    constexpr int KB = ly.KB, RB = ly.RB, E = ly.E;
    static_assert(KB % E == 0 && E <= 8, "lane vectors of at most 8 values");
    __shared__ TIn cs[kColMaxL * kColRL];   // coefficients of the pass: [t][l - l0]
    const int64_t ct = tix % J.ncol, gt = tix / J.ncol;
    const int64_t p = ct * kColW + threadIdx.x;
    const int64_t j0 = gt * KB;
    const int L = J.L, r = J.r;
    const bool live = p < J.P;
    const int64_t pc = live ? p : J.P - 1;   // reads stay inside the source
    for (int l0 = 0; l0 < r; l0 += kColRL) {
        __syncthreads();
        for (int x = threadIdx.x; x < L * kColRL; x += kColW) {
            const int t = x / kColRL, lq = x % kColRL;
            cs[x] = l0 + lq < r ? J.coef[(int64_t)t * L + l0 + lq] : (TIn)0;
        }
        __syncthreads();
        for (int g0 = 0; g0 < KB; g0 += E) {
            TIn acc[kColRL][E];
#pragma unroll
            for (int q = 0; q < kColRL; ++q)
#pragma unroll
                for (int e = 0; e < E; ++e) acc[q][e] = (TIn)0;
            // rows past K read row K - 1 and count as zero; the loads of
            // index t + 1 are issued before the products of index t
            auto ld = [&](int t, TIn (&x)[E]) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int64_t k = (j0 + g0 + e) * L + t;
                    x[e] = J.X[(k < J.K ? k : J.K - 1) * J.ld + pc];
                }
            };
            auto fma = [&](int t, const TIn (&x)[E]) {
                const TIn* c = cs + t * kColRL;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const TIn xe = (j0 + g0 + e) * L + t < J.K ? x[e] : (TIn)0;
#pragma unroll
                    for (int q = 0; q < kColRL; ++q) acc[q][e] += c[q] * xe;
                }
            };
            TIn xa[E], xb[E];
            ld(0, xa);
            for (int t = 0; t < L; t += 2) {
                if (t + 1 < L) ld(t + 1, xb);
                fma(t, xa);
                if (t + 1 < L) {
                    if (t + 2 < L) ld(t + 2, xa);
                    fma(t + 1, xb);
                }
            }
            if (live) {
                const int64_t rb = p / RB;
                const int rib = (int)(p % RB), g = g0 / E;
#pragma unroll
                for (int q = 0; q < kColRL; ++q) {
                    const int l = l0 + q;
                    if (l >= r) break;
                    const int64_t kb = ((int64_t)l * J.Gp + j0) / KB;
                    const int64_t off = ((rb * J.nkb + kb) * 64 + g * RB + rib) * (int64_t)ly.LB;
                    store_lane<PREC, E, TIn>(J.out, off, J.plane_stride, 0, acc[q]);
                    if (J.keep) {
                        TIn* dst = J.keep + p * J.keep_ld + (int64_t)l * J.Gp + j0 + g0;
#pragma unroll
                        for (int e = 0; e < E; ++e) dst[e] = acc[q][e];
                    }
                }
            }
        }
    }
}

template <typename TIn, int PREC>
__global__ __launch_bounds__(kColW) void colpack_grouped_kernel(const ColJob<TIn>* __restrict__ jobs,
                                                               const int64_t* __restrict__ prefix, int njobs)
{
    const int64_t b = blockIdx.x;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    colpack_tile<TIn, PREC>(jobs[lo], b - prefix[lo]);
}

template <typename TIn, int PREC>
ColJob<TIn> make_coljob(const PackArgs& a)
{
    ColJob<TIn> j;
    j.X = (const TIn*)a.X;
    j.ld = a.ld;
    j.P = a.P;
    j.K = a.K;
    j.L = a.L;
    j.r = a.r;
    j.coef = (const TIn*)a.coef;
    j.out = (char*)a.out;
    j.nkb = a.geom.nkb;
    j.Gp = a.geom.Gp;
    j.plane_stride = a.geom.plane_bytes + a.geom.scale_plane;
    j.ncol = cdiv(a.P, kColW);
    j.keep = (TIn*)a.keep;
    j.keep_ld = a.keep_ld;
    return j;
}

// Formats the column-wise path serves (16-byte lane vectors of at most 8 values).
template <int PREC>
constexpr bool colpack_ok() { return layout_of(PREC).E <= 8; }

template <typename TIn, int PREC>
int launch_colpack_grouped(const PackArgs* a, int n, char* jobs_at, char* prefix_at, hipStream_t s)
{
    if constexpr (!colpack_ok<PREC>()) {
        return -2;
    } else {
        std::vector<ColJob<TIn>> jobs(n);
        std::vector<int64_t> prefix(n + 1, 0);
        for (int i = 0; i < n; ++i) {
            jobs[i] = make_coljob<TIn, PREC>(a[i]);
            prefix[i + 1] = prefix[i] + jobs[i].ncol * (a[i].geom.Gp / layout_of(PREC).KB);
        }
        if (prefix[n] == 0) return 0;
        if (prefix[n] > 0x7fffffff) return -2;
        if (hipMemcpyAsync(jobs_at, jobs.data(), sizeof(ColJob<TIn>) * n, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(prefix_at, prefix.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s) !=
                hipSuccess)
            return -1;
        hipLaunchKernelGGL((colpack_grouped_kernel<TIn, PREC>), dim3((unsigned)prefix[n]), dim3(kColW), 0, s,
                           (const ColJob<TIn>*)jobs_at, (const int64_t*)prefix_at, n);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
}

template <typename TIn, int PREC, int RL, int NCH>
int launch_grouped_t(const PackArgs* a, int n, void* table, hipStream_t s)
{
    // jobs ordered by round layout (swizzled, transposed, padded): one launch
    // per layout present, sharing the job array; the table holds the jobs
    // and one prefix array per layout
    std::vector<PackJob<TIn>> jobs;
    jobs.reserve(n);
    int start[4] = {0, 0, 0, 0};
    const int order[3] = {1, 2, 0};
    for (int o = 0; o < 3; ++o) {
        start[o] = (int)jobs.size();
        for (int i = 0; i < n; ++i) {
            PackJob<TIn> j = make_job<TIn, PREC>(a[i]);
            if (job_layout(j) == order[o]) jobs.push_back(j);
        }
    }
    start[3] = n;
    std::vector<int64_t> prefix[3];
    size_t lds_e[3] = {0, 0, 0};
    int64_t total = 0;
    for (int o = 0; o < 3; ++o) {
        prefix[o].assign(start[o + 1] - start[o] + 1, 0);
        for (int i = start[o]; i < start[o + 1]; ++i) {
            prefix[o][i - start[o] + 1] = prefix[o][i - start[o]] + jobs[i].nrt * jobs[i].ngt;
            lds_e[o] = std::max(lds_e[o], round_lds_elems<TIn, PREC>(jobs[i], order[o]));
        }
        if (prefix[o].back() > 0x7fffffff) return -2;
        total += prefix[o].back();
    }
    if (total == 0) return -2;
    char* t = (char*)table;
    const size_t jbytes = rup((int64_t)sizeof(PackJob<double>) * n, 256);
    const size_t pbytes = rup(8 * (int64_t)(n + 1), 256);
    if (hipMemcpyAsync(t, jobs.data(), sizeof(PackJob<TIn>) * n, hipMemcpyHostToDevice, s) != hipSuccess) return -1;
    for (int o = 0; o < 3; ++o) {
        const int64_t grid = prefix[o].back();
        if (grid == 0) continue;
        char* pre = t + jbytes + o * pbytes;
        if (hipMemcpyAsync(pre, prefix[o].data(), sizeof(int64_t) * prefix[o].size(), hipMemcpyHostToDevice, s) !=
            hipSuccess)
            return -1;
        size_t lds = lds_e[o] * sizeof(TIn);
        if constexpr (pack_mfma<TIn, PREC, RL, NCH>())
            lds = std::max(lds, (size_t)16 * pack_mfma_ds<PREC>() * sizeof(float));
        const int e = launch_lay<TIn, PREC, RL, NCH, true>(order[o], dim3((unsigned)grid), lds, s,
                                                           (const PackJob<TIn>*)t + start[o], (const int64_t*)pre,
                                                           start[o + 1] - start[o]);
        if (e != 0) return e;
    }
    return 0;
}

size_t pack_grouped_table_bytes_rows(int n)
{
    return (size_t)rup((int64_t)sizeof(PackJob<double>) * n, 256) + 3 * (size_t)rup(8 * (int64_t)(n + 1), 256);
}

template <typename TIn, int PREC>
int launch_grouped_rows(const PackArgs* a, int n, void* table, hipStream_t s);

template <typename TIn, int PREC>
int launch_grouped_p(const PackArgs* a, int n, void* table, hipStream_t s)
{
    if constexpr (colpack_ok<PREC>()) {
        // transposed sources go column-wise; the rest through the tile packer
        std::vector<PackArgs> rows, cols;
        for (int i = 0; i < n; ++i) (a[i].trans ? cols : rows).push_back(a[i]);
        if (!cols.empty()) {
            char* t = (char*)table;
            const size_t base = pack_grouped_table_bytes_rows(n);
            const int e = launch_colpack_grouped<TIn, PREC>(cols.data(), (int)cols.size(), t + base,
                                                            t + base + rup((int64_t)sizeof(ColJob<double>) * n, 256), s);
            if (e != 0) return e;
            if (rows.empty()) return 0;
            a = rows.data();
            n = (int)rows.size();
            return launch_grouped_rows<TIn, PREC>(a, n, table, s);
        }
    }
    return launch_grouped_rows<TIn, PREC>(a, n, table, s);
}

template <typename TIn, int PREC>
int launch_grouped_rows(const PackArgs* a, int n, void* table, hipStream_t s)
{
    int r = 1;
    for (int i = 0; i < n; ++i) r = a[i].r > r ? a[i].r : r;
    if (r == 1) return launch_grouped_t<TIn, PREC, 1, 1>(a, n, table, s);
    if constexpr (layout_of(PREC).E > 8) {
        return launch_grouped_t<TIn, PREC, 2, 1>(a, n, table, s);
    } else {
        if (r <= 16 || pack_mfma<TIn, PREC, 4, 1>()) return launch_grouped_t<TIn, PREC, 4, 1>(a, n, table, s);
        return launch_grouped_t<TIn, PREC, 4, 4>(a, n, table, s);
    }
}

// ---- unprojected operands ----------------------------------------------------
// A workgroup copies a kRpRows x kRpK block of the source (rows p, natural
// contraction index k) into LDS with coalesced loads along whichever index
// is contiguous in memory, then writes the block's packed tiles, one 16-byte
// lane vector per lane slot, converted as the format's packer does.
constexpr int kRpRows = 64, kRpK = 64;

template <typename TIn>
struct RepackJob {
    const TIn* X; int64_t ld; int trans;
    int64_t P, K;
    char* out;
    int64_t nrb, nkb, plane_stride;
    int64_t ntk, nblk;            // k blocks of the workgroup grid, workgroups
};

template <typename TIn, int PREC>
__device__ __forceinline__ void repack_block(const RepackJob<TIn>& J, int64_t b)
{
    constexpr Layout ly = layout_of(PREC);
    constexpr int RB = ly.RB, KB = ly.KB, E = ly.E;
    __shared__ TIn sm[kRpRows][kRpK + 1];
    const int64_t p0 = (b / J.ntk) * kRpRows, k0 = (b % J.ntk) * kRpK;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // 64 consecutive elements of the contiguous index per wave instruction
#pragma unroll 4
    for (int q = wave; q < kRpRows; q += kPackThreads / 64) {
        int rr, kk;
        if (J.trans) { kk = q; rr = lane; }      // source row k0 + q, elements p0 .. p0 + 63
        else { rr = q; kk = lane; }              // source row p0 + q, elements k0 .. k0 + 63
        const int64_t p = p0 + rr, k = k0 + kk;
        TIn v = (TIn)0;
        if (p < J.P && k < J.K) v = J.trans ? J.X[k * J.ld + p] : J.X[p * J.ld + k];
        sm[rr][kk] = v;
    }
    __syncthreads();
    constexpr int NTB = (kRpRows / RB) * (kRpK / KB);     // tiles of the block
#pragma unroll
    for (int s0 = 0; s0 < NTB * 64; s0 += kPackThreads) {
        const int s = s0 + tid;
        const int q = s / 64, ln = s % 64;
        const int rbl = q / (kRpK / KB), kbl = q % (kRpK / KB);
        const int64_t rb = p0 / RB + rbl, kb = k0 / KB + kbl;
        if (rb < J.nrb && kb < J.nkb) {
            const int g = ln / RB, rib = ln % RB;
            TIn v[E];
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = sm[rbl * RB + rib][kbl * KB + g * E + e];
            store_lane<PREC, E, TIn>(J.out, ((rb * J.nkb + kb) * 64 + ln) * (int64_t)ly.LB, J.plane_stride, 0, v);
        }
    }
    (void)lane;
}

template <typename TIn, int PREC>
__global__ __launch_bounds__(kPackThreads) void repack_kernel(RepackJob<TIn> ja, RepackJob<TIn> jb)
{
    const int64_t b = blockIdx.x;
    if (b < ja.nblk) repack_block<TIn, PREC>(ja, b);
    else repack_block<TIn, PREC>(jb, b - ja.nblk);
}

template <typename TIn, int PREC>
RepackJob<TIn> make_repack(const PackArgs& a)
{
    constexpr Layout ly = layout_of(PREC);
    RepackJob<TIn> j;
    j.X = (const TIn*)a.X;
    j.ld = a.ld;
    j.trans = a.trans;
    j.P = a.P;
    j.K = a.K;
    j.out = (char*)a.out;
    j.nrb = a.geom.nrb;
    j.nkb = a.geom.nkb;
    j.plane_stride = a.geom.plane_bytes + a.geom.scale_plane;
    j.ntk = cdiv(j.nkb * ly.KB, kRpK);
    j.nblk = cdiv(j.nrb * ly.RB, kRpRows) * j.ntk;
    return j;
}

template <typename TIn, int PREC>
int launch_repack_t(const PackArgs* a, int n, hipStream_t s)
{
    const RepackJob<TIn> ja = make_repack<TIn, PREC>(a[0]);
    RepackJob<TIn> jb = n > 1 ? make_repack<TIn, PREC>(a[1]) : ja;
    if (n < 2) jb.nblk = 0;
    const int64_t grid = ja.nblk + jb.nblk;
    if (grid > 0x7fffffff) return -2;
    if (grid == 0) return 0;
    hipLaunchKernelGGL((repack_kernel<TIn, PREC>), dim3((unsigned)grid), dim3(kPackThreads), 0, s, ja, jb);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int launch_repack_n(int prec, const PackArgs* a, int n, hipStream_t s)
{
    switch (prec) {
    case P_F64:    return launch_repack_t<double, P_F64>(a, n, s);
    case P_F32:    return launch_repack_t<float, P_F32>(a, n, s);
    case P_BF16:   return launch_repack_t<float, P_BF16>(a, n, s);
    case P_BF16X3: return launch_repack_t<float, P_BF16X3>(a, n, s);
    case P_F16:    return launch_repack_t<float, P_F16>(a, n, s);
    case P_F16X3:  return launch_repack_t<float, P_F16X3>(a, n, s);
    default:       return -2;
    }
}

int launch_pack_n(int prec, const PackArgs* a, int n, hipStream_t s)
{
    switch (prec) {
    case P_F64:    return launch_p<double, P_F64>(a, n, s);
    case P_F32:    return launch_p<float, P_F32>(a, n, s);
    case P_BF16:   return launch_p<float, P_BF16>(a, n, s);
    case P_BF16X3: return launch_p<float, P_BF16X3>(a, n, s);
    case P_F16:    return launch_p<float, P_F16>(a, n, s);
    case P_F16X3:  return launch_p<float, P_F16X3>(a, n, s);
    case P_FP8:    return launch_p<float, P_FP8>(a, n, s);
    case P_FP8X2:  return launch_p<float, P_FP8X2>(a, n, s);
    case P_PLAIN32: return launch_p<float, P_PLAIN32>(a, n, s);
    case P_PLAIN64: return launch_p<double, P_PLAIN64>(a, n, s);
    default:       return -2;
    }
}

int launch_pack(int prec, const PackArgs& a, hipStream_t s) { return launch_pack_n(prec, &a, 1, s); }

size_t pack_grouped_table_bytes(int n)
{
    // the tile packer's jobs and one prefix array per round layout, then the
    // column-wise jobs and their prefix array
    return pack_grouped_table_bytes_rows(n) + (size_t)rup((int64_t)sizeof(ColJob<double>) * n, 256) +
           (size_t)rup(8 * (int64_t)(n + 1), 256);
}

int launch_pack_grouped(int prec, const PackArgs* a, int n, void* table, hipStream_t s)
{
    switch (prec) {
    case P_F64:    return launch_grouped_p<double, P_F64>(a, n, table, s);
    case P_F32:    return launch_grouped_p<float, P_F32>(a, n, table, s);
    case P_BF16:   return launch_grouped_p<float, P_BF16>(a, n, table, s);
    case P_BF16X3: return launch_grouped_p<float, P_BF16X3>(a, n, table, s);
    case P_F16:    return launch_grouped_p<float, P_F16>(a, n, table, s);
    case P_F16X3:  return launch_grouped_p<float, P_F16X3>(a, n, table, s);
    case P_FP8:    return launch_grouped_p<float, P_FP8>(a, n, table, s);
    case P_FP8X2:  return launch_grouped_p<float, P_FP8X2>(a, n, table, s);
    default:       return -2;
    }
}

}  // namespace pj
