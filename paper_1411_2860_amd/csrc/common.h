// common.h -- internal definitions shared by the host code and the HIP
// kernels of libprojgemm: packed-operand layouts, MFMA operand traits and
// small helpers.  Not part of the public ABI (include/projgemm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pj {

enum Prec { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_BF16X3 = 3, P_F16 = 4, P_F16X3 = 5, P_FP8 = 6, P_FP8X2 = 7,
            // internal: projections written as a plain row-major matrix
            // (rows x r*Gp, element (p, l*Gp + j)) in FP32 or FP64
            P_PLAIN32 = 8, P_PLAIN64 = 9 };

// ---------------------------------------------------------------------------
// Packed ("fragment-order") operand layout.
//
// A packed operand X has `rows` rows and a contraction length Kc.  It is cut
// into tiles of RB rows x KB contraction indices.  A tile is exactly what one
// 64-lane wavefront feeds to the matrix cores for that slice of the
// contraction: lane i = g * RB + row holds the E consecutive indices
// g*E .. g*E+E-1 of row `row` (g < NG = 64 / RB).  One tile is 64 * LB bytes
// (LB = E * element bytes) and a wave loads it with one fully coalesced
// LB-byte access per lane.
//
// Tiles are stored [plane][row_block][k_block][lane][LB], then, for FP8,
// one E8M0 scale byte per lane per tile: [plane][row_block][k_block][lane].
// FP8 is the exception to the lane rule above: the block-scaled 8-bit
// instruction takes 64-index tiles whose MX block h (32 indices, one scale)
// of a row is split over bytes 16h..16h+15 of lanes row and 32 + row; the
// scale of block h comes from lane 32h + row.
//
// Projected operands use the contraction order k = l * Gp + j (projection
// major, group j < G zero-padded up to Gp = roundup(G, KB)), so the first
// r * Gp / KB k-blocks of a row block are exactly the first r projections:
// one buffer packed at rmax serves every r <= rmax.
// ---------------------------------------------------------------------------
struct Layout {
    int elem;    // bytes per element
    int RB;      // rows per tile
    int NG;      // lane groups along the contraction (64 / RB)
    int E;       // consecutive contraction indices per lane
    int KB;      // contraction indices per tile (NG * E)
    int LB;      // bytes per lane per tile
    int planes;  // 1, or 2 for hi + lo split modes
    int scales;  // 1 if an E8M0 scale byte accompanies each lane vector
};

__host__ __device__ constexpr Layout layout_of(int prec)
{
    switch (prec) {
    case P_F64:   return Layout{8, 16, 4, 2, 8, 16, 1, 0};
    case P_F32:   return Layout{4, 32, 2, 4, 8, 16, 1, 0};
    case P_BF16:  return Layout{2, 32, 2, 8, 16, 16, 1, 0};
    case P_BF16X3:return Layout{2, 32, 2, 8, 16, 16, 2, 0};
    case P_F16:   return Layout{2, 32, 2, 8, 16, 16, 1, 0};
    case P_F16X3: return Layout{2, 32, 2, 8, 16, 16, 2, 0};
    case P_FP8:   return Layout{1, 32, 2, 32, 64, 32, 1, 1};
    case P_FP8X2: return Layout{1, 32, 2, 32, 64, 32, 2, 1};
    case P_PLAIN32: return Layout{4, 32, 2, 4, 8, 16, 1, 0};
    case P_PLAIN64: return Layout{8, 16, 4, 2, 8, 16, 1, 0};
    default:      return Layout{0, 0, 0, 0, 0, 0, 0, 0};
    }
}

__host__ __device__ constexpr int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ constexpr int64_t rup(int64_t a, int64_t b) { return cdiv(a, b) * b; }

// Geometry of one packed operand.
struct PackGeom {
    int64_t rows, K;
    int L, rmax;
    int64_t G, Gp;       // groups, padded groups
    int64_t nrb, nkb;    // row blocks, k-blocks per row block
    int64_t plane_bytes; // bytes of one plane of tiles
    int64_t scale_plane; // bytes of one plane of scales
    int64_t total;       // all bytes
};

inline PackGeom pack_geom(int64_t rows, int64_t K, int L, int rmax, int prec)
{
    Layout ly = layout_of(prec);
    PackGeom g;
    g.rows = rows; g.K = K; g.L = L; g.rmax = rmax;
    g.G = cdiv(K, L);
    g.Gp = rup(g.G, ly.KB);
    g.nrb = cdiv(rows, ly.RB);
    g.nkb = (int64_t)rmax * g.Gp / ly.KB;
    g.plane_bytes = g.nrb * g.nkb * 64 * ly.LB;
    g.scale_plane = ly.scales ? g.nrb * g.nkb * 64 : 0;
    g.total = ly.planes * (g.plane_bytes + g.scale_plane);
    return g;
}

// ---------------------------------------------------------------------------
// Vector types for MFMA operands.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));

// Launch helpers implemented in the .hip files (host side).
struct PackArgs {
    const void* X;     // float or double source
    int64_t ld;        // leading dimension of X in elements
    int trans;         // 0: element (p, k) at X[p*ld + k]; 1: at X[k*ld + p]
    int64_t P, K;      // rows and contraction length of the source
    int L, r;          // projection size, projections to pack (r <= rmax)
    const void* coef;  // L x L row-major, element (t, l) = coefficient of
                       // source index t in projection l (float or double)
    void* out;         // packed operand
    PackGeom geom;
    int64_t plain_ld = 0;  // row stride of a plain output (P_PLAIN32 / P_PLAIN64)
    // optional second output of a packed (not plain) pass: the same projected
    // values before conversion, as a plain matrix keep[p * keep_ld + l * Gp + j]
    // (FP32, FP64 for P_F64) with the packed geometry's Gp; rows p < P only
    void* keep = nullptr;
    int64_t keep_ld = 0;
};
int launch_pack(int prec, const PackArgs& a, hipStream_t s);
// Packs n (1 or 2) operands of the same precision in one launch.
int launch_pack_n(int prec, const PackArgs* a, int n, hipStream_t s);
// Fragment-order copy of an operand that is not projected (the contraction
// index kept in its natural order, zero past K up to the geometry's padded
// length nkb * KB; rows past P zero): the operands of the backward's
// contractions over the rows or columns of R.  a.L, a.r and a.coef are
// unused; a.geom gives the padded shape.  Not for the FP8 formats (-2).
int launch_repack_n(int prec, const PackArgs* a, int n, hipStream_t s);
// Packs any number of operands in one launch, driven by a job table that is
// copied into `table` (device memory of pack_grouped_table_bytes(n) bytes).
size_t pack_grouped_table_bytes(int n);
int launch_pack_grouped(int prec, const PackArgs* a, int n, void* table, hipStream_t s);

struct GemmArgs {
    const void* X; PackGeom gx;  // P rows
    const void* Y; PackGeom gy;  // Q rows
    int64_t nkb;                 // k-blocks to contract (r * Gp / KB)
    int64_t P, Q;
    void* R; int64_t ldr;        // P x Q row-major, float (double for F64)
    float beta;
    int nsplit = 1;              // > 1: contiguous k-block ranges with partials in `part`
    void* part = nullptr;        // nsplit x P x Q partials (output type), caller workspace
};
// Synthesis with the projection coefficients (the transpose of the pack's
// projection): out(p, jL + t) = sum_{l<r} in(p, l*Gp + j) coef[t, l].
struct ExpandArgs {
    const void* in; int64_t ldi; int in_trans;     // in(p, kk) at in[p*ldi+kk] or in[kk*ldi+p]
    void* out; int64_t ldo; int out_trans;         // out(p, k) at out[p*ldo+k] or out[k*ldo+p]
    int64_t P, K;
    int L, r;
    int64_t Gp;
    const void* coef;                              // L x L, element (t, l)
};
int launch_expand(int is_double, const ExpandArgs& a, hipStream_t s);

// One problem of a grouped launch, as stored in device memory.
struct GroupedProblem {
    const void* X; int64_t x_nrb, x_nkb, x_plane, x_pb;
    const void* Y; int64_t y_nrb, y_nkb, y_plane, y_pb;
    int64_t nkb, P, Q;
    void* R; int64_t ldr;
    float beta;
};
struct GroupedItem {
    int32_t prob;
    int32_t tm, tn;      // tile of the item's body
    int32_t body;        // 0: the launch's tile configuration; 1: its small tile
};                       // (one MFMA block per wave, same waves)
// Persistent launch over `nitems` items: as many workgroups as `cus` compute
// units hold at once (at most one per item).
int launch_gemm_grouped(int prec, const GroupedProblem* probs, const GroupedItem* items, int64_t nitems,
                        int64_t cus, int cfg, hipStream_t s);

// cfg < 0 picks the default tile configuration for the shape.
int launch_gemm(int prec, const GemmArgs& a, int cfg, hipStream_t s);
int gemm_num_configs();
int gemm_config_tile(int prec, int cfg, int* tile_m, int* tile_n);
// The small tile grouped launches of configuration cfg can also run.
int gemm_config_small_tile(int prec, int cfg, int* tile_m, int* tile_n);
int gemm_default_config(int prec, int64_t P, int64_t Q, int64_t nkb);
int gemm_split_count(int prec, int64_t P, int64_t Q, int64_t nkb, int cfg);

}  // namespace pj
