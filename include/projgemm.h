/*
 * projgemm.h -- C ABI of libprojgemm.so: projection-based precision-scalable
 * GEMM and 1-D cross-correlation / convolution on AMD MI355X (gfx950).
 *
 * Method: Anam, Whatmough, Andreopoulos, "Precision-Energy-Throughput
 * Scaling of Generic Matrix Multiplication and Convolution Kernels via
 * Linear Projections", IEEE TCSVT 24(11), 2014 (arXiv:1411.2860).
 *
 * Notation (paper Sec. III, Table I):
 *   A is M x K, B is K x W, R = A B is M x W.  The contraction index k is
 *   split into G = ceil(K / L) groups of L consecutive indices starting at
 *   0 (the block-diagonal C_N, D_N of eq. (15)); indices past K are treated
 *   as zeros.  C is the L x L projection matrix, column l being projection
 *   l (a_c = a C, eq. (5)); D = C^{-1} projects the B side (b_d = D b).
 *   r is the NUMBER of projections kept, 1 <= r <= L (the paper counts them
 *   as l + 1, 0 <= l < L).  With r = L the result is exact (eq. (6)); with
 *   r < L it is the partial sum of eq. (8):
 *       R_hat = sum_{l<r} A_c^{(l)} B_d^{(l)} = A Q_{r,K} B,
 *       Q_{r,K} = blockdiag(C[:, :r] D[:r, :]).
 *
 * Conventions of every entry point:
 *   - Matrices are row-major with a leading dimension (in elements).
 *   - Tensors and workspaces are device memory owned by the caller; the
 *     library keeps no pointer to them after the call.  Calls allocate no
 *     device memory: scratch comes from the caller's workspace, whose size
 *     the matching *_workspace_bytes query returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued asynchronously; no call synchronises the stream.
 *   - Every argument check runs on the host before any device work, so an
 *     invalid call returns an error code and touches no device state.
 *     Errors are returned, never raised or aborted on.
 */
#ifndef PROJGEMM_H
#define PROJGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PJ_OK = 0,
    PJ_ERR_ARG = -1,          /* null pointer, bad enum, r or L out of range   */
    PJ_ERR_SHAPE = -2,        /* non-positive size, leading dimension too small */
    PJ_ERR_UNSUPPORTED = -3,  /* valid request the library does not implement   */
    PJ_ERR_WORKSPACE = -4,    /* workspace missing or smaller than the query    */
    PJ_ERR_SINGULAR = -5,     /* custom projection matrix is not invertible     */
    PJ_ERR_HIP = -6,          /* a HIP runtime call or kernel launch failed     */
    PJ_ERR_SCRATCH = -7       /* proj_gemm_noalloc: request exceeds its scratch */
} pj_status;

typedef enum {
    PJ_BASIS_DCT2 = 0,        /* DCT-II, eq. (7); stored orthonormal (see below) */
    PJ_BASIS_HAAR = 1,        /* Haar decomposition basis; L a power of two      */
    PJ_BASIS_IDENTITY = 2,    /* C = I: keeps indices k with (k mod L) < r       */
    PJ_BASIS_CUSTOM = 3       /* any invertible C given by the caller            */
} pj_basis_kind;

/* Arithmetic of the reduced contraction.  Inputs and outputs are FP64 for
 * PJ_F64 and FP32 for every other mode; projections are computed in FP32
 * (FP64 for PJ_F64) and rounded to the mode's operand format.
 *   PJ_BF16 / PJ_F16   : one rounded operand, FP32 accumulation;
 *   PJ_BF16X3 / PJ_F16X3: x = hi + lo split, R = hi*hi + hi*lo + lo*hi,
 *                         FP32 accumulation (about FP32-level error);
 *   PJ_FP8             : OCP FP8 e4m3 operands with one power-of-two (E8M0)
 *                         scale per 32 consecutive contraction indices,
 *                         FP32 accumulation; r <= 8 only;
 *   PJ_FP8X2           : FP8 hi + lo split, three products; r <= 8 only. */
typedef enum {
    PJ_F64 = 0, PJ_F32 = 1, PJ_BF16 = 2, PJ_BF16X3 = 3,
    PJ_F16 = 4, PJ_F16X3 = 5, PJ_FP8 = 6, PJ_FP8X2 = 7
} pj_precision;

typedef enum { PJ_XCORR = 0, PJ_CONV = 1 } pj_conv_mode;
/* Realisation of the full-rate projected CONV: the library's choice, the
 * direct contraction of the projected signal with the projected kernel
 * phases, or the frequency-domain one (proj_conv1d_fft). */
typedef enum { PJ_CONV_AUTO = 0, PJ_CONV_DIRECT = 1, PJ_CONV_FFT = 2 } pj_conv_method;
/* Output rate of proj_conv1d_rate: every output, or only the outputs at the
 * aligned lags m = aL with the others interpolated. */
typedef enum { PJ_RATE_FULL = 0, PJ_RATE_BLOCK = 1 } pj_conv_rate;

typedef struct pj_basis_s* pj_basis;

/* Human-readable name of a status code (static string). */
const char* pj_status_str(int status);

/* ------------------------------------------------------------------ basis */

/* Builds the L x L projection matrix C of the given kind and D = C^{-1}
 * (paper eq. (5)-(7); Haar: Sec. IV-A / V-B), in FP64 on the host, and
 * uploads FP32 and FP64 copies to the current device (synchronously).
 *   kind  : PJ_BASIS_*.  DCT-II is stored orthonormal (column j scaled by
 *           sqrt(1/L) for j = 0, sqrt(2/L) otherwise) with D = C^T: the
 *           projected result does not depend on the scale of the columns of
 *           C, so this equals eq. (7)'s unnormalised matrix.  Haar is the
 *           orthonormal Haar basis with column 0 the scaling function, then
 *           wavelets from coarse to fine scale, shifts ascending.
 *   L     : 1 <= L <= 256 (Haar: a power of two).
 *   C     : row-major L x L (C[t*L + l]) for PJ_BASIS_CUSTOM, else NULL.
 *           D is found by LU with partial pivoting; PJ_ERR_SINGULAR if a
 *           pivot is below 1e-12 times the largest |C| entry.
 * The basis is immutable and may be shared by concurrent calls.  If no
 * device is present the host copy is still built and device calls using it
 * return PJ_ERR_HIP. */
int pj_basis_create(pj_basis* out, int kind, int L, const double* C);

/* FP64 copies of C and D (row-major L x L each); either pointer may be NULL. */
int pj_basis_get(pj_basis b, double* C_out, double* D_out);

/* L of the basis, or a negative status. */
int pj_basis_L(pj_basis b);

int pj_basis_destroy(pj_basis b);

/* --------------------------------------------------------- projected GEMM */

/* Bytes of workspace proj_gemm needs (0 for invalid arguments): the two
 * packed operands, plus, when the output is too small to fill the device
 * with tiles and the contraction is long (skinny outputs such as scatter or
 * Gram matrices), room for the partial results of contiguous ranges of the
 * contraction that are contracted concurrently and summed afterwards. */
size_t pj_gemm_workspace_bytes(int M, int W, int K, int L, int r, int prec);

/* R <- A Q_{r,K} B + beta R  (paper Sec. III-A/B, eq. (5)-(8), (15)).
 *   transA = 'N': A is M x K (element (i,k) at A[i*lda + k]);
 *            'T': A is stored K x M (element (i,k) at A[k*lda + i]).
 *   transB = 'N': B is K x W (element (k,w) at B[k*ldb + w]);
 *            'T': B is stored W x K (element (k,w) at B[w*ldb + k]).
 *   R is M x W, element (i,w) at R[i*ldr + w]; beta = 0 never reads R.
 *   A, B, R are double for PJ_F64 and float otherwise.
 * Steps (all on `stream`): project-and-pack A (Sec. III-B, rows of A times
 * columns of C), project-and-pack B (columns of B times rows of D), one
 * MFMA contraction over r*G projected indices accumulating all r partial
 * products (eq. (8)).  Requires ws_bytes >= pj_gemm_workspace_bytes(...). */
int proj_gemm(pj_basis b, int r, char transA, char transB, int M, int W, int K,
              const void* A, int64_t lda, const void* B, int64_t ldb,
              float beta, void* R, int64_t ldr, int prec,
              void* ws, size_t ws_bytes, void* stream);

/* ---- allocation-free variant ------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): proj_gemm
 * with no workspace argument.  Its scratch (the two packed operands and, for
 * skinny outputs, the contraction-range partials) lives in one fixed array of
 * PJ_NOALLOC_SCRATCH_BYTES in device memory per GPU, reserved when the
 * library is loaded and held until the process ends.  The call allocates
 * nothing and calls no allocating routine.
 *   - Same arguments, results, layouts and errors as proj_gemm, plus
 *     PJ_ERR_SCRATCH (returned before any device work) when
 *     pj_gemm_workspace_bytes(M, W, K, L, r, prec) > PJ_NOALLOC_SCRATCH_BYTES.
 *   - Every call on one GPU shares that GPU's array and leaves its contents
 *     behind; nothing in it needs to start at zero.  Calls that overlap on
 *     one GPU (e.g. on two streams without ordering between them) race on the
 *     array and must not be issued.
 *   - The first call on a device looks the array's address up (a runtime
 *     query, no allocation) with that device current. */
#define PJ_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

int proj_gemm_noalloc(pj_basis b, int r, char transA, char transB, int M, int W, int K,
                      const void* A, int64_t lda, const void* B, int64_t ldb,
                      float beta, void* R, int64_t ldr, int prec, void* stream);

/* ---- the same path in separate steps (a static B packed once, r sweeps) --
 * A packed operand holds `rows` rows of a matrix projected onto the first
 * rmax projections, in the MFMA fragment order of `prec` (opaque layout).
 * A buffer packed at rmax serves every r <= rmax in pj_gemm_packed. */

/* Bytes of one packed operand with `rows` rows and contraction length K. */
size_t pj_packed_bytes(int rows, int K, int L, int rmax, int prec);

/* Packs the A side: rows i < M of A (layout as proj_gemm's transA),
 * projected with the columns of C (A_c = A C_N, eq. (5), (15)). */
int pj_pack_a(pj_basis b, int rmax, char transA, int M, int K, const void* A, int64_t lda,
              int prec, void* packed, size_t packed_bytes, void* stream);

/* Packs the B side: columns w < W of B (layout as proj_gemm's transB),
 * projected with the rows of D (B_d = D_N B, eq. (5), (15)). */
int pj_pack_b(pj_basis b, int rmax, char transB, int W, int K, const void* B, int64_t ldb,
              int prec, void* packed, size_t packed_bytes, void* stream);

/* Packs both sides in one launch (same arguments as pj_pack_a and pj_pack_b
 * together); the small side overlaps with the large one.  Two launches when
 * the sides need different staging (e.g. one row-contiguous, one
 * transposed with unaligned rows). */
int pj_pack_ab(pj_basis b, int rmax, char transA, char transB, int M, int W, int K,
               const void* A, int64_t lda, const void* B, int64_t ldb, int prec,
               void* Ap, size_t a_bytes, void* Bp, size_t b_bytes, void* stream);

/* R <- sum_{l<r} A_c^{(l)} B_d^{(l)} + beta R from operands packed with the
 * same (K, L, prec) at rmax_a >= r and rmax_b >= r; a_bytes and b_bytes are
 * the sizes of the two buffers (PJ_ERR_WORKSPACE if smaller than
 * pj_packed_bytes for their rmax).  tile_cfg selects the workgroup tile
 * (0 .. pj_gemm_tile_configs() - 1), or -1 for the built-in choice. */
int pj_gemm_packed(int r, int M, int W, int K, int L, int prec,
                   const void* Ap, int rmax_a, size_t a_bytes,
                   const void* Bp, int rmax_b, size_t b_bytes,
                   float beta, void* R, int64_t ldr, int tile_cfg, void* stream);

/* Number of workgroup tile configurations of the reduced contraction; writes
 * the tile sizes (rows x columns of R) of the first max_configs into tile_m,
 * tile_n when both are non-NULL.  Used by the autotuner. */
int pj_gemm_tile_configs(int prec, int* tile_m, int* tile_n, int max_configs);

/* ---------------------------------------------- projected GEMM, backward */

/* Bytes of workspace proj_gemm_backward needs (0 for invalid arguments). */
size_t pj_gemm_backward_workspace_bytes(int M, int W, int K, int L, int r, int prec);

/* Gradients of R = A Q_{r,K} B (the forward of proj_gemm) for the upstream
 * gradient dR (M x W, row stride lddr):
 *   dA = dR (D_N B)_r^T C_N^T restricted to the first r projections of each
 *        group: dA_hat = dR B_hat^T is one reduced contraction over W, then
 *        every projected value is spread back over its group with C;
 *   dB = D_N^T (A C_N)_r^T dR: dB_hat = A_hat^T dR, one reduced contraction
 *        over M, then spread back with D.
 * Both reduced contractions have r * ceil(K / L) projected indices on one
 * side, so they cost r / L of the exact gradients (paper Sec. III-C counts
 * applied to the two products of the backward pass).  A_hat and B_hat are
 * re-projected from A and B.  dA (layout of A, stride ldda) and dB (layout of
 * B, stride lddb) are overwritten; either may be NULL to skip it.  Arrays are
 * double for PJ_F64 and float otherwise; the two contractions run in `prec`. */
int proj_gemm_backward(pj_basis b, int r, char transA, char transB, int M, int W, int K,
                       const void* A, int64_t lda, const void* B, int64_t ldb,
                       const void* dR, int64_t lddr, void* dA, int64_t ldda, void* dB, int64_t lddb,
                       int prec, void* ws, size_t ws_bytes, void* stream);

/* Bytes of the plain projections proj_gemm_save keeps (0 for invalid
 * arguments): A_hat (M x r*Gp) then, at the next 256-byte boundary, B_hat
 * (W x r*Gp), row-major, element (p, l*Gp + j) = projection l of group j of
 * row p, Gp = ceil(K / L) rounded up to the precision's k-block (16 for the
 * 16-bit formats, 64 for FP8, 8 otherwise); double for PJ_F64, else float. */
size_t pj_gemm_saved_bytes(int M, int W, int K, int L, int r, int prec);

/* proj_gemm that also writes the plain projections A C_N and D_N B of its
 * pack step (paper Sec. III-B, the projected operands of eq. (8)) into
 * `saved` (pj_gemm_saved_bytes, caller-owned device memory), so that
 * proj_gemm_backward_saved pays the projection cost of eq. (17) once per
 * operand instead of again in the backward.  The values are the ones the
 * contraction consumed, before their conversion to `prec`.  Errors as
 * proj_gemm, plus PJ_ERR_ARG for a NULL `saved` and PJ_ERR_WORKSPACE when
 * saved_bytes is too small. */
int proj_gemm_save(pj_basis b, int r, char transA, char transB, int M, int W, int K,
                   const void* A, int64_t lda, const void* B, int64_t ldb,
                   float beta, void* R, int64_t ldr, int prec, void* ws, size_t ws_bytes,
                   void* saved, size_t saved_bytes, void* stream);

/* Bytes of workspace proj_gemm_backward_saved needs (0 for invalid arguments). */
size_t pj_gemm_backward_saved_workspace_bytes(int M, int W, int K, int L, int r, int prec);

/* proj_gemm_backward from the projections a proj_gemm_save call with the same
 * basis, r, shapes and prec kept: the same two reduced contractions and
 * syntheses, without re-projecting A and B.  `saved` is read only.  Errors
 * as proj_gemm_backward; PJ_ERR_WORKSPACE when saved_bytes is too small. */
int proj_gemm_backward_saved(pj_basis b, int r, char transA, char transB, int M, int W, int K,
                             const void* saved, size_t saved_bytes,
                             const void* dR, int64_t lddr, void* dA, int64_t ldda, void* dB, int64_t lddb,
                             int prec, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------- batched projected GEMM */

/* One problem of a batch: R <- A Q_{r,K} B + beta R with proj_gemm's
 * layout conventions (trans 'N' / 'T', row-major, leading dimensions). */
typedef struct {
    int M, W, K;
    char transA, transB;
    const void* A; int64_t lda;
    const void* B; int64_t ldb;
    void* R; int64_t ldr;
} pj_gemm_desc;

/* Bytes of workspace proj_gemm_batched needs (0 for invalid arguments). */
size_t pj_gemm_batched_workspace_bytes(int count, const pj_gemm_desc* problems, int L, int r, int prec,
                                       int tile_cfg);

/* Many independent projected GEMMs of any sizes sharing one basis, r and
 * precision (paper Sec. III-B applied to each problem): one grouped launch
 * per operand staging mode (at most three: rows streamed straight into LDS,
 * transposed rows streamed into LDS, register staging) projects and packs
 * every A and B side, and ONE persistent launch computes every (problem,
 * output tile) item, the items sorted by decreasing contraction length and
 * dealt round-robin over a grid sized to the device.
 *   problems : host array of `count` descriptors (device pointers inside).
 *   tile_cfg : workgroup tile as in pj_gemm_packed (-1: built-in choice);
 *              the autotuner picks it per batch.
 * The problem and item tables (a few KB) are copied into the workspace with
 * hipMemcpyAsync from host memory; the call returns once they are staged.
 * That copy reads host memory the call owns, so the batched calls are not for
 * stream capture (proj_gemm, proj_gemm_noalloc and proj_conv1d enqueue
 * kernels only and are).
 * Errors: any invalid descriptor rejects the whole batch before device work. */
int proj_gemm_batched(pj_basis b, int r, int count, const pj_gemm_desc* problems, float beta, int prec,
                      int tile_cfg, void* ws, size_t ws_bytes, void* stream);

/* The persistent launch runs each problem's output tiles either in the tile
 * of configuration tile_cfg or in its small tile (one 32 x 32 MFMA block per
 * wave on the same waves: 64 x 64 for four-wave configurations), so that
 * problems whose sides the large tile would mostly pad get tiles of their own
 * size within the same launch (paper Sec. II-A: the block size is a tuned,
 * per-case choice).  proj_gemm_batched picks per problem by padded area;
 * proj_gemm_batched_tiles takes the choice from `small` (host array of
 * `count` bytes, nonzero = small tile), e.g. from the autotuner.  Workspace
 * and errors as proj_gemm_batched; a NULL `small` is PJ_ERR_ARG (0 bytes). */
size_t pj_gemm_batched_tiles_workspace_bytes(int count, const pj_gemm_desc* problems, const unsigned char* small,
                                             int L, int r, int prec, int tile_cfg);
int proj_gemm_batched_tiles(pj_basis b, int r, int count, const pj_gemm_desc* problems, const unsigned char* small,
                            float beta, int prec, int tile_cfg, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------- projected cross-correlation */

/* Bytes of workspace proj_conv1d needs (0 for invalid arguments); that of
 * the realisation it picks for these sizes (see proj_conv1d_method). */
size_t pj_conv1d_workspace_bytes(int64_t W, int N, int L, int r, int prec);

/* Valid cross-correlation (mode PJ_XCORR) or convolution (PJ_CONV) of the
 * signal s (W samples) with the kernel k (N samples, 1 <= N <= W), computed on
 * the first r projections (paper Sec. II-B eq. (3); Sec. III-A eq. (10)-(14);
 * Sec. III-B, projection during the blocking of the input):
 *   XCORR: y[m] = sum_{n<N} k[n]       s_r[m + n],  m = 0 .. W - N
 *   CONV : y[m] = sum_{n<N} k[N-1-n]   s_r[m + n]
 * where s_r is s with every aligned block of L samples (zero-extended past W)
 * replaced by its reconstruction from the first r projections,
 * s_r|block = s|block C[:, :r] D[:r, :].  Equivalently the signal blocks are
 * projected with C, the kernel is projected with D at each of the L phases,
 * and each output accumulates r products (exact at r = L).
 *   s, k, y : device float arrays (y has W - N + 1 elements).
 *   prec    : PJ_F32 (FP32 projections, FP32 matrix-core accumulation).
 * Requires ws_bytes >= pj_conv1d_workspace_bytes(...). */
int proj_conv1d(pj_basis b, int r, int mode, int64_t W, const float* s, int N, const float* k,
                float* y, int prec, void* ws, size_t ws_bytes, void* stream);

/* proj_conv1d with the realisation chosen by the caller (pj_conv_method).
 * PJ_CONV_AUTO is proj_conv1d itself: it takes the frequency-domain
 * realisation when a cost model of both (fitted to MI355X measurements; the
 * direct cost grows with r * (N / L + 1) per output, the FFT cost with
 * (r + L) log2 F per output row) estimates it at least 20 % faster, which
 * happens for long kernels at small L.  Same arguments, results and errors as
 * proj_conv1d; PJ_ERR_ARG for another method; PJ_CONV_FFT as
 * proj_conv1d_fft.  Requires ws_bytes >=
 * pj_conv1d_method_workspace_bytes(W, N, L, r, method, prec). */
int proj_conv1d_method(pj_basis b, int r, int mode, int method, int64_t W, const float* s, int N,
                       const float* k, float* y, int prec, void* ws, size_t ws_bytes, void* stream);
size_t pj_conv1d_method_workspace_bytes(int64_t W, int N, int L, int r, int method, int prec);

/* Bytes of workspace proj_conv1d_fft needs (0 for invalid arguments, or when
 * the kernel is too long for the largest transform: more than 4096 taps per
 * phase, (N + L - 2) / L + 1 > 4096). */
size_t pj_conv1d_fft_workspace_bytes(int64_t W, int N, int L, int r, int prec);

/* proj_conv1d's result (full rate, every output) computed in the frequency
 * domain (paper Sec. III-A: the correlation of the projected signal with the
 * projected kernel may use FFTs; Sec. III-C eq. (21) models its cost).  For
 * every output phase b and projection l the T = (N + L - 2) / L + 1 taps
 * h_{l,b}[c] = sum_u D[l, u] k'(cL - b + u) and overlapping segments of the
 * projected signal row are transformed with F-point FFTs (F a power of two,
 * 512 <= F <= 4096, three quarters of it left for outputs where the taps
 * allow), the spectra are
 * multiplied (conjugate taps) and summed over l, and one inverse transform
 * per phase and segment gives F - T + 1 consecutive rows of outputs.  FP32
 * throughout; the rounding error is that of the FFTs, about u log2(F) times
 * the product of the segment's l2 norm and the taps' l1 norm, spread over all
 * outputs (rather than the per-output bound of the direct path).  Worth it
 * when ceil(N / L) is large and L small: the direct contraction costs about
 * N / L products per output and projection, this one about 4 log2 F.
 * Same arguments, errors and ownership as proj_conv1d; PJ_ERR_UNSUPPORTED when
 * the taps do not fit.  Requires ws_bytes >= pj_conv1d_fft_workspace_bytes(...). */
int proj_conv1d_fft(pj_basis b, int r, int mode, int64_t W, const float* s, int N, const float* k,
                    float* y, int prec, void* ws, size_t ws_bytes, void* stream);

/* Bytes of workspace proj_conv1d_rate needs for the given rate (0 for
 * invalid arguments).  For PJ_RATE_FULL this is pj_conv1d_workspace_bytes. */
size_t pj_conv1d_rate_workspace_bytes(int64_t W, int N, int L, int r, int rate, int prec);

/* proj_conv1d with a choice of output rate (paper Sec. III-A: results may be
 * omitted and interpolated from the neighbouring ones; Sec. IV-A: one
 * projection at half the sampling rate with L = 2, interpolating the missing
 * samples):
 *   PJ_RATE_FULL : every output, exactly as proj_conv1d.
 *   PJ_RATE_BLOCK: only the outputs m = aL (a = 0 .. (W - N) / L) are
 *     computed -- the aligned signal blocks projected with C against the
 *     aligned kernel blocks projected with D, summed over the first r
 *     projections (the same values proj_conv1d gives there).  An output
 *     aL + f, 0 < f < L, with a next computed output (a+1)L <= W - N is the
 *     linear interpolation y[aL] + (f / L) (y[(a+1)L] - y[aL]) (for L = 2 the
 *     average of its two neighbours); past the last computed output the value
 *     of that output is held.  The work is about 1/L of the full rate.
 * Same arguments, errors and ownership as proj_conv1d; rate outside the enum
 * gives PJ_ERR_ARG.  Requires ws_bytes >= pj_conv1d_rate_workspace_bytes(...). */
int proj_conv1d_rate(pj_basis b, int r, int mode, int rate, int64_t W, const float* s, int N, const float* k,
                     float* y, int prec, void* ws, size_t ws_bytes, void* stream);

/* Bytes of workspace proj_conv1d_circular needs (0 for invalid arguments). */
size_t pj_conv1d_circular_workspace_bytes(int64_t W, int N, int L, int r, int prec);

/* Circular cross-correlation (PJ_XCORR) or convolution (PJ_CONV) of the
 * periodic signal s (period W) with the kernel k (N samples, 1 <= N <= W),
 * computed on the first r projections (paper Sec. II-B eq. (4); Sec. III-A,
 * cyclic translations of the input):
 *   XCORR: y[m] = sum_{n<N} k[n]     s_r[(m + n) mod W],  m = 0 .. W - 1
 *   CONV : y[m] = sum_{n<N} k[N-1-n] s_r[(m + n) mod W]
 * with s_r the signal whose aligned L-blocks are replaced by their
 * reconstruction from the first r projections (as in proj_conv1d).  W must be
 * a multiple of L (the block grid of a periodic signal repeats only then).
 *   s, k : device float arrays; y : device float array of W elements.
 *   prec : PJ_F32.
 * Errors as proj_conv1d; W not a multiple of L gives PJ_ERR_SHAPE.
 * Requires ws_bytes >= pj_conv1d_circular_workspace_bytes(...). */
int proj_conv1d_circular(pj_basis b, int r, int mode, int64_t W, const float* s, int N, const float* k, float* y,
                         int prec, void* ws, size_t ws_bytes, void* stream);

/* ---- data-adaptive (Karhunen-Loeve) basis ------------------------------------
 * The paper uses fixed bases (DCT-II, Haar) and names projection coefficients
 * derived offline from training data by principal component analysis as the
 * route to higher precision at fewer projections (Sec. IV-B footnote, Sec. VI).
 * These two calls build such a basis: the block second moments of training
 * rows on the device, then an orthonormal eigenbasis on the host. */

/* Bytes of workspace pj_block_moments needs (0 for invalid arguments). */
size_t pj_block_moments_workspace_bytes(int64_t rows, int64_t K, int L);

/* M[t, u] = sum_i sum_j X[i, jL + t] X[i, jL + u]  (t, u < L): the second-moment
 * matrix of the aligned L-blocks of the rows of X (K zero-extended to a
 * multiple of L), accumulated in FP64.
 *   X : device FP32, rows x K row-major, leading dimension ld >= K.
 *   M : device FP64, L x L row-major, overwritten.
 * Errors: PJ_ERR_ARG (null pointer, L outside 1..256), PJ_ERR_SHAPE (rows,
 * K < 1 or ld < K), PJ_ERR_WORKSPACE, PJ_ERR_HIP.  Asynchronous on `stream`. */
int pj_block_moments(int L, int64_t rows, int64_t K, const float* X, int64_t ld, double* M, void* ws,
                     size_t ws_bytes, void* stream);

/* Orthonormal basis from a symmetric positive semidefinite L x L matrix M
 * (host FP64, row-major; typically pj_block_moments' result copied to the
 * host): the columns of C are the eigenvectors of M in order of decreasing
 * eigenvalue (cyclic Jacobi rotations in FP64), each with its largest-
 * magnitude entry positive, and D = C^T.  With this basis the first r
 * projections keep the largest possible share of the training blocks' energy
 * (the residual is the sum of the eigenvalues past r).
 *   eig_out : host, L doubles in the same order, or NULL.
 * The basis is used like any other (kind reported as PJ_BASIS_CUSTOM).
 * Errors: PJ_ERR_ARG (null out or M, L outside 1..256, non-finite or
 * non-symmetric M).  Uploads synchronously, like pj_basis_create. */
int pj_basis_create_klt(pj_basis* out, int L, const double* M, double* eig_out);

/* ------------------------------------------------- 2D-PCA support (Sec. V-A) */

/* Mean image and centred images of a training set (eq. (22)): X holds J
 * images of mn = m * n floats each, contiguous (device, row-major);
 * mean[e] = (1/J) sum_j X[j mn + e] (FP32, summed in image order) and
 * out[j mn + e] = X[j mn + e] - mean[e].  `out` may equal X.  Device pointers;
 * asynchronous on `stream`.  Errors: PJ_ERR_ARG (null pointer), PJ_ERR_SHAPE
 * (J or mn < 1), PJ_ERR_HIP (no device). */
int pj_images_center(int J, int64_t mn, const float* X, float* mean, float* out, void* stream);

/* out[j mn + e] = X[j mn + e] - mean[e] for T images (the test images minus
 * the training mean image, before their features Y = (B - mean) X of eq.
 * (24)).  Errors as pj_images_center. */
int pj_images_subtract(int T, int64_t mn, const float* X, const float* mean, float* out, void* stream);

/* G <- (G + G^T) / 2 in place for an n x n device matrix with row stride ld:
 * the image scatter matrix of eq. (23) is a Gram matrix, symmetric up to the
 * rounding of its projected product; the eigensolver takes the symmetric
 * part.  Errors: PJ_ERR_ARG (null G), PJ_ERR_SHAPE (n < 1, ld < n). */
int pj_symmetrize(int n, float* G, int64_t ld, void* stream);

/* Squared Frobenius distances between feature matrices (eq. (25), (26)):
 * out[i * ldo + j] = sum_{e < d} (F[i * ldf + e] - Y[j * ldy + e])^2 for the T
 * test and J training features flattened to d values each (device, FP32
 * accumulation per lane, lanes combined pairwise).  Errors: PJ_ERR_ARG (null
 * pointer), PJ_ERR_SHAPE (sizes < 1 or strides too small). */
int pj_sq_distances(int T, int J, int64_t d, const float* F, int64_t ldf, const float* Y, int64_t ldy,
                    float* out, int64_t ldo, void* stream);

/* Eigen-decomposition of a symmetric n x n matrix on the host (the same FP64
 * cyclic Jacobi rotations): w[l] are the eigenvalues in decreasing order and
 * column l of V (row-major n x n) the matching unit eigenvector, its largest-
 * magnitude entry positive.  Used for the projection axes of 2D-PCA (the
 * eigenvectors of the image scatter matrix, paper Sec. V-A) and for any
 * other principal-component step.  A, w, V are host arrays; n <= 4096.
 * Errors: PJ_ERR_ARG (null pointer, n outside 1..4096, non-finite or
 * non-symmetric A).  Cost O(n^3) per sweep. */
int pj_sym_eig(int n, const double* A, double* w, double* V);

#ifdef __cplusplus
}
#endif
#endif /* PROJGEMM_H */
