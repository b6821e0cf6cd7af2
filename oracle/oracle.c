/*
 * oracle.c -- plain FP64 CPU reference for projection-based GEMM and 1-D
 * cross-correlation / convolution, following Anam, Whatmough and
 * Andreopoulos, "Precision-Energy-Throughput Scaling of Generic Matrix
 * Multiplication and Convolution Kernels via Linear Projections"
 * (IEEE TCSVT 24(11), 2014; arXiv:1411.2860).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library under
 * paper_1411_2860_amd/ includes, links or calls this file; only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark load it.  It
 * shares no code, header or table with the HIP path.
 *
 * Every routine is a direct, unblocked transcription of a definition in the
 * paper: natural-order sums in double precision, no blocking, no fusion.
 * Outer loops over independent outputs may run under OpenMP; that changes
 * no arithmetic.
 *
 * Conventions (paper Sec. III, Table I):
 *   A is M x K, B is K x W, both row-major.  The projection matrix C is
 *   L x L, row-major, C[t*L + l] = c[t, l]; column l of C is projection l
 *   (a_c = a C, eq. (5)).  D = C^{-1} (eq. (5)-(6)); row l of D projects the
 *   B side.  r is the number of projections kept, 1 <= r <= L (the paper's
 *   l + 1).  The contraction index k is split into G = ceil(K / L) groups of
 *   L consecutive indices starting at 0 (the block-diagonal C_N, D_N of
 *   eq. (15)); indices past K are zero-extended.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of OpenMP threads for the following calls (n >= 1); for timing the
 * oracle on a given number of host cores.  No effect on any result. */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

/* ------------------------------------------------------------------ bases */

/* DCT-II of eq. (7), unnormalised exactly as printed:
 * c[i, j] = cos(pi / L * (i + 1/2) * j). */
void or_basis_dct2(int L, double* C)
{
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j)
            C[i * L + j] = cos(M_PI / (double)L * ((double)i + 0.5) * (double)j);
}

/* Haar decomposition basis (Sec. IV-A, CONV experiment; Sec. V-B), as
 * +1 / -1 / 0 entries without normalisation.  Column 0 is the scaling
 * function (all ones); then the wavelets from the coarsest scale to the
 * finest, shifts ascending within a scale.  L must be a power of two.
 * Returns 0, or -1 if L is not a power of two. */
int or_basis_haar(int L, double* C)
{
    if (L < 1 || (L & (L - 1)) != 0) return -1;
    memset(C, 0, sizeof(double) * (size_t)L * (size_t)L);
    for (int t = 0; t < L; ++t) C[t * L + 0] = 1.0;
    int col = 1;
    for (int count = 1; count < L; count *= 2) {   /* 2^s wavelets at scale s */
        int len = L / count;                       /* support of each wavelet */
        for (int p = 0; p < count; ++p, ++col) {
            for (int t = 0; t < len / 2; ++t) C[(p * len + t) * L + col] = 1.0;
            for (int t = len / 2; t < len; ++t) C[(p * len + t) * L + col] = -1.0;
        }
    }
    return 0;
}

void or_basis_identity(int L, double* C)
{
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < L; ++j) C[i * L + j] = (i == j) ? 1.0 : 0.0;
}

/* D = C^{-1} by Gauss-Jordan elimination with partial pivoting on [C | I].
 * Returns 0, or -1 if a pivot is exactly zero (singular C). */
int or_invert(int L, const double* C, double* D)
{
    int n = L, w = 2 * L;
    double* aug = (double*)malloc(sizeof(double) * (size_t)n * (size_t)w);
    if (!aug) return -2;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < w; ++j)
            aug[i * w + j] = (j < n) ? C[i * n + j] : ((j - n == i) ? 1.0 : 0.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int i = col + 1; i < n; ++i)
            if (fabs(aug[i * w + col]) > fabs(aug[piv * w + col])) piv = i;
        if (aug[piv * w + col] == 0.0) { free(aug); return -1; }
        if (piv != col)
            for (int j = 0; j < w; ++j) {
                double tmp = aug[col * w + j];
                aug[col * w + j] = aug[piv * w + j];
                aug[piv * w + j] = tmp;
            }
        double p = aug[col * w + col];
        for (int j = 0; j < w; ++j) aug[col * w + j] /= p;
        for (int i = 0; i < n; ++i) {
            if (i == col) continue;
            double f = aug[i * w + col];
            if (f == 0.0) continue;
            for (int j = 0; j < w; ++j) aug[i * w + j] -= f * aug[col * w + j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) D[i * n + j] = aug[i * w + n + j];
    free(aug);
    return 0;
}

/* ------------------------------------------------------------ exact kernels */

/* R = A B (M x K times K x W); the blocked sum of eq. (2) collapsed to the
 * plain matrix product it equals. */
void or_gemm(int64_t M, int64_t K, int64_t W, const double* A, const double* B, double* R)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i)
        for (int64_t w = 0; w < W; ++w) {
            double acc = 0.0;
            for (int64_t k = 0; k < K; ++k) acc += A[i * K + k] * B[k * W + w];
            R[i * W + w] = acc;
        }
}

/* Valid cross-correlation, eq. (3) with k[m - n] replaced by k[m + n]
 * (Sec. II-B): y[m] = sum_{n<N} k[n] s[m + n], for m = 0 .. Ws - N. */
void or_xcorr(int64_t Ws, const double* s, int64_t N, const double* k, double* y)
{
    int64_t nout = Ws - N + 1;
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < nout; ++m) {
        double acc = 0.0;
        for (int64_t n = 0; n < N; ++n) acc += k[n] * s[m + n];
        y[m] = acc;
    }
}

/* Valid convolution, eq. (3): y[m] = sum_n s[n] k[m - n] over the positions
 * where the kernel lies inside the signal, written with the output index
 * starting where the kernel is fully inside: y[m] = sum_{n<N} k[N-1-n] s[m+n]. */
void or_conv(int64_t Ws, const double* s, int64_t N, const double* k, double* y)
{
    int64_t nout = Ws - N + 1;
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < nout; ++m) {
        double acc = 0.0;
        for (int64_t n = 0; n < N; ++n) acc += k[N - 1 - n] * s[m + n];
        y[m] = acc;
    }
}

/* -------------------------------------------- projected GEMM (Sec. III-A/B) */

/* Projection of the rows of A during block reordering (Sec. III-B, left half
 * of the GEMM projection figure): for each projection l < r and group j < G,
 *   Ac[l][i][j] = sum_{t<L} A[i, jL + t] * c[t, l]
 * with A zero-extended past column K.  Output Ac is r x M x G. */
void or_project_a(int64_t M, int64_t K, int L, int r, const double* A, const double* C, double* Ac)
{
    int64_t G = ceil_div(K, L);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i)
        for (int l = 0; l < r; ++l)
            for (int64_t j = 0; j < G; ++j) {
                double acc = 0.0;
                for (int t = 0; t < L; ++t) {
                    int64_t kk = j * L + t;
                    double a = (kk < K) ? A[i * K + kk] : 0.0;
                    acc += a * C[t * L + l];
                }
                Ac[((int64_t)l * M + i) * G + j] = acc;
            }
}

/* Projection of the columns of B (right half of the same figure):
 *   Bd[l][j][w] = sum_{u<L} d[l, u] * B[jL + u, w]
 * with B zero-extended past row K.  Output Bd is r x G x W. */
void or_project_b(int64_t K, int64_t W, int L, int r, const double* B, const double* D, double* Bd)
{
    int64_t G = ceil_div(K, L);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < G; ++j)
        for (int l = 0; l < r; ++l)
            for (int64_t w = 0; w < W; ++w) {
                double acc = 0.0;
                for (int u = 0; u < L; ++u) {
                    int64_t kk = j * L + u;
                    double b = (kk < K) ? B[kk * W + w] : 0.0;
                    acc += D[l * L + u] * b;
                }
                Bd[((int64_t)l * G + j) * W + w] = acc;
            }
}

/* Accumulation of the per-projection products, eq. (8) lifted to matrices
 * (Sec. III-B: (l+1) smaller GEMMs A_c B_d whose results are summed):
 *   R[i, w] = sum_{l<r} sum_{j<G} Ac[l][i][j] * Bd[l][j][w]. */
void or_accumulate(int64_t M, int64_t G, int64_t W, int r, const double* Ac, const double* Bd, double* R)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i)
        for (int64_t w = 0; w < W; ++w) {
            double acc = 0.0;
            for (int l = 0; l < r; ++l)
                for (int64_t j = 0; j < G; ++j)
                    acc += Ac[((int64_t)l * M + i) * G + j] * Bd[((int64_t)l * G + j) * W + w];
            R[i * W + w] = acc;
        }
}

/* Whole projected GEMM: project A, project B, accumulate (the three steps
 * in the order the paper applies them).  Returns 0, or -2 on allocation
 * failure. */
int or_gemm_proj(int64_t M, int64_t K, int64_t W, int L, int r, const double* A, const double* B,
                 const double* C, const double* D, double* R)
{
    int64_t G = ceil_div(K, L);
    double* Ac = (double*)malloc(sizeof(double) * (size_t)r * (size_t)M * (size_t)G);
    double* Bd = (double*)malloc(sizeof(double) * (size_t)r * (size_t)G * (size_t)W);
    if (!Ac || !Bd) { free(Ac); free(Bd); return -2; }
    or_project_a(M, K, L, r, A, C, Ac);
    or_project_b(K, W, L, r, B, D, Bd);
    or_accumulate(M, G, W, r, Ac, Bd, R);
    free(Ac);
    free(Bd);
    return 0;
}

/* Selected entries of the projected GEMM: R[rows[a], cols[b]] for all a < nr,
 * b < nc, written to out[a * nc + b].  Same three steps, restricted to the
 * requested rows of A and columns of B. */
int or_gemm_proj_block(int64_t M, int64_t K, int64_t W, int L, int r, const double* A, const double* B,
                       const double* C, const double* D, int64_t nr, const int64_t* rows, int64_t nc,
                       const int64_t* cols, double* out)
{
    int64_t G = ceil_div(K, L);
    double* As = (double*)malloc(sizeof(double) * (size_t)nr * (size_t)K);
    double* Bs = (double*)malloc(sizeof(double) * (size_t)K * (size_t)nc);
    double* Ac = (double*)malloc(sizeof(double) * (size_t)r * (size_t)nr * (size_t)G);
    double* Bd = (double*)malloc(sizeof(double) * (size_t)r * (size_t)G * (size_t)nc);
    if (!As || !Bs || !Ac || !Bd) { free(As); free(Bs); free(Ac); free(Bd); return -2; }
    (void)M;
    for (int64_t a = 0; a < nr; ++a)
        for (int64_t k = 0; k < K; ++k) As[a * K + k] = A[rows[a] * K + k];
    for (int64_t k = 0; k < K; ++k)
        for (int64_t b = 0; b < nc; ++b) Bs[k * nc + b] = B[k * W + cols[b]];
    or_project_a(nr, K, L, r, As, C, Ac);
    or_project_b(K, nc, L, r, Bs, D, Bd);
    or_accumulate(nr, G, nc, r, Ac, Bd, out);
    free(As); free(Bs); free(Ac); free(Bd);
    return 0;
}

/* Gradients of R = A Q_{r,K} B, where Q_{r,K} = blockdiag(Q_r) and
 * Q_r = C[:, :r] D[:r, :] (the product the projected GEMM computes).  Plain
 * definitions: dA = dR (Q B)^T and dB = (A Q)^T dR, with Q applied group by
 * group (zero-extended past K). */
int or_gemm_proj_grad(int64_t M, int64_t K, int64_t W, int L, int r, const double* A, const double* B,
                      const double* C, const double* D, const double* dR, double* dA, double* dB)
{
    int64_t G = ceil_div(K, L), Kp = G * L;
    double* Q = (double*)malloc(sizeof(double) * (size_t)L * (size_t)L);
    double* QB = (double*)calloc((size_t)Kp * (size_t)W, sizeof(double));   /* Kp x W */
    double* AQ = (double*)calloc((size_t)M * (size_t)Kp, sizeof(double));   /* M x Kp */
    if (!Q || !QB || !AQ) { free(Q); free(QB); free(AQ); return -2; }
    for (int t = 0; t < L; ++t)
        for (int u = 0; u < L; ++u) {
            double acc = 0.0;
            for (int l = 0; l < r; ++l) acc += C[t * L + l] * D[l * L + u];
            Q[t * L + u] = acc;
        }
    /* (Q B)[jL + t, w] = sum_u Q[t, u] B[jL + u, w] */
    for (int64_t j = 0; j < G; ++j)
        for (int t = 0; t < L; ++t)
            for (int64_t w = 0; w < W; ++w) {
                double acc = 0.0;
                for (int u = 0; u < L; ++u) {
                    int64_t kk = j * L + u;
                    if (kk < K) acc += Q[t * L + u] * B[kk * W + w];
                }
                QB[(j * L + t) * W + w] = acc;
            }
    /* (A Q)[i, jL + u] = sum_t A[i, jL + t] Q[t, u] */
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < G; ++j)
            for (int u = 0; u < L; ++u) {
                double acc = 0.0;
                for (int t = 0; t < L; ++t) {
                    int64_t kk = j * L + t;
                    if (kk < K) acc += A[i * K + kk] * Q[t * L + u];
                }
                AQ[i * Kp + j * L + u] = acc;
            }
    /* dA[i, k] = sum_w dR[i, w] (QB)[k, w] */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i)
        for (int64_t k = 0; k < K; ++k) {
            double acc = 0.0;
            for (int64_t w = 0; w < W; ++w) acc += dR[i * W + w] * QB[k * W + w];
            dA[i * K + k] = acc;
        }
    /* dB[k, w] = sum_i (AQ)[i, k] dR[i, w] */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < K; ++k)
        for (int64_t w = 0; w < W; ++w) {
            double acc = 0.0;
            for (int64_t i = 0; i < M; ++i) acc += AQ[i * Kp + k] * dR[i * W + w];
            dB[k * W + w] = acc;
        }
    free(Q); free(QB); free(AQ);
    return 0;
}

/* ------------------------------------- projected cross-correlation (Sec. III) */

/* Block projection of the signal during overlap-save blocking (Sec. III-B,
 * CONV projection figure, top half): aligned, non-overlapping groups of L
 * samples are projected onto the columns of C,
 *   sc[l][i] = sum_{t<L} s[iL + t] * c[t, l],  i < nb,
 * with s zero-extended past Ws.  Output sc is r x nb. */
void or_project_signal(int64_t Ws, int L, int r, const double* s, const double* C, int64_t nb, double* sc)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nb; ++i)
        for (int l = 0; l < r; ++l) {
            double acc = 0.0;
            for (int t = 0; t < L; ++t) {
                int64_t n = i * L + t;
                double v = (n < Ws) ? s[n] : 0.0;
                acc += v * C[t * L + l];
            }
            sc[(int64_t)l * nb + i] = acc;
        }
}

/* Projection of the kernel with the rows of D (CONV projection figure,
 * bottom half), taken at every sample offset so that outputs at all L
 * phases can be formed (the "all samples" operating point):
 *   kd[l][q + L - 1] = sum_{u<L} d[l, u] * k[q + u],  q = -(L-1) .. N-1,
 * with k zero outside [0, N).  Output kd is r x (N + L - 1). */
void or_project_kernel(int64_t N, int L, int r, const double* k, const double* D, double* kd)
{
    int64_t nq = N + L - 1;
#pragma omp parallel for schedule(static)
    for (int64_t qi = 0; qi < nq; ++qi) {
        int64_t q = qi - (L - 1);
        for (int l = 0; l < r; ++l) {
            double acc = 0.0;
            for (int u = 0; u < L; ++u) {
                int64_t n = q + u;
                double v = (n >= 0 && n < N) ? k[n] : 0.0;
                acc += D[l * L + u] * v;
            }
            kd[(int64_t)l * nq + qi] = acc;
        }
    }
}

/* Projected valid cross-correlation: every output sample accumulates the
 * products of the projected signal blocks with the projected kernel over
 * the first r projections (eq. (13) with zero extension in place of cyclic
 * translation, truncated after r terms as in eq. (14)):
 *   y[m] = sum_{l<r} sum_i sc[l][i] * kd[l][iL - m],   m = 0 .. Ws - N,
 * over the blocks i with -(L-1) <= iL - m <= N - 1.  At r = L this equals
 * or_xcorr exactly (D = C^{-1}). */
int or_xcorr_proj_at(int64_t Ws, const double* s, int64_t N, const double* k, int L, int r,
                     const double* C, const double* D, int64_t nm, const int64_t* ms, double* y)
{
    int64_t nb = ceil_div(Ws, L) + 1, nq = N + L - 1;
    double* sc = (double*)malloc(sizeof(double) * (size_t)r * (size_t)nb);
    double* kd = (double*)malloc(sizeof(double) * (size_t)r * (size_t)nq);
    if (!sc || !kd) { free(sc); free(kd); return -2; }
    or_project_signal(Ws, L, r, s, C, nb, sc);
    or_project_kernel(N, L, r, k, D, kd);
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < nm; ++a) {
        int64_t m = ms[a];
        /* smallest i with iL - m >= -(L-1) */
        int64_t i_lo = (m - (L - 1) <= 0) ? 0 : ceil_div(m - (L - 1), L);
        int64_t i_hi = (m + N - 1) / L;                     /* largest i with iL - m <= N-1 */
        double acc = 0.0;
        for (int l = 0; l < r; ++l)
            for (int64_t i = i_lo; i <= i_hi && i < nb; ++i)
                acc += sc[(int64_t)l * nb + i] * kd[(int64_t)l * nq + (i * L - m) + (L - 1)];
        y[a] = acc;
    }
    free(sc);
    free(kd);
    return 0;
}

/* All outputs m = 0 .. Ws - N of the projected cross-correlation. */
int or_xcorr_proj(int64_t Ws, const double* s, int64_t N, const double* k, int L, int r,
                  const double* C, const double* D, double* y)
{
    int64_t nout = Ws - N + 1;
    int64_t* ms = (int64_t*)malloc(sizeof(int64_t) * (size_t)nout);
    if (!ms) return -2;
    for (int64_t m = 0; m < nout; ++m) ms[m] = m;
    int rc = or_xcorr_proj_at(Ws, s, N, k, L, r, C, D, nout, ms, y);
    free(ms);
    return rc;
}
