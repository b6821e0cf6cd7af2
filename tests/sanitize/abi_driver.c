/* Drives the host side of libprojgemm's C ABI (include/projgemm.h) for an
 * AddressSanitizer / UndefinedBehaviorSanitizer build of api.cpp: basis
 * construction of every kind and size, the custom and singular paths, the
 * host eigensolvers, every workspace query and the argument checks of every
 * device entry point.  No call here reaches device work: each device entry
 * point is given an argument that its checks reject (fake pointers are never
 * dereferenced), so the driver is safe with or without a GPU. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "projgemm.h"

#define FAKE ((void*)(uintptr_t)0x1000)
#define EXPECT(cond)                                                          \
    do {                                                                      \
        if (!(cond)) {                                                        \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #cond);  \
            return 1;                                                         \
        }                                                                     \
    } while (0)

static uint64_t state = 0x9e3779b97f4a7c15ull;
static double rnd(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) / 9007199254740992.0 - 0.5;
}

int main(void)
{
    for (int s = -8; s <= 1; ++s) EXPECT(pj_status_str(s) != NULL);
    const int Ls[] = {1, 2, 3, 4, 8, 16, 64, 100, 256};
    for (size_t li = 0; li < sizeof(Ls) / sizeof(Ls[0]); ++li) {
        const int L = Ls[li];
        double* C = (double*)malloc(sizeof(double) * L * L);
        double* D = (double*)malloc(sizeof(double) * L * L);
        for (int kind = PJ_BASIS_DCT2; kind <= PJ_BASIS_IDENTITY; ++kind) {
            pj_basis b = NULL;
            int rc = pj_basis_create(&b, kind, L, NULL);
            if (kind == PJ_BASIS_HAAR && (L & (L - 1)) != 0) {
                EXPECT(rc == PJ_ERR_ARG && b == NULL);
                continue;
            }
            EXPECT(rc == PJ_OK && b != NULL);
            EXPECT(pj_basis_L(b) == L);
            EXPECT(pj_basis_get(b, C, D) == PJ_OK);
            EXPECT(pj_basis_get(b, NULL, D) == PJ_OK);
            /* argument checks of every device entry point (rejected on the host) */
            EXPECT(proj_gemm(b, 0, 'N', 'N', 8, 8, 8, FAKE, 8, FAKE, 8, 0.f, FAKE, 8, PJ_F32, FAKE, 1 << 20, NULL) == PJ_ERR_ARG);
            EXPECT(proj_gemm(b, 1, 'N', 'N', 8, 8, 8, FAKE, 7, FAKE, 8, 0.f, FAKE, 8, PJ_F32, FAKE, 1 << 20, NULL) == PJ_ERR_SHAPE);
            EXPECT(proj_gemm(b, 1, 'N', 'N', 8, 8, 8, FAKE, 8, FAKE, 8, 0.f, FAKE, 8, PJ_F32, FAKE, 16, NULL) == PJ_ERR_WORKSPACE);
            EXPECT(proj_gemm_noalloc(b, 1, 'N', 'N', 8, 8, 8, FAKE, 8, FAKE, 8, 0.f, NULL, 8, PJ_F32, NULL) == PJ_ERR_ARG);
            EXPECT(proj_gemm_noalloc(b, L, 'N', 'N', 8192, 8192, 65536, FAKE, 65536, FAKE, 8192, 0.f, FAKE, 8192, PJ_F32, NULL) == PJ_ERR_SCRATCH);
            EXPECT(pj_pack_a(b, 1, 'N', 8, 8, FAKE, 8, PJ_F32, FAKE, 1, NULL) == PJ_ERR_WORKSPACE);
            EXPECT(pj_pack_b(b, 1, 'T', 8, 8, FAKE, 4, PJ_F32, FAKE, 1 << 20, NULL) == PJ_ERR_SHAPE);
            EXPECT(pj_pack_ab(b, 1, 'N', 'X', 8, 8, 8, FAKE, 8, FAKE, 8, PJ_F32, FAKE, 1 << 20, FAKE, 1 << 20, NULL) == PJ_ERR_ARG);
            EXPECT(proj_gemm_backward(b, 1, 'N', 'N', 8, 8, 8, FAKE, 8, FAKE, 8, FAKE, 8, NULL, 8, NULL, 8, PJ_F32, FAKE, 1 << 20, NULL) == PJ_ERR_ARG);
            EXPECT(proj_conv1d(b, 1, PJ_XCORR, 10, FAKE, 11, FAKE, FAKE, PJ_F32, FAKE, 1 << 20, NULL) == PJ_ERR_SHAPE);
            EXPECT(proj_conv1d(b, 1, 7, 10, FAKE, 2, FAKE, FAKE, PJ_F32, FAKE, 1 << 20, NULL) == PJ_ERR_ARG);
            EXPECT(proj_conv1d_rate(b, 1, PJ_XCORR, 5, 10, FAKE, 2, FAKE, FAKE, PJ_F32, FAKE, 1 << 20, NULL) == PJ_ERR_ARG);
            EXPECT(proj_conv1d_rate(b, 1, PJ_XCORR, PJ_RATE_BLOCK, 100, FAKE, 20, FAKE, FAKE, PJ_F32, FAKE, 1, NULL) == PJ_ERR_WORKSPACE);
            EXPECT(proj_conv1d_circular(b, 1, PJ_XCORR, 100, FAKE, 200, FAKE, FAKE, PJ_F32, FAKE, 1 << 20, NULL) == PJ_ERR_SHAPE);
            pj_gemm_desc d;
            memset(&d, 0, sizeof(d));
            d.M = d.W = d.K = 8; d.transA = 'N'; d.transB = 'N'; d.A = FAKE; d.lda = 8; d.B = FAKE; d.ldb = 8;
            d.R = FAKE; d.ldr = 4;
            EXPECT(proj_gemm_batched(b, 1, 1, &d, 0.f, PJ_F32, -1, FAKE, 1 << 20, NULL) == PJ_ERR_SHAPE);
            EXPECT(pj_basis_destroy(b) == PJ_OK);
        }
        /* custom basis: a random (invertible) matrix, then a singular one */
        for (int i = 0; i < L * L; ++i) C[i] = rnd();
        for (int i = 0; i < L; ++i) C[i * L + i] += 4.0;
        pj_basis b = NULL;
        EXPECT(pj_basis_create(&b, PJ_BASIS_CUSTOM, L, C) == PJ_OK);
        EXPECT(pj_basis_destroy(b) == PJ_OK);
        memset(C, 0, sizeof(double) * L * L);
        EXPECT(pj_basis_create(&b, PJ_BASIS_CUSTOM, L, C) == PJ_ERR_SINGULAR && b == NULL);
        /* KLT basis and the symmetric eigensolver on a random PSD matrix */
        double* G = (double*)malloc(sizeof(double) * L * L);
        double* w = (double*)malloc(sizeof(double) * L);
        for (int i = 0; i < L * L; ++i) C[i] = rnd();
        for (int i = 0; i < L; ++i)
            for (int j = 0; j < L; ++j) {
                double acc = 0.0;
                for (int t = 0; t < L; ++t) acc += C[t * L + i] * C[t * L + j];
                G[i * L + j] = acc;
            }
        for (int i = 0; i < L; ++i)
            for (int j = 0; j < i; ++j) G[i * L + j] = G[j * L + i];
        EXPECT(pj_basis_create_klt(&b, L, G, w) == PJ_OK);
        EXPECT(pj_basis_destroy(b) == PJ_OK);
        EXPECT(pj_sym_eig(L, G, w, D) == PJ_OK);
        for (int i = 1; i < L; ++i) EXPECT(w[i] <= w[i - 1]);
        G[1 % (L * L)] += (L > 1) ? 1.0 : 0.0;          /* non-symmetric for L > 1 */
        if (L > 1) EXPECT(pj_sym_eig(L, G, w, D) == PJ_ERR_ARG);
        free(G); free(w); free(C); free(D);
    }
    pj_basis b = NULL;
    EXPECT(pj_basis_create(&b, PJ_BASIS_DCT2, 0, NULL) == PJ_ERR_ARG);
    EXPECT(pj_basis_create(&b, PJ_BASIS_DCT2, 257, NULL) == PJ_ERR_ARG);
    EXPECT(pj_basis_create(&b, 9, 8, NULL) == PJ_ERR_ARG);
    /* workspace queries over many shapes and every precision */
    for (int prec = PJ_F64; prec <= PJ_FP8X2; ++prec)
        for (int r = 1; r <= 16; r += 5) {
            EXPECT(pj_gemm_workspace_bytes(1 + r, 3000, 4097, 16, r, prec) > 0 || prec >= PJ_FP8);
            (void)pj_packed_bytes(513, 777, 16, r, prec);
            (void)pj_gemm_backward_workspace_bytes(33, 65, 100, 16, r, prec);
        }
    for (int L = 1; L <= 256; L *= 2)
        for (int rate = 0; rate < 2; ++rate) {
            EXPECT(pj_conv1d_rate_workspace_bytes(1 << 20, 1000, L, L, rate, PJ_F32) > 0);
            EXPECT(pj_conv1d_rate_workspace_bytes(5000, 4999, L, 1, rate, PJ_F32) > 0);
        }
    EXPECT(pj_conv1d_circular_workspace_bytes(4096, 300, 16, 4, PJ_F32) > 0);
    EXPECT(pj_block_moments_workspace_bytes(100, 1000, 16) > 0);
    EXPECT(pj_conv1d_workspace_bytes(10, 11, 4, 1, PJ_F32) == 0);
    int tm[32], tn[32];
    EXPECT(pj_gemm_tile_configs(PJ_F32, tm, tn, 32) > 0);
    printf("abi driver ok\n");
    return 0;
}
