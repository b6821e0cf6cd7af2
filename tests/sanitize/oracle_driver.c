/* Drives the C oracle (oracle/oracle.c) over small shapes, every r and the
 * ragged tails, for an AddressSanitizer / UndefinedBehaviorSanitizer build:
 * any out-of-bounds access, leak or undefined operation aborts the run.
 * The values are not checked here (the pinned oracle tests do that). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void or_basis_dct2(int L, double* C);
int or_basis_haar(int L, double* C);
void or_basis_identity(int L, double* C);
int or_invert(int L, const double* C, double* D);
void or_gemm(int64_t M, int64_t K, int64_t W, const double* A, const double* B, double* R);
void or_xcorr(int64_t Ws, const double* s, int64_t N, const double* k, double* y);
void or_conv(int64_t Ws, const double* s, int64_t N, const double* k, double* y);
int or_gemm_proj(int64_t M, int64_t K, int64_t W, int L, int r, const double* A, const double* B, const double* C,
                 const double* D, double* R);
int or_gemm_proj_block(int64_t M, int64_t K, int64_t W, int L, int r, const double* A, const double* B,
                       const double* C, const double* D, int64_t nr, const int64_t* rows, int64_t nc,
                       const int64_t* cols, double* out);
int or_gemm_proj_grad(int64_t M, int64_t K, int64_t W, int L, int r, const double* A, const double* B,
                      const double* C, const double* D, const double* dR, double* dA, double* dB);
void or_project_signal(int64_t Ws, int L, int r, const double* s, const double* C, int64_t nb, double* sc);
void or_project_kernel(int64_t N, int L, int r, const double* k, const double* D, double* kd);
int or_xcorr_proj_at(int64_t Ws, const double* s, int64_t N, const double* k, int L, int r, const double* C,
                     const double* D, int64_t nm, const int64_t* ms, double* y);
int or_xcorr_proj(int64_t Ws, const double* s, int64_t N, const double* k, int L, int r, const double* C,
                  const double* D, double* y);

static uint64_t state = 88172645463325252ull;
static double rnd(void)
{
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) / 9007199254740992.0 - 0.5;
}
static double* vec(size_t n)
{
    double* p = (double*)malloc(sizeof(double) * (n ? n : 1));
    for (size_t i = 0; i < n; ++i) p[i] = rnd();
    return p;
}

int main(void)
{
    const int Ls[] = {1, 2, 3, 4, 5, 8, 16};
    for (size_t li = 0; li < sizeof(Ls) / sizeof(Ls[0]); ++li) {
        const int L = Ls[li];
        double* C = vec((size_t)L * L);
        double* D = vec((size_t)L * L);
        double* Ch = vec((size_t)L * L);
        or_basis_identity(L, C);
        or_basis_dct2(L, C);
        if (or_invert(L, C, D) != 0) return 2;
        if ((L & (L - 1)) == 0 && or_basis_haar(L, Ch) != 0) return 3;
        const int64_t Ks[] = {L, 3 * L, 3 * L + 1};
        for (int ki = 0; ki < 3; ++ki) {
            const int64_t M = 5, K = Ks[ki], W = 4;
            double* A = vec((size_t)(M * K));
            double* B = vec((size_t)(K * W));
            double* R = vec((size_t)(M * W));
            double* dR = vec((size_t)(M * W));
            double* dA = vec((size_t)(M * K));
            double* dB = vec((size_t)(K * W));
            or_gemm(M, K, W, A, B, R);
            for (int r = 1; r <= L; ++r) {
                if (or_gemm_proj(M, K, W, L, r, A, B, C, D, R) != 0) return 4;
                const int64_t rows[2] = {0, M - 1}, cols[2] = {W - 1, 1};
                double out[4];
                if (or_gemm_proj_block(M, K, W, L, r, A, B, C, D, 2, rows, 2, cols, out) != 0) return 5;
                if (or_gemm_proj_grad(M, K, W, L, r, A, B, C, D, dR, dA, dB) != 0) return 6;
            }
            free(A); free(B); free(R); free(dR); free(dA); free(dB);
        }
        const int64_t Wss[] = {1, 2 * L + 1, 7 * L + 3};
        for (int wi = 0; wi < 3; ++wi) {
            const int64_t Ws = Wss[wi];
            double* s = vec((size_t)Ws);
            for (int64_t N = 1; N <= Ws; N += 1 + Ws / 3) {
                double* k = vec((size_t)N);
                double* y = vec((size_t)(Ws - N + 1));
                or_xcorr(Ws, s, N, k, y);
                or_conv(Ws, s, N, k, y);
                for (int r = 1; r <= L; ++r) {
                    const int64_t nb = (Ws + L - 1) / L + 1;
                    double* sc = vec((size_t)(r * nb));
                    double* kd = vec((size_t)(r * (N + L - 1)));
                    or_project_signal(Ws, L, r, s, C, nb, sc);
                    or_project_kernel(N, L, r, k, D, kd);
                    if (or_xcorr_proj(Ws, s, N, k, L, r, C, D, y) != 0) return 7;
                    const int64_t ms[2] = {0, Ws - N};
                    double y2[2];
                    if (or_xcorr_proj_at(Ws, s, N, k, L, r, C, D, 2, ms, y2) != 0) return 8;
                    free(sc); free(kd);
                }
                free(k); free(y);
            }
            free(s);
        }
        free(C); free(D); free(Ch);
    }
    printf("oracle driver ok\n");
    return 0;
}
