// api.cpp -- the C ABI of libprojgemm (include/projgemm.h): FP64 basis
// construction on the host, argument validation (always before any device
// work), workspace carving and kernel launches.
#include "../../include/projgemm.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "common.h"
#include "conv.h"
#include "moments.h"
#include "pca2d.h"

using namespace pj;

struct pj_basis_s {
    int kind;
    int L;
    std::vector<double> C, D;        // FP64 host copies, row-major L x L
    bool on_device = false;
    int device = -1;
    float* Cf = nullptr;             // C[t][l]           (A side coefficients)
    float* DTf = nullptr;            // D^T[t][l] = D[l][t] (B side coefficients)
    float* CTf = nullptr;            // C^T[l][t] = C[t][l] (synthesis with C, coalesced over t)
    double* Cd = nullptr;
    double* DTd = nullptr;
    float* I4f = nullptr;            // 4 x 4 identity: packs an operand unprojected
    double* I4d = nullptr;
};

namespace {

constexpr int kMaxL = 256;

bool valid_prec(int p) { return p >= PJ_F64 && p <= PJ_FP8X2; }
bool implemented_prec(int p) { return p >= PJ_F64 && p <= PJ_FP8X2; }
bool is_n(char t) { return t == 'N' || t == 'n'; }
bool is_t(char t) { return t == 'T' || t == 't'; }

// Orthonormal DCT-II: C[t][l] = a_l cos(pi/L (t + 1/2) l), a_0 = sqrt(1/L),
// a_l = sqrt(2/L); columns are the basis vectors of eq. (7), rescaled.
void make_dct2(int L, std::vector<double>& C)
{
    const double pi = 3.14159265358979323846;
    for (int t = 0; t < L; ++t)
        for (int l = 0; l < L; ++l) {
            double a = (l == 0) ? std::sqrt(1.0 / L) : std::sqrt(2.0 / L);
            C[(size_t)t * L + l] = a * std::cos(pi / L * (t + 0.5) * l);
        }
}

// Orthonormal Haar: column 0 the scaling function, then for each scale from
// coarse to fine the shifted wavelets (+ on the first half of the support,
// - on the second), each normalised to unit length.
void make_haar(int L, std::vector<double>& C)
{
    std::fill(C.begin(), C.end(), 0.0);
    for (int t = 0; t < L; ++t) C[(size_t)t * L] = 1.0 / std::sqrt((double)L);
    int col = 1;
    for (int count = 1; count < L; count *= 2) {
        const int len = L / count;
        const double v = 1.0 / std::sqrt((double)len);
        for (int p = 0; p < count; ++p, ++col)
            for (int t = 0; t < len; ++t) C[(size_t)(p * len + t) * L + col] = (t < len / 2) ? v : -v;
    }
}

// Eigen-decomposition of a symmetric L x L matrix by cyclic Jacobi rotations
// in FP64: on return A is (numerically) diagonal with the eigenvalues and the
// columns of V are the eigenvectors.  Each rotation J in the (p, q) plane
// (J_pp = J_qq = c, J_pq = s, J_qp = -s) is chosen so that (J^T A J)_pq = 0,
// with the smaller of the two rotation angles.
void jacobi_eig(int L, std::vector<double>& A, std::vector<double>& V)
{
    V.assign((size_t)L * L, 0.0);
    for (int i = 0; i < L; ++i) V[(size_t)i * L + i] = 1.0;
    auto a = [&](int i, int j) -> double& { return A[(size_t)i * L + j]; };
    double total = 0.0;
    for (double x : A) total += x * x;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < L; ++p)
            for (int q = 0; q < L; ++q)
                if (p != q) off += a(p, q) * a(p, q);
        if (off <= 1e-30 * total || off == 0.0) break;
        for (int p = 0; p < L - 1; ++p)
            for (int q = p + 1; q < L; ++q) {
                const double apq = a(p, q);
                if (apq == 0.0) continue;
                const double tau = (a(q, q) - a(p, p)) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
                for (int k = 0; k < L; ++k) {          // columns p, q: A J
                    const double akp = a(k, p), akq = a(k, q);
                    a(k, p) = c * akp - sn * akq;
                    a(k, q) = sn * akp + c * akq;
                }
                for (int k = 0; k < L; ++k) {          // rows p, q: J^T (A J)
                    const double apk = a(p, k), aqk = a(q, k);
                    a(p, k) = c * apk - sn * aqk;
                    a(q, k) = sn * apk + c * aqk;
                }
                for (int k = 0; k < L; ++k) {          // V J
                    const double vkp = V[(size_t)k * L + p], vkq = V[(size_t)k * L + q];
                    V[(size_t)k * L + p] = c * vkp - sn * vkq;
                    V[(size_t)k * L + q] = sn * vkp + c * vkq;
                }
            }
    }
}

// D = C^{-1} by LU with partial pivoting; false if C is (numerically) singular.
bool invert_lu(int L, const std::vector<double>& C, std::vector<double>& D)
{
    std::vector<double> a(C);
    std::vector<int> piv(L);
    double amax = 0.0;
    for (double v : C) amax = std::fmax(amax, std::fabs(v));
    if (!(amax > 0.0) || !std::isfinite(amax)) return false;
    for (int k = 0; k < L; ++k) {
        int p = k;
        for (int i = k + 1; i < L; ++i)
            if (std::fabs(a[(size_t)i * L + k]) > std::fabs(a[(size_t)p * L + k])) p = i;
        if (std::fabs(a[(size_t)p * L + k]) <= 1e-12 * amax) return false;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < L; ++j) std::swap(a[(size_t)k * L + j], a[(size_t)p * L + j]);
        for (int i = k + 1; i < L; ++i) {
            a[(size_t)i * L + k] /= a[(size_t)k * L + k];
            const double f = a[(size_t)i * L + k];
            for (int j = k + 1; j < L; ++j) a[(size_t)i * L + j] -= f * a[(size_t)k * L + j];
        }
    }
    // solve A X = I column by column (rows of the identity permuted as P)
    for (int c = 0; c < L; ++c) {
        std::vector<double> x(L, 0.0);
        x[c] = 1.0;
        for (int k = 0; k < L; ++k)
            if (piv[k] != k) std::swap(x[k], x[piv[k]]);
        for (int i = 0; i < L; ++i)
            for (int j = 0; j < i; ++j) x[i] -= a[(size_t)i * L + j] * x[j];
        for (int i = L - 1; i >= 0; --i) {
            for (int j = i + 1; j < L; ++j) x[i] -= a[(size_t)i * L + j] * x[j];
            x[i] /= a[(size_t)i * L + i];
        }
        for (int i = 0; i < L; ++i) D[(size_t)i * L + c] = x[i];
    }
    return true;
}

void free_device(pj_basis b)
{
    if (!b->on_device) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(b->device);
    (void)hipFree(b->Cf);
    (void)hipFree(b->DTf);
    (void)hipFree(b->CTf);
    (void)hipFree(b->Cd);
    (void)hipFree(b->DTd);
    (void)hipFree(b->I4f);
    (void)hipFree(b->I4d);
    if (prev >= 0) (void)hipSetDevice(prev);
    b->on_device = false;
}

bool device_present()
{
    int ndev = 0;
    return hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0;
}

bool upload(pj_basis b)
{
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return false;
    }
    if (hipGetDevice(&b->device) != hipSuccess) return false;
    const int L = b->L;
    const size_t n = (size_t)L * L;
    std::vector<float> cf(n), dtf(n), ctf(n);
    std::vector<double> dtd(n);
    for (int t = 0; t < L; ++t)
        for (int l = 0; l < L; ++l) {
            cf[(size_t)t * L + l] = (float)b->C[(size_t)t * L + l];
            ctf[(size_t)l * L + t] = (float)b->C[(size_t)t * L + l];
            dtd[(size_t)t * L + l] = b->D[(size_t)l * L + t];
            dtf[(size_t)t * L + l] = (float)b->D[(size_t)l * L + t];
        }
    bool ok = hipMalloc((void**)&b->Cf, n * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&b->DTf, n * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&b->CTf, n * sizeof(float)) == hipSuccess &&
              hipMemcpy(b->CTf, ctf.data(), n * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
              hipMalloc((void**)&b->Cd, n * sizeof(double)) == hipSuccess &&
              hipMalloc((void**)&b->DTd, n * sizeof(double)) == hipSuccess &&
              hipMemcpy(b->Cf, cf.data(), n * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(b->DTf, dtf.data(), n * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(b->Cd, b->C.data(), n * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(b->DTd, dtd.data(), n * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
    const float i4f[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
    const double i4d[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
    ok = ok && hipMalloc((void**)&b->I4f, sizeof(i4f)) == hipSuccess &&
         hipMalloc((void**)&b->I4d, sizeof(i4d)) == hipSuccess &&
         hipMemcpy(b->I4f, i4f, sizeof(i4f), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->I4d, i4d, sizeof(i4d), hipMemcpyHostToDevice) == hipSuccess;
    b->on_device = true;   // so that free_device releases partial allocations
    if (!ok) {
        free_device(b);
        (void)hipGetLastError();
        return false;
    }
    return true;
}

// Common checks of one packed operand request.
int check_pack(pj_basis b, int rmax, char trans, int rows, int K, const void* X, int64_t ld, int prec,
               const void* packed, size_t packed_bytes)
{
    if (!b || !X || !packed) return PJ_ERR_ARG;
    if (!valid_prec(prec)) return PJ_ERR_ARG;
    if (rmax < 1 || rmax > b->L) return PJ_ERR_ARG;
    if (!is_n(trans) && !is_t(trans)) return PJ_ERR_ARG;
    if (rows < 1 || K < 1) return PJ_ERR_SHAPE;
    if (ld < (is_n(trans) ? (int64_t)K : (int64_t)rows)) return PJ_ERR_SHAPE;
    if ((prec == PJ_FP8 || prec == PJ_FP8X2) && rmax > 8) return PJ_ERR_UNSUPPORTED;
    if (!implemented_prec(prec)) return PJ_ERR_UNSUPPORTED;
    if (packed_bytes < (size_t)pack_geom(rows, K, b->L, rmax, prec).total) return PJ_ERR_WORKSPACE;
    return PJ_OK;
}

PackArgs pack_args(pj_basis b, int rmax, bool a_side, char trans, int rows, int K, const void* X, int64_t ld,
                   int prec, void* packed)
{
    PackArgs a;
    a.X = X;
    a.ld = ld;
    // A side: rows of A are rows (trans 'N' = k contiguous).  B side: the rows
    // of the packed operand are the columns of B, so 'N' (B is K x W) is the
    // strided case and 'T' (B stored W x K) the contiguous one.
    a.trans = a_side ? (is_t(trans) ? 1 : 0) : (is_n(trans) ? 1 : 0);
    a.P = rows;
    a.K = K;
    a.L = b->L;
    a.r = rmax;
    if (prec == PJ_F64 || prec == P_PLAIN64) a.coef = a_side ? (const void*)b->Cd : (const void*)b->DTd;
    else a.coef = a_side ? (const void*)b->Cf : (const void*)b->DTf;
    a.out = packed;
    a.geom = pack_geom(rows, K, b->L, rmax, prec);
    return a;
}

int run_pack(int prec, const PackArgs* a, int n, void* stream)
{
    for (int i = 0; i < n; ++i)
        if (a[i].geom.nrb * (a[i].geom.Gp / layout_of(prec).KB) > 0x3fffffff) return PJ_ERR_UNSUPPORTED;
    int rc = launch_pack_n(prec, a, n, (hipStream_t)stream);
    return rc == 0 ? PJ_OK : (rc == -2 ? PJ_ERR_UNSUPPORTED : PJ_ERR_HIP);
}

int do_pack(pj_basis b, int rmax, bool a_side, char trans, int rows, int K, const void* X, int64_t ld,
            int prec, void* packed, void* stream)
{
    PackArgs a = pack_args(b, rmax, a_side, trans, rows, K, X, ld, prec, packed);
    return run_pack(prec, &a, 1, stream);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

const char* pj_status_str(int s)
{
    switch (s) {
    case PJ_OK: return "ok";
    case PJ_ERR_ARG: return "invalid argument";
    case PJ_ERR_SHAPE: return "invalid shape or leading dimension";
    case PJ_ERR_UNSUPPORTED: return "unsupported request";
    case PJ_ERR_WORKSPACE: return "workspace missing or too small";
    case PJ_ERR_SINGULAR: return "projection matrix is singular";
    case PJ_ERR_HIP: return "HIP runtime or launch failure";
    case PJ_ERR_SCRATCH: return "request needs more than the fixed scratch of the allocation-free entry point";
    default: return "unknown status";
    }
}

int pj_basis_create(pj_basis* out, int kind, int L, const double* C)
{
    if (!out) return PJ_ERR_ARG;
    *out = nullptr;
    if (L < 1 || L > kMaxL) return PJ_ERR_ARG;
    if (kind < PJ_BASIS_DCT2 || kind > PJ_BASIS_CUSTOM) return PJ_ERR_ARG;
    if (kind == PJ_BASIS_CUSTOM && !C) return PJ_ERR_ARG;
    if (kind != PJ_BASIS_CUSTOM && C) return PJ_ERR_ARG;
    if (kind == PJ_BASIS_HAAR && (L & (L - 1)) != 0) return PJ_ERR_ARG;
    pj_basis b = new (std::nothrow) pj_basis_s;
    if (!b) return PJ_ERR_ARG;
    b->kind = kind;
    b->L = L;
    const size_t n = (size_t)L * L;
    b->C.assign(n, 0.0);
    b->D.assign(n, 0.0);
    switch (kind) {
    case PJ_BASIS_DCT2: make_dct2(L, b->C); break;
    case PJ_BASIS_HAAR: make_haar(L, b->C); break;
    case PJ_BASIS_IDENTITY:
        for (int i = 0; i < L; ++i) b->C[(size_t)i * L + i] = 1.0;
        break;
    default: std::memcpy(b->C.data(), C, n * sizeof(double)); break;
    }
    if (kind == PJ_BASIS_CUSTOM) {
        if (!invert_lu(L, b->C, b->D)) {
            delete b;
            return PJ_ERR_SINGULAR;
        }
    } else {   // orthonormal kinds: D = C^T
        for (int t = 0; t < L; ++t)
            for (int l = 0; l < L; ++l) b->D[(size_t)l * L + t] = b->C[(size_t)t * L + l];
    }
    upload(b);
    *out = b;
    return PJ_OK;
}

int pj_basis_get(pj_basis b, double* C_out, double* D_out)
{
    if (!b) return PJ_ERR_ARG;
    const size_t n = (size_t)b->L * b->L;
    if (C_out) std::memcpy(C_out, b->C.data(), n * sizeof(double));
    if (D_out) std::memcpy(D_out, b->D.data(), n * sizeof(double));
    return PJ_OK;
}

int pj_basis_L(pj_basis b) { return b ? b->L : PJ_ERR_ARG; }

int pj_basis_destroy(pj_basis b)
{
    if (!b) return PJ_ERR_ARG;
    free_device(b);
    delete b;
    return PJ_OK;
}

size_t pj_packed_bytes(int rows, int K, int L, int rmax, int prec)
{
    if (rows < 1 || K < 1 || L < 1 || L > kMaxL || rmax < 1 || rmax > L || !valid_prec(prec)) return 0;
    return (size_t)pack_geom(rows, K, L, rmax, prec).total;
}

// Bytes of the k-range partials proj_gemm uses for a skinny output (0 if the
// contraction is not split).
static size_t gemm_split_bytes(int M, int W, int K, int L, int r, int prec)
{
    const PackGeom g = pack_geom(M, K, L, r, prec);
    const int64_t nkb = (int64_t)r * g.Gp / layout_of(prec).KB;
    const int ns = gemm_split_count(prec, M, W, nkb, -1);
    if (ns <= 1) return 0;
    return align256((size_t)ns * M * W * (prec == PJ_F64 ? 8 : 4));
}

size_t pj_gemm_workspace_bytes(int M, int W, int K, int L, int r, int prec)
{
    size_t a = pj_packed_bytes(M, K, L, r, prec), b = pj_packed_bytes(W, K, L, r, prec);
    if (!a || !b) return 0;
    return align256(a) + align256(b) + gemm_split_bytes(M, W, K, L, r, prec);
}

int pj_pack_a(pj_basis b, int rmax, char transA, int M, int K, const void* A, int64_t lda, int prec,
              void* packed, size_t packed_bytes, void* stream)
{
    int rc = check_pack(b, rmax, transA, M, K, A, lda, prec, packed, packed_bytes);
    if (rc != PJ_OK) return rc;
    if (!b->on_device) return PJ_ERR_HIP;
    return do_pack(b, rmax, true, transA, M, K, A, lda, prec, packed, stream);
}

int pj_pack_b(pj_basis b, int rmax, char transB, int W, int K, const void* B, int64_t ldb, int prec,
              void* packed, size_t packed_bytes, void* stream)
{
    // B side: 'N' means B is K x W, so the required leading dimension is W
    if (!b || !B || !packed) return PJ_ERR_ARG;
    if (!is_n(transB) && !is_t(transB)) return PJ_ERR_ARG;
    if (W >= 1 && K >= 1 && ldb < (is_n(transB) ? (int64_t)W : (int64_t)K)) return PJ_ERR_SHAPE;
    int rc = check_pack(b, rmax, is_n(transB) ? 'T' : 'N', W, K, B, ldb, prec, packed, packed_bytes);
    if (rc != PJ_OK) return rc;
    if (!b->on_device) return PJ_ERR_HIP;
    return do_pack(b, rmax, false, transB, W, K, B, ldb, prec, packed, stream);
}

int pj_gemm_tile_configs(int prec, int* tile_m, int* tile_n, int max_configs)
{
    if (!valid_prec(prec)) return PJ_ERR_ARG;
    const int n = gemm_num_configs();
    for (int i = 0; i < n && i < max_configs; ++i)
        if (tile_m && tile_n) gemm_config_tile(prec, i, &tile_m[i], &tile_n[i]);
    return n;
}

int pj_pack_ab(pj_basis b, int rmax, char transA, char transB, int M, int W, int K, const void* A, int64_t lda,
               const void* B, int64_t ldb, int prec, void* Ap, size_t a_bytes, void* Bp, size_t b_bytes,
               void* stream)
{
    if (!b || !B || !Bp) return PJ_ERR_ARG;
    if (!is_n(transB) && !is_t(transB)) return PJ_ERR_ARG;
    int rc = check_pack(b, rmax, transA, M, K, A, lda, prec, Ap, a_bytes);
    if (rc != PJ_OK) return rc;
    rc = check_pack(b, rmax, is_n(transB) ? 'T' : 'N', W, K, B, ldb, prec, Bp, b_bytes);
    if (rc != PJ_OK) return rc;
    if (!b->on_device) return PJ_ERR_HIP;
    PackArgs pa[2] = {pack_args(b, rmax, true, transA, M, K, A, lda, prec, Ap),
                      pack_args(b, rmax, false, transB, W, K, B, ldb, prec, Bp)};
    return run_pack(prec, pa, 2, stream);
}

// pj_gemm_packed with optional k-range partials (nsplit > 1 needs `part`).
static int gemm_packed_impl(int r, int M, int W, int K, int L, int prec, const void* Ap, int rmax_a,
                            size_t a_bytes, const void* Bp, int rmax_b, size_t b_bytes, float beta, void* R,
                            int64_t ldr, int tile_cfg, int nsplit, void* part, void* stream);

int pj_gemm_packed(int r, int M, int W, int K, int L, int prec, const void* Ap, int rmax_a, size_t a_bytes,
                   const void* Bp, int rmax_b, size_t b_bytes, float beta, void* R, int64_t ldr, int tile_cfg,
                   void* stream)
{
    return gemm_packed_impl(r, M, W, K, L, prec, Ap, rmax_a, a_bytes, Bp, rmax_b, b_bytes, beta, R, ldr, tile_cfg, 1,
                            nullptr, stream);
}

static int gemm_packed_impl(int r, int M, int W, int K, int L, int prec, const void* Ap, int rmax_a,
                            size_t a_bytes, const void* Bp, int rmax_b, size_t b_bytes, float beta, void* R,
                            int64_t ldr, int tile_cfg, int nsplit, void* part, void* stream)
{
    if (!Ap || !Bp || !R) return PJ_ERR_ARG;
    if (!valid_prec(prec)) return PJ_ERR_ARG;
    if (L < 1 || L > kMaxL) return PJ_ERR_ARG;
    if (r < 1 || r > L || rmax_a < r || rmax_b < r || rmax_a > L || rmax_b > L) return PJ_ERR_ARG;
    if (M < 1 || W < 1 || K < 1) return PJ_ERR_SHAPE;
    if (ldr < W) return PJ_ERR_SHAPE;
    if ((prec == PJ_FP8 || prec == PJ_FP8X2) && r > 8) return PJ_ERR_UNSUPPORTED;
    if (!implemented_prec(prec)) return PJ_ERR_UNSUPPORTED;
    if (a_bytes < (size_t)pack_geom(M, K, L, rmax_a, prec).total ||
        b_bytes < (size_t)pack_geom(W, K, L, rmax_b, prec).total)
        return PJ_ERR_WORKSPACE;
    GemmArgs g;
    g.X = Ap;
    g.gx = pack_geom(M, K, L, rmax_a, prec);
    g.Y = Bp;
    g.gy = pack_geom(W, K, L, rmax_b, prec);
    g.nkb = (int64_t)r * g.gx.Gp / layout_of(prec).KB;
    g.P = M;
    g.Q = W;
    g.R = R;
    g.ldr = ldr;
    g.beta = beta;
    g.nsplit = part ? nsplit : 1;
    g.part = part;
    if (tile_cfg >= gemm_num_configs()) return PJ_ERR_ARG;
    int rc = launch_gemm(prec, g, tile_cfg, (hipStream_t)stream);
    return rc == 0 ? PJ_OK : (rc == -2 ? PJ_ERR_UNSUPPORTED : PJ_ERR_HIP);
}

// Plain projections kept by proj_gemm_save: A_hat (M x rG) then B_hat
// (W x rG), rG = r * Gp with the packed geometry's Gp, FP64 for PJ_F64.
struct SavedGeom {
    int64_t Gp, rg;
    size_t bhat, total;
};
static SavedGeom saved_geom(int M, int W, int K, int L, int r, int prec)
{
    SavedGeom g;
    g.Gp = pack_geom(1, K, L, r, prec).Gp;
    g.rg = (int64_t)r * g.Gp;
    const int64_t T = prec == PJ_F64 ? 8 : 4;
    g.bhat = align256((size_t)M * g.rg * T);
    g.total = g.bhat + align256((size_t)W * g.rg * T);
    return g;
}

// Argument checks of proj_gemm (host only, before any device work).
static int check_proj_gemm(pj_basis b, int r, char transA, char transB, int M, int W, int K, const void* A,
                           int64_t lda, const void* B, int64_t ldb, const void* R, int64_t ldr, int prec)
{
    if (!b || !A || !B || !R) return PJ_ERR_ARG;
    if (!valid_prec(prec)) return PJ_ERR_ARG;
    if (r < 1 || r > b->L) return PJ_ERR_ARG;
    if ((!is_n(transA) && !is_t(transA)) || (!is_n(transB) && !is_t(transB))) return PJ_ERR_ARG;
    if (M < 1 || W < 1 || K < 1) return PJ_ERR_SHAPE;
    if (lda < (is_n(transA) ? (int64_t)K : (int64_t)M)) return PJ_ERR_SHAPE;
    if (ldb < (is_n(transB) ? (int64_t)W : (int64_t)K)) return PJ_ERR_SHAPE;
    if (ldr < W) return PJ_ERR_SHAPE;
    if ((prec == PJ_FP8 || prec == PJ_FP8X2) && r > 8) return PJ_ERR_UNSUPPORTED;
    if (!implemented_prec(prec)) return PJ_ERR_UNSUPPORTED;
    return PJ_OK;
}

// The device work of proj_gemm on a checked request and a workspace of at
// least pj_gemm_workspace_bytes: pack both sides, then contract.
static int run_proj_gemm(pj_basis b, int r, char transA, char transB, int M, int W, int K, const void* A,
                         int64_t lda, const void* B, int64_t ldb, float beta, void* R, int64_t ldr, int prec,
                         void* ws, void* stream, void* keep = nullptr)
{
    char* wa = (char*)ws;
    char* wb = wa + align256(pj_packed_bytes(M, K, b->L, r, prec));
    char* wp = wb + align256(pj_packed_bytes(W, K, b->L, r, prec));
    PackArgs pa[2] = {pack_args(b, r, true, transA, M, K, A, lda, prec, wa),
                      pack_args(b, r, false, transB, W, K, B, ldb, prec, wb)};
    if (keep) {
        const SavedGeom sg = saved_geom(M, W, K, b->L, r, prec);
        pa[0].keep = keep;
        pa[1].keep = (char*)keep + sg.bhat;
        pa[0].keep_ld = pa[1].keep_ld = sg.rg;
    }
    int rc = run_pack(prec, pa, 2, stream);
    if (rc != PJ_OK) return rc;
    const PackGeom ga = pack_geom(M, K, b->L, r, prec);
    const int ns = gemm_split_bytes(M, W, K, b->L, r, prec) > 0
                       ? gemm_split_count(prec, M, W, (int64_t)r * ga.Gp / layout_of(prec).KB, -1)
                       : 1;
    return gemm_packed_impl(r, M, W, K, b->L, prec, wa, r, pj_packed_bytes(M, K, b->L, r, prec), wb, r,
                            pj_packed_bytes(W, K, b->L, r, prec), beta, R, ldr, -1, ns, ns > 1 ? wp : nullptr,
                            stream);
}

int proj_gemm(pj_basis b, int r, char transA, char transB, int M, int W, int K, const void* A, int64_t lda,
              const void* B, int64_t ldb, float beta, void* R, int64_t ldr, int prec, void* ws, size_t ws_bytes,
              void* stream)
{
    int rc = check_proj_gemm(b, r, transA, transB, M, W, K, A, lda, B, ldb, R, ldr, prec);
    if (rc != PJ_OK) return rc;
    const size_t need = pj_gemm_workspace_bytes(M, W, K, b->L, r, prec);
    if (!ws || ws_bytes < need) return PJ_ERR_WORKSPACE;
    if (!b->on_device) return PJ_ERR_HIP;
    return run_proj_gemm(b, r, transA, transB, M, W, K, A, lda, B, ldb, beta, R, ldr, prec, ws, stream);
}

size_t pj_gemm_saved_bytes(int M, int W, int K, int L, int r, int prec)
{
    if (M < 1 || W < 1 || K < 1 || L < 1 || L > kMaxL || r < 1 || r > L || !valid_prec(prec)) return 0;
    return saved_geom(M, W, K, L, r, prec).total;
}

int proj_gemm_save(pj_basis b, int r, char transA, char transB, int M, int W, int K, const void* A, int64_t lda,
                   const void* B, int64_t ldb, float beta, void* R, int64_t ldr, int prec, void* ws,
                   size_t ws_bytes, void* saved, size_t saved_bytes, void* stream)
{
    int rc = check_proj_gemm(b, r, transA, transB, M, W, K, A, lda, B, ldb, R, ldr, prec);
    if (rc != PJ_OK) return rc;
    if (!saved) return PJ_ERR_ARG;
    if (saved_bytes < saved_geom(M, W, K, b->L, r, prec).total) return PJ_ERR_WORKSPACE;
    const size_t need = pj_gemm_workspace_bytes(M, W, K, b->L, r, prec);
    if (!ws || ws_bytes < need) return PJ_ERR_WORKSPACE;
    if (!b->on_device) return PJ_ERR_HIP;
    return run_proj_gemm(b, r, transA, transB, M, W, K, A, lda, B, ldb, beta, R, ldr, prec, ws, stream, saved);
}

}  // extern "C"

// ------------------------------------------------- allocation-free variant
//
// proj_gemm_noalloc runs proj_gemm's kernels on a fixed scratch array in
// device memory instead of a caller workspace, for callers that cannot
// allocate.  Each device holds its own copy of the array at its own address;
// in host code `scratch` is only a stand-in for that address, so the address
// is looked up once per device (hipGetSymbolAddress, with that device
// current) and only the looked-up pointer is ever handed to kernels.
namespace {

static_assert(PJ_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");
static __device__ __align__(256) unsigned char scratch[PJ_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the current device's copy of `scratch`.
int current_scratch(void** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) {
        (void)hipGetLastError();
        return PJ_ERR_HIP;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return PJ_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PJ_OK;
}

}  // namespace

extern "C" {

int proj_gemm_noalloc(pj_basis b, int r, char transA, char transB, int M, int W, int K, const void* A, int64_t lda,
                      const void* B, int64_t ldb, float beta, void* R, int64_t ldr, int prec, void* stream)
{
    int rc = check_proj_gemm(b, r, transA, transB, M, W, K, A, lda, B, ldb, R, ldr, prec);
    if (rc != PJ_OK) return rc;
    if (pj_gemm_workspace_bytes(M, W, K, b->L, r, prec) > PJ_NOALLOC_SCRATCH_BYTES) return PJ_ERR_SCRATCH;
    if (!b->on_device) return PJ_ERR_HIP;
    void* ws = nullptr;
    rc = current_scratch(&ws);
    if (rc != PJ_OK) return rc;
    return run_proj_gemm(b, r, transA, transB, M, W, K, A, lda, B, ldb, beta, R, ldr, prec, ws, stream);
}

// ---------------------------------------------------------------- batched

namespace {

struct BatchPlan {
    size_t pack_table, probs_off, items_off, ops_off, total;
    std::vector<size_t> a_off, b_off;
    std::vector<unsigned char> small;   // per problem: the small tile body
    int64_t nitems;
    int cfg;
};

// Automatic per-problem body: the small tile when the configuration's tile
// pads the problem's M x W to more than 1.6 times the area the small tile
// pads it to (about the small body's loss of rate per unit of area).
bool prefer_small(int M, int W, int tm, int tn, int sm, int sn)
{
    const double big = (double)rup(M, tm) * (double)rup(W, tn);
    const double small = (double)rup(M, sm) * (double)rup(W, sn);
    return big > 1.6 * small;
}

int check_desc(const pj_gemm_desc& d)
{
    if (!d.A || !d.B || !d.R) return PJ_ERR_ARG;
    if ((!is_n(d.transA) && !is_t(d.transA)) || (!is_n(d.transB) && !is_t(d.transB))) return PJ_ERR_ARG;
    if (d.M < 1 || d.W < 1 || d.K < 1) return PJ_ERR_SHAPE;
    if (d.lda < (is_n(d.transA) ? (int64_t)d.K : (int64_t)d.M)) return PJ_ERR_SHAPE;
    if (d.ldb < (is_n(d.transB) ? (int64_t)d.W : (int64_t)d.K)) return PJ_ERR_SHAPE;
    if (d.ldr < d.W) return PJ_ERR_SHAPE;
    return PJ_OK;
}

int plan_batch(int count, const pj_gemm_desc* p, int L, int r, int prec, int tile_cfg, BatchPlan& bp,
               const unsigned char* small = nullptr)
{
    if (count < 1 || !p) return PJ_ERR_ARG;
    if (L < 1 || L > kMaxL || r < 1 || r > L || !valid_prec(prec)) return PJ_ERR_ARG;
    if (tile_cfg >= gemm_num_configs()) return PJ_ERR_ARG;
    for (int i = 0; i < count; ++i) {
        int rc = check_desc(p[i]);
        if (rc != PJ_OK) return rc;
    }
    if ((prec == PJ_FP8 || prec == PJ_FP8X2) && r > 8) return PJ_ERR_UNSUPPORTED;
    bp.cfg = tile_cfg;
    if (bp.cfg < 0) bp.cfg = 0;
    int tm = 0, tn = 0, sm = 0, sn = 0;
    gemm_config_tile(prec, bp.cfg, &tm, &tn);
    gemm_config_small_tile(prec, bp.cfg, &sm, &sn);
    bp.nitems = 0;
    bp.a_off.resize(count);
    bp.b_off.resize(count);
    bp.small.resize(count);
    for (int i = 0; i < count; ++i)
        bp.small[i] = small ? (small[i] ? 1 : 0) : (prefer_small(p[i].M, p[i].W, tm, tn, sm, sn) ? 1 : 0);
    size_t off = 0;
    bp.pack_table = rup((int64_t)pack_grouped_table_bytes(2 * count), 256);
    off += bp.pack_table;
    bp.probs_off = off;
    off += rup((int64_t)sizeof(GroupedProblem) * count, 256);
    for (int i = 0; i < count; ++i)
        bp.nitems += bp.small[i] ? cdiv(p[i].M, sm) * cdiv(p[i].W, sn) : cdiv(p[i].M, tm) * cdiv(p[i].W, tn);
    bp.items_off = off;
    off += rup((int64_t)sizeof(GroupedItem) * bp.nitems, 256);
    bp.ops_off = off;
    for (int i = 0; i < count; ++i) {
        bp.a_off[i] = off;
        off += align256(pj_packed_bytes(p[i].M, p[i].K, L, r, prec));
        bp.b_off[i] = off;
        off += align256(pj_packed_bytes(p[i].W, p[i].K, L, r, prec));
    }
    bp.total = off;
    return PJ_OK;
}

int device_cus()
{
    static int cached = 0;
    if (cached > 0) return cached;
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        n = 256;
    cached = n;
    return n;
}

}  // namespace

size_t pj_gemm_batched_workspace_bytes(int count, const pj_gemm_desc* problems, int L, int r, int prec,
                                       int tile_cfg)
{
    BatchPlan bp;
    if (plan_batch(count, problems, L, r, prec, tile_cfg, bp) != PJ_OK) return 0;
    return bp.total;
}

size_t pj_gemm_batched_tiles_workspace_bytes(int count, const pj_gemm_desc* problems, const unsigned char* small,
                                             int L, int r, int prec, int tile_cfg)
{
    BatchPlan bp;
    if (!small || plan_batch(count, problems, L, r, prec, tile_cfg, bp, small) != PJ_OK) return 0;
    return bp.total;
}

static int run_batched(pj_basis b, int r, int count, const pj_gemm_desc* problems, float beta, int prec,
                       int tile_cfg, const unsigned char* small, void* ws, size_t ws_bytes, void* stream);

int proj_gemm_batched(pj_basis b, int r, int count, const pj_gemm_desc* problems, float beta, int prec,
                      int tile_cfg, void* ws, size_t ws_bytes, void* stream)
{
    return run_batched(b, r, count, problems, beta, prec, tile_cfg, nullptr, ws, ws_bytes, stream);
}

int proj_gemm_batched_tiles(pj_basis b, int r, int count, const pj_gemm_desc* problems, const unsigned char* small,
                            float beta, int prec, int tile_cfg, void* ws, size_t ws_bytes, void* stream)
{
    if (!small) return PJ_ERR_ARG;
    return run_batched(b, r, count, problems, beta, prec, tile_cfg, small, ws, ws_bytes, stream);
}

static int run_batched(pj_basis b, int r, int count, const pj_gemm_desc* problems, float beta, int prec,
                       int tile_cfg, const unsigned char* small, void* ws, size_t ws_bytes, void* stream)
{
    if (!b) return PJ_ERR_ARG;
    BatchPlan bp;
    int rc = plan_batch(count, problems, b->L, r, prec, tile_cfg, bp, small);
    if (rc != PJ_OK) return rc;
    if (!ws || ws_bytes < bp.total) return PJ_ERR_WORKSPACE;
    if (!b->on_device) return PJ_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    char* w = (char*)ws;
    const Layout ly = layout_of(prec);
    std::vector<PackArgs> pa(2 * (size_t)count);
    std::vector<GroupedProblem> gp(count);
    int tm = 0, tn = 0, sm = 0, sn = 0;
    gemm_config_tile(prec, bp.cfg, &tm, &tn);
    gemm_config_small_tile(prec, bp.cfg, &sm, &sn);
    std::vector<GroupedItem> items;
    items.reserve(bp.nitems);
    for (int i = 0; i < count; ++i) {
        const pj_gemm_desc& d = problems[i];
        pa[2 * i] = pack_args(b, r, true, d.transA, d.M, d.K, d.A, d.lda, prec, w + bp.a_off[i]);
        pa[2 * i + 1] = pack_args(b, r, false, d.transB, d.W, d.K, d.B, d.ldb, prec, w + bp.b_off[i]);
        const PackGeom& ga = pa[2 * i].geom;
        const PackGeom& gb = pa[2 * i + 1].geom;
        GroupedProblem& g = gp[i];
        g.X = w + bp.a_off[i]; g.x_nrb = ga.nrb; g.x_nkb = ga.nkb;
        g.x_plane = ga.plane_bytes + ga.scale_plane; g.x_pb = ga.plane_bytes;
        g.Y = w + bp.b_off[i]; g.y_nrb = gb.nrb; g.y_nkb = gb.nkb;
        g.y_plane = gb.plane_bytes + gb.scale_plane; g.y_pb = gb.plane_bytes;
        g.nkb = (int64_t)r * ga.Gp / ly.KB;
        g.P = d.M; g.Q = d.W; g.R = d.R; g.ldr = d.ldr; g.beta = beta;
        const int body = bp.small[i];
        const int64_t ntm = cdiv(d.M, body ? sm : tm), ntn = cdiv(d.W, body ? sn : tn);
        for (int64_t y = 0; y < ntn; ++y)
            for (int64_t x = 0; x < ntm; ++x) items.push_back(GroupedItem{i, (int32_t)x, (int32_t)y, body});
    }
    // longest contractions first (stable: problem order, then tile order)
    std::stable_sort(items.begin(), items.end(), [&](const GroupedItem& u, const GroupedItem& v) {
        return gp[u.prob].nkb > gp[v.prob].nkb;
    });
    for (const PackArgs& x : pa)
        if (x.geom.nrb * (x.geom.Gp / ly.KB) > 0x3fffffff) return PJ_ERR_UNSUPPORTED;
    rc = launch_pack_grouped(prec, pa.data(), 2 * count, w, st);
    if (rc != 0) return rc == -2 ? PJ_ERR_UNSUPPORTED : PJ_ERR_HIP;
    if (hipMemcpyAsync(w + bp.probs_off, gp.data(), sizeof(GroupedProblem) * count, hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(w + bp.items_off, items.data(), sizeof(GroupedItem) * items.size(), hipMemcpyHostToDevice,
                       st) != hipSuccess)
        return PJ_ERR_HIP;
    rc = launch_gemm_grouped(prec, (const GroupedProblem*)(w + bp.probs_off), (const GroupedItem*)(w + bp.items_off),
                             bp.nitems, device_cus(), bp.cfg, st);
    return rc == 0 ? PJ_OK : (rc == -2 ? PJ_ERR_UNSUPPORTED : PJ_ERR_HIP);
}

// ---------------------------------------------------------------- backward

namespace {

struct BwdPlan {
    int64_t Gp, rg, T;
    size_t ahat, bhat, pk, dahat, dbhat, total;
    size_t p1, p2, p3, p4;
};

// Workspace of the backward for projections of Gp padded groups; with
// `proj` the plain projections of A and B are computed into it first (else
// the caller's saved ones are used).  Plain projections use the FP32 / FP64
// fragment geometry (k-blocks of 8).
BwdPlan plan_bwd(int M, int W, int K, int L, int r, int prec, int64_t Gp, bool proj)
{
    BwdPlan p;
    p.T = (prec == PJ_F64) ? 8 : 4;
    p.Gp = Gp;
    p.rg = (int64_t)r * p.Gp;
    p.p1 = align256(pj_packed_bytes(M, W, 4, 4, prec));
    p.p2 = align256(pj_packed_bytes((int)p.rg, W, 4, 4, prec));
    p.p3 = align256(pj_packed_bytes((int)p.rg, M, 4, 4, prec));
    p.p4 = align256(pj_packed_bytes(W, M, 4, 4, prec));
    size_t off = 0;
    p.ahat = p.bhat = 0;
    if (proj) {
        p.ahat = off; off += align256((size_t)M * p.rg * p.T);
        p.bhat = off; off += align256((size_t)W * p.rg * p.T);
    }
    p.pk = off; off += std::max(p.p1 + p.p2, p.p3 + p.p4);
    p.dahat = off; off += align256((size_t)M * p.rg * p.T);
    p.dbhat = off; off += align256((size_t)p.rg * W * p.T);
    p.total = off;
    return p;
}

int64_t bwd_plain_gp(int K, int L) { return rup(cdiv(K, L), 8); }

int check_bwd(pj_basis b, int r, char transA, char transB, int M, int W, int K, const void* dR, int64_t lddr,
              void* dA, int64_t ldda, void* dB, int64_t lddb, int prec)
{
    if (!b || !dR || (!dA && !dB)) return PJ_ERR_ARG;
    if (!valid_prec(prec)) return PJ_ERR_ARG;
    if (r < 1 || r > b->L) return PJ_ERR_ARG;
    if ((!is_n(transA) && !is_t(transA)) || (!is_n(transB) && !is_t(transB))) return PJ_ERR_ARG;
    if (M < 1 || W < 1 || K < 1) return PJ_ERR_SHAPE;
    if (lddr < W) return PJ_ERR_SHAPE;
    if (dA && ldda < (is_n(transA) ? (int64_t)K : (int64_t)M)) return PJ_ERR_SHAPE;
    if (dB && lddb < (is_n(transB) ? (int64_t)W : (int64_t)K)) return PJ_ERR_SHAPE;
    return PJ_OK;
}

// Steps 2-5 of the backward from the plain projections ahat (M x rG) and
// bhat (W x rG), row stride rG = r * pl.Gp.
int run_bwd(pj_basis b, int r, char transA, char transB, int M, int W, int K, const char* ahat, const char* bhat,
            const BwdPlan& pl, const void* dR, int64_t lddr, void* dA, int64_t ldda, void* dB, int64_t lddb,
            int prec, char* w, hipStream_t st)
{
    const bool f64 = (prec == PJ_F64);
    const void* I4 = f64 ? (const void*)b->I4d : (const void*)b->I4f;
    // packs an unprojected operand: rows x Kc of src (trans as given), the
    // contraction index kept as it is
    auto unproj = [&](const void* src, int64_t ld, int trans, int64_t rows, int64_t Kc, void* dst) {
        PackArgs u;
        u.X = src; u.ld = ld; u.trans = trans; u.P = rows; u.K = Kc; u.L = 4; u.r = 4;
        u.coef = I4; u.out = dst; u.geom = pack_geom(rows, Kc, 4, 4, prec);
        return u;
    };
    auto gemm = [&](const void* X, int64_t P, const void* Y, int64_t Q, int64_t Kc, void* R, int64_t ldr) {
        GemmArgs g;
        g.X = X; g.gx = pack_geom(P, Kc, 4, 4, prec);
        g.Y = Y; g.gy = pack_geom(Q, Kc, 4, 4, prec);
        g.nkb = 4 * g.gx.Gp / layout_of(prec).KB;
        g.P = P; g.Q = Q; g.R = R; g.ldr = ldr; g.beta = 0.0f;
        return launch_gemm(prec, g, -1, st);
    };
    // the unprojected operands are only re-laid out (natural contraction
    // order); FP8 keeps the packer's identity pass for its MX scales
    const bool fp8 = (prec == PJ_FP8 || prec == PJ_FP8X2);
    auto pack2 = [&](const PackArgs* u) { return fp8 ? launch_pack_n(prec, u, 2, st) : launch_repack_n(prec, u, 2, st); };
    char* p1 = w + pl.pk;
    if (dA) {
        // 2. dA_hat = dR B_hat: contraction over the W columns of R
        PackArgs u[2] = {unproj(dR, lddr, 0, M, W, p1), unproj(bhat, pl.rg, 1, pl.rg, W, p1 + pl.p1)};
        if (pack2(u) != 0) return PJ_ERR_HIP;
        if (gemm(p1, M, p1 + pl.p1, pl.rg, W, w + pl.dahat, pl.rg) != 0) return PJ_ERR_HIP;
        // 3. dA = dA_hat spread back over each group with C
        ExpandArgs e;
        e.in = w + pl.dahat; e.ldi = pl.rg; e.in_trans = 0;
        e.out = dA; e.ldo = ldda; e.out_trans = is_t(transA) ? 1 : 0;
        e.P = M; e.K = K; e.L = b->L; e.r = r; e.Gp = pl.Gp;
        e.coef = f64 ? (const void*)b->Cd : (const void*)b->Cf;
        if (launch_expand(f64, e, st) != 0) return PJ_ERR_HIP;
    }
    if (dB) {
        // 4. dB_hat = A_hat^T dR: contraction over the M rows of R
        PackArgs u[2] = {unproj(ahat, pl.rg, 1, pl.rg, M, p1), unproj(dR, lddr, 1, W, M, p1 + pl.p3)};
        if (pack2(u) != 0) return PJ_ERR_HIP;
        if (gemm(p1, pl.rg, p1 + pl.p3, W, M, w + pl.dbhat, W) != 0) return PJ_ERR_HIP;
        // 5. dB = dB_hat spread back over each group with D
        ExpandArgs e;
        e.in = w + pl.dbhat; e.ldi = W; e.in_trans = 1;
        e.out = dB; e.ldo = lddb; e.out_trans = is_n(transB) ? 1 : 0;
        e.P = W; e.K = K; e.L = b->L; e.r = r; e.Gp = pl.Gp;
        e.coef = f64 ? (const void*)b->DTd : (const void*)b->DTf;
        if (launch_expand(f64, e, st) != 0) return PJ_ERR_HIP;
    }
    return PJ_OK;
}

}  // namespace

size_t pj_gemm_backward_workspace_bytes(int M, int W, int K, int L, int r, int prec)
{
    if (M < 1 || W < 1 || K < 1 || L < 1 || L > kMaxL || r < 1 || r > L || !valid_prec(prec)) return 0;
    return plan_bwd(M, W, K, L, r, prec, bwd_plain_gp(K, L), true).total;
}

int proj_gemm_backward(pj_basis b, int r, char transA, char transB, int M, int W, int K, const void* A, int64_t lda,
                       const void* B, int64_t ldb, const void* dR, int64_t lddr, void* dA, int64_t ldda, void* dB,
                       int64_t lddb, int prec, void* ws, size_t ws_bytes, void* stream)
{
    if (!A || !B) return PJ_ERR_ARG;
    int rc = check_bwd(b, r, transA, transB, M, W, K, dR, lddr, dA, ldda, dB, lddb, prec);
    if (rc != PJ_OK) return rc;
    if (lda < (is_n(transA) ? (int64_t)K : (int64_t)M)) return PJ_ERR_SHAPE;
    if (ldb < (is_n(transB) ? (int64_t)W : (int64_t)K)) return PJ_ERR_SHAPE;
    const BwdPlan pl = plan_bwd(M, W, K, b->L, r, prec, bwd_plain_gp(K, b->L), true);
    if (pl.rg > 0x7fffffff) return PJ_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < pl.total) return PJ_ERR_WORKSPACE;
    if (!b->on_device) return PJ_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    char* w = (char*)ws;
    const int plain = (prec == PJ_F64) ? P_PLAIN64 : P_PLAIN32;

    // 1. plain projections of A (with C) and B (with D^T): M x rG and W x rG
    PackArgs pa[2] = {pack_args(b, r, true, transA, M, K, A, lda, plain, w + pl.ahat),
                      pack_args(b, r, false, transB, W, K, B, ldb, plain, w + pl.bhat)};
    pa[0].geom = pack_geom(M, K, b->L, r, plain);
    pa[1].geom = pack_geom(W, K, b->L, r, plain);
    pa[0].plain_ld = pa[1].plain_ld = pl.rg;
    if (launch_pack_n(plain, pa, 2, st) != 0) return PJ_ERR_HIP;
    return run_bwd(b, r, transA, transB, M, W, K, w + pl.ahat, w + pl.bhat, pl, dR, lddr, dA, ldda, dB, lddb, prec,
                   w, st);
}

size_t pj_gemm_backward_saved_workspace_bytes(int M, int W, int K, int L, int r, int prec)
{
    if (M < 1 || W < 1 || K < 1 || L < 1 || L > kMaxL || r < 1 || r > L || !valid_prec(prec)) return 0;
    return plan_bwd(M, W, K, L, r, prec, saved_geom(M, W, K, L, r, prec).Gp, false).total;
}

int proj_gemm_backward_saved(pj_basis b, int r, char transA, char transB, int M, int W, int K, const void* saved,
                             size_t saved_bytes, const void* dR, int64_t lddr, void* dA, int64_t ldda, void* dB,
                             int64_t lddb, int prec, void* ws, size_t ws_bytes, void* stream)
{
    if (!saved) return PJ_ERR_ARG;
    int rc = check_bwd(b, r, transA, transB, M, W, K, dR, lddr, dA, ldda, dB, lddb, prec);
    if (rc != PJ_OK) return rc;
    const SavedGeom sg = saved_geom(M, W, K, b->L, r, prec);
    if (saved_bytes < sg.total) return PJ_ERR_WORKSPACE;
    const BwdPlan pl = plan_bwd(M, W, K, b->L, r, prec, sg.Gp, false);
    if (pl.rg > 0x7fffffff) return PJ_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < pl.total) return PJ_ERR_WORKSPACE;
    if (!b->on_device) return PJ_ERR_HIP;
    const char* sv = (const char*)saved;
    return run_bwd(b, r, transA, transB, M, W, K, sv, sv + sg.bhat, pl, dR, lddr, dA, ldda, dB, lddb, prec,
                   (char*)ws, (hipStream_t)stream);
}

size_t pj_conv1d_method_workspace_bytes(int64_t W, int N, int L, int r, int method, int prec)
{
    if (W < 1 || N < 1 || N > W || L < 1 || L > kMaxL || r < 1 || r > L || !valid_prec(prec)) return 0;
    if (method < PJ_CONV_AUTO || method > PJ_CONV_FFT) return 0;
    if (method == PJ_CONV_FFT || (method == PJ_CONV_AUTO && conv_prefers_fft(W, N, L, r))) {
        const ConvFftGeom g = conv_fft_geom(W, N, L, r);
        return g.ok ? (size_t)g.total : 0;
    }
    return (size_t)conv_geom(W, N, L, r).total;
}

size_t pj_conv1d_workspace_bytes(int64_t W, int N, int L, int r, int prec)
{
    return pj_conv1d_method_workspace_bytes(W, N, L, r, PJ_CONV_AUTO, prec);
}

int proj_conv1d(pj_basis b, int r, int mode, int64_t W, const float* s, int N, const float* k, float* y,
                int prec, void* ws, size_t ws_bytes, void* stream)
{
    return proj_conv1d_method(b, r, mode, PJ_CONV_AUTO, W, s, N, k, y, prec, ws, ws_bytes, stream);
}

int proj_conv1d_method(pj_basis b, int r, int mode, int method, int64_t W, const float* s, int N, const float* k,
                       float* y, int prec, void* ws, size_t ws_bytes, void* stream)
{
    if (method < PJ_CONV_AUTO || method > PJ_CONV_FFT) return PJ_ERR_ARG;
    if (!b || !s || !k || !y) return PJ_ERR_ARG;
    if (r < 1 || r > b->L) return PJ_ERR_ARG;
    if (mode != PJ_XCORR && mode != PJ_CONV) return PJ_ERR_ARG;
    if (!valid_prec(prec)) return PJ_ERR_ARG;
    if (W < 1 || N < 1 || N > W) return PJ_ERR_SHAPE;
    if (prec != PJ_F32) return PJ_ERR_UNSUPPORTED;
    if (method == PJ_CONV_FFT || (method == PJ_CONV_AUTO && conv_prefers_fft(W, N, b->L, r)))
        return proj_conv1d_fft(b, r, mode, W, s, N, k, y, prec, ws, ws_bytes, stream);
    const ConvGeom g = conv_geom(W, N, b->L, r);
    if (g.tiles_m * g.tiles_n > 0x7fffffff || g.k_nrb * g.k_nkb * 64 / 256 > 0x7fffffff || cdiv(g.nout, 256) > 0x7fffffff ||
        cdiv(g.nbp, 64) > 0x7fffffff || g.ncp * b->L > 0x7fffffff)
        return PJ_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < (size_t)g.total) return PJ_ERR_WORKSPACE;
    if (!b->on_device) return PJ_ERR_HIP;
    ConvArgs a;
    a.s = s; a.W = W; a.k = k; a.N = N;
    a.reverse = (mode == PJ_CONV);
    a.L = b->L; a.r = r;
    a.C = b->Cf; a.DT = b->DTf; a.CT = b->CTf;
    a.y = y; a.ws = ws;
    return launch_conv(a, (hipStream_t)stream) == 0 ? PJ_OK : PJ_ERR_HIP;
}

size_t pj_conv1d_fft_workspace_bytes(int64_t W, int N, int L, int r, int prec)
{
    if (W < 1 || N < 1 || N > W || L < 1 || L > kMaxL || r < 1 || r > L || !valid_prec(prec)) return 0;
    const ConvFftGeom g = conv_fft_geom(W, N, L, r);
    return g.ok ? (size_t)g.total : 0;
}

int proj_conv1d_fft(pj_basis b, int r, int mode, int64_t W, const float* s, int N, const float* k, float* y,
                    int prec, void* ws, size_t ws_bytes, void* stream)
{
    if (!b || !s || !k || !y) return PJ_ERR_ARG;
    if (r < 1 || r > b->L) return PJ_ERR_ARG;
    if (mode != PJ_XCORR && mode != PJ_CONV) return PJ_ERR_ARG;
    if (!valid_prec(prec)) return PJ_ERR_ARG;
    if (W < 1 || N < 1 || N > W) return PJ_ERR_SHAPE;
    if (prec != PJ_F32) return PJ_ERR_UNSUPPORTED;
    const ConvFftGeom g = conv_fft_geom(W, N, b->L, r);
    if (!g.ok) return PJ_ERR_UNSUPPORTED;
    if ((int64_t)r * b->L > 0x7fffffff || (int64_t)r * g.nseg > 0x7fffffff || (int64_t)b->L * g.nseg > 0x7fffffff ||
        cdiv(g.nseg, 2) > 65535 || cdiv(g.nbp, 32) > 0x7fffffff)
        return PJ_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < (size_t)g.total) return PJ_ERR_WORKSPACE;
    if (!b->on_device) return PJ_ERR_HIP;
    ConvArgs a;
    a.s = s; a.W = W; a.k = k; a.N = N;
    a.reverse = (mode == PJ_CONV);
    a.L = b->L; a.r = r;
    a.C = b->Cf; a.DT = b->DTf; a.CT = b->CTf;
    a.y = y; a.ws = ws;
    return launch_conv_fft(a, (hipStream_t)stream) == 0 ? PJ_OK : PJ_ERR_HIP;
}

size_t pj_conv1d_circular_workspace_bytes(int64_t W, int N, int L, int r, int prec)
{
    if (W < 1 || N < 1 || N > W || L < 1 || L > kMaxL || r < 1 || r > L || !valid_prec(prec) || W % L != 0) return 0;
    return (size_t)conv_geom(W + N - 1, N, L, r).total;
}

int proj_conv1d_circular(pj_basis b, int r, int mode, int64_t W, const float* s, int N, const float* k, float* y,
                         int prec, void* ws, size_t ws_bytes, void* stream)
{
    if (!b || !s || !k || !y) return PJ_ERR_ARG;
    if (r < 1 || r > b->L) return PJ_ERR_ARG;
    if (mode != PJ_XCORR && mode != PJ_CONV) return PJ_ERR_ARG;
    if (!valid_prec(prec)) return PJ_ERR_ARG;
    if (W < 1 || N < 1 || N > W || W % b->L != 0) return PJ_ERR_SHAPE;
    if (prec != PJ_F32) return PJ_ERR_UNSUPPORTED;
    const int64_t Wv = W + N - 1;
    const ConvGeom g = conv_geom(Wv, N, b->L, r);
    if (g.tiles_m * g.tiles_n > 0x7fffffff || g.k_nrb * g.k_nkb * 64 / 256 > 0x7fffffff || cdiv(g.nout, 256) > 0x7fffffff ||
        cdiv(g.nbp, 64) > 0x7fffffff || g.ncp * b->L > 0x7fffffff || cdiv((int64_t)r * g.nbp, 256) > 0x7fffffff)
        return PJ_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < (size_t)g.total) return PJ_ERR_WORKSPACE;
    if (!b->on_device) return PJ_ERR_HIP;
    ConvArgs a;
    a.s = s; a.W = Wv; a.k = k; a.N = N;
    a.reverse = (mode == PJ_CONV);
    a.L = b->L; a.r = r;
    a.C = b->Cf; a.DT = b->DTf; a.CT = b->CTf;
    a.y = y; a.ws = ws;
    a.period = W;
    return launch_conv(a, (hipStream_t)stream) == 0 ? PJ_OK : PJ_ERR_HIP;
}

size_t pj_conv1d_rate_workspace_bytes(int64_t W, int N, int L, int r, int rate, int prec)
{
    if (rate == PJ_RATE_FULL) return pj_conv1d_workspace_bytes(W, N, L, r, prec);
    if (rate != PJ_RATE_BLOCK) return 0;
    if (W < 1 || N < 1 || N > W || L < 1 || L > kMaxL || r < 1 || r > L || !valid_prec(prec)) return 0;
    return (size_t)conv_block_geom(W, N, L, r).total;
}

int proj_conv1d_rate(pj_basis b, int r, int mode, int rate, int64_t W, const float* s, int N, const float* k,
                     float* y, int prec, void* ws, size_t ws_bytes, void* stream)
{
    if (rate == PJ_RATE_FULL) return proj_conv1d(b, r, mode, W, s, N, k, y, prec, ws, ws_bytes, stream);
    if (rate != PJ_RATE_BLOCK) return PJ_ERR_ARG;
    if (!b || !s || !k || !y) return PJ_ERR_ARG;
    if (r < 1 || r > b->L) return PJ_ERR_ARG;
    if (mode != PJ_XCORR && mode != PJ_CONV) return PJ_ERR_ARG;
    if (!valid_prec(prec)) return PJ_ERR_ARG;
    if (W < 1 || N < 1 || N > W) return PJ_ERR_SHAPE;
    if (prec != PJ_F32) return PJ_ERR_UNSUPPORTED;
    const ConvBlockGeom g = conv_block_geom(W, N, b->L, r);
    if (cdiv(g.nbp, 32) > 0x7fffffff || cdiv((int64_t)g.nch * g.ntp, 256) > 0x7fffffff ||
        cdiv(g.nout, 256) > 0x7fffffff || g.ntp > 0x7fffffff)
        return PJ_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < (size_t)g.total) return PJ_ERR_WORKSPACE;
    if (!b->on_device) return PJ_ERR_HIP;
    ConvArgs a;
    a.s = s; a.W = W; a.k = k; a.N = N;
    a.reverse = (mode == PJ_CONV);
    a.L = b->L; a.r = r;
    a.C = b->Cf; a.DT = b->DTf; a.CT = b->CTf;
    a.y = y; a.ws = ws;
    return launch_conv_block(a, (hipStream_t)stream) == 0 ? PJ_OK : PJ_ERR_HIP;
}

int pj_basis_create_klt(pj_basis* out, int L, const double* M, double* eig_out)
{
    if (!out) return PJ_ERR_ARG;
    *out = nullptr;
    if (L < 1 || L > kMaxL || !M) return PJ_ERR_ARG;
    const size_t n = (size_t)L * L;
    double big = 0.0;
    for (size_t i = 0; i < n; ++i) {
        if (!std::isfinite(M[i])) return PJ_ERR_ARG;
        big = std::max(big, std::fabs(M[i]));
    }
    for (int t = 0; t < L; ++t)
        for (int u = t + 1; u < L; ++u)
            if (std::fabs(M[(size_t)t * L + u] - M[(size_t)u * L + t]) > 1e-12 * big) return PJ_ERR_ARG;
    std::vector<double> A(M, M + n), V;
    jacobi_eig(L, A, V);
    std::vector<int> order(L);
    for (int i = 0; i < L; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return A[(size_t)x * L + x] > A[(size_t)y * L + y]; });
    pj_basis b = new (std::nothrow) pj_basis_s;
    if (!b) return PJ_ERR_ARG;
    b->kind = PJ_BASIS_CUSTOM;
    b->L = L;
    b->C.assign(n, 0.0);
    b->D.assign(n, 0.0);
    for (int l = 0; l < L; ++l) {
        const int src = order[l];
        int imax = 0;
        for (int t = 1; t < L; ++t)
            if (std::fabs(V[(size_t)t * L + src]) > std::fabs(V[(size_t)imax * L + src])) imax = t;
        const double sg = V[(size_t)imax * L + src] < 0.0 ? -1.0 : 1.0;
        for (int t = 0; t < L; ++t) b->C[(size_t)t * L + l] = sg * V[(size_t)t * L + src];
        if (eig_out) eig_out[l] = A[(size_t)src * L + src];
    }
    for (int t = 0; t < L; ++t)          // orthonormal: D = C^T
        for (int l = 0; l < L; ++l) b->D[(size_t)l * L + t] = b->C[(size_t)t * L + l];
    upload(b);
    *out = b;
    return PJ_OK;
}

size_t pj_block_moments_workspace_bytes(int64_t rows, int64_t K, int L)
{
    if (rows < 1 || K < 1 || L < 1 || L > kMaxL) return 0;
    return (size_t)std::max<int64_t>(moments_geom(rows, K, L).ws_bytes, 256);
}

int pj_block_moments(int L, int64_t rows, int64_t K, const float* X, int64_t ld, double* M, void* ws,
                     size_t ws_bytes, void* stream)
{
    if (!X || !M) return PJ_ERR_ARG;
    if (L < 1 || L > kMaxL) return PJ_ERR_ARG;
    if (rows < 1 || K < 1 || ld < K) return PJ_ERR_SHAPE;
    const MomentsGeom g = moments_geom(rows, K, L);
    if (g.chunk > 0x7fffffff || g.nchunk > 65535) return PJ_ERR_UNSUPPORTED;
    if (g.ws_bytes > 0 && (!ws || ws_bytes < (size_t)g.ws_bytes)) return PJ_ERR_WORKSPACE;
    if (!device_present()) return PJ_ERR_HIP;
    return launch_moments(X, ld, rows, K, L, M, ws, (hipStream_t)stream) == 0 ? PJ_OK : PJ_ERR_HIP;
}

int pj_images_center(int J, int64_t mn, const float* X, float* mean, float* out, void* stream)
{
    if (!X || !mean || !out) return PJ_ERR_ARG;
    if (J < 1 || mn < 1) return PJ_ERR_SHAPE;
    if (!device_present()) return PJ_ERR_HIP;
    const int rc = launch_center(J, mn, X, mean, out, false, (hipStream_t)stream);
    return rc == 0 ? PJ_OK : (rc == -2 ? PJ_ERR_UNSUPPORTED : PJ_ERR_HIP);
}

int pj_images_subtract(int T, int64_t mn, const float* X, const float* mean, float* out, void* stream)
{
    if (!X || !mean || !out) return PJ_ERR_ARG;
    if (T < 1 || mn < 1) return PJ_ERR_SHAPE;
    if (!device_present()) return PJ_ERR_HIP;
    const int rc = launch_center(T, mn, X, const_cast<float*>(mean), out, true, (hipStream_t)stream);
    return rc == 0 ? PJ_OK : (rc == -2 ? PJ_ERR_UNSUPPORTED : PJ_ERR_HIP);
}

int pj_symmetrize(int n, float* G, int64_t ld, void* stream)
{
    if (!G) return PJ_ERR_ARG;
    if (n < 1 || n > 65535 * 16 || ld < n) return PJ_ERR_SHAPE;
    if (!device_present()) return PJ_ERR_HIP;
    return launch_symmetrize(n, G, ld, (hipStream_t)stream) == 0 ? PJ_OK : PJ_ERR_HIP;
}

int pj_sq_distances(int T, int J, int64_t d, const float* F, int64_t ldf, const float* Y, int64_t ldy, float* out,
                    int64_t ldo, void* stream)
{
    if (!F || !Y || !out) return PJ_ERR_ARG;
    if (T < 1 || J < 1 || d < 1 || ldf < d || ldy < d || ldo < J) return PJ_ERR_SHAPE;
    if (!device_present()) return PJ_ERR_HIP;
    const int rc = launch_sqdist(T, J, d, F, ldf, Y, ldy, out, ldo, (hipStream_t)stream);
    return rc == 0 ? PJ_OK : (rc == -2 ? PJ_ERR_UNSUPPORTED : PJ_ERR_HIP);
}

int pj_sym_eig(int n, const double* A, double* w, double* V)
{
    if (n < 1 || n > 4096 || !A || !w || !V) return PJ_ERR_ARG;
    const size_t nn = (size_t)n * n;
    double big = 0.0;
    for (size_t i = 0; i < nn; ++i) {
        if (!std::isfinite(A[i])) return PJ_ERR_ARG;
        big = std::max(big, std::fabs(A[i]));
    }
    for (int t = 0; t < n; ++t)
        for (int u = t + 1; u < n; ++u)
            if (std::fabs(A[(size_t)t * n + u] - A[(size_t)u * n + t]) > 1e-12 * big) return PJ_ERR_ARG;
    std::vector<double> a(A, A + nn), v;
    jacobi_eig(n, a, v);
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return a[(size_t)x * n + x] > a[(size_t)y * n + y]; });
    for (int l = 0; l < n; ++l) {
        const int src = order[l];
        int imax = 0;
        for (int t = 1; t < n; ++t)
            if (std::fabs(v[(size_t)t * n + src]) > std::fabs(v[(size_t)imax * n + src])) imax = t;
        const double sg = v[(size_t)imax * n + src] < 0.0 ? -1.0 : 1.0;
        for (int t = 0; t < n; ++t) V[(size_t)t * n + l] = sg * v[(size_t)t * n + src];
        w[l] = a[(size_t)src * n + src];
    }
    return PJ_OK;
}

}  // extern "C"
