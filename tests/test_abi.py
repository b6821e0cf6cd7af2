"""CPU tests of the C ABI: the library loads, exports every function that
include/projgemm.h declares, rejects invalid calls with the documented status
before touching a device, and builds its FP64 bases correctly on the host.
No compute call is made here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1411_2860_amd import projgemm as pg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "projgemm.h")

OK, ARG, SHAPE, UNSUP, WS, SING, HIP, SCRATCH = 0, -1, -2, -3, -4, -5, -6, -7
FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(p[jr]\w*)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pg.lib_path()):
        pytest.fail("libprojgemm.so is not built (python -m paper_1411_2860_amd.build)")
    return pg.lib()


@pytest.fixture(scope="module")
def basis16(lib):
    return pg.Basis("dct2", 16)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 10
    raw = ctypes.CDLL(pg.lib_path())
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, missing
    for n in names:
        assert n in pg._SIGNATURES, f"binding lacks {n}"


def test_tile_configs(lib):
    cfgs = pg.tile_configs("f32")
    assert len(cfgs) == 19 and (128, 128) in cfgs
    assert all(m % 32 == 0 and n % 32 == 0 for m, n in cfgs)
    assert all(m % 16 == 0 for m, _ in pg.tile_configs("f64"))


def test_status_strings(lib):
    for c in (OK, ARG, SHAPE, UNSUP, WS, SING, HIP, SCRATCH):
        assert pg.status_str(c) and pg.status_str(c) != "unknown status"


# ------------------------------------------------------------------ basis

@pytest.mark.parametrize("kind,L", [("dct2", 1), ("dct2", 16), ("dct2", 64), ("dct2", 256), ("haar", 2),
                                    ("haar", 8), ("haar", 256), ("identity", 5)])
def test_basis_inverse_orthonormal_and_same_projector_as_oracle(kind, L):
    b = pg.Basis(kind, L)
    C, D = b.matrices()
    np.testing.assert_allclose(D @ C, np.eye(L), atol=1e-12)
    np.testing.assert_allclose(C.T @ C, np.eye(L), atol=1e-12)
    Co, Do = oracle.basis(kind, L)
    for r in sorted({1, 2, max(1, L // 2), L}):
        # column scaling does not change Q_r, and both orderings agree
        np.testing.assert_allclose(C[:, :r] @ D[:r, :], Co[:, :r] @ Do[:r, :], atol=1e-12)
    assert pg.lib().pj_basis_L(b.handle) == L


def test_custom_basis_and_singular(lib):
    C = np.random.default_rng(0).standard_normal((6, 6)) + 3 * np.eye(6)
    b = pg.Basis("custom", 6, C)
    Cb, Db = b.matrices()
    np.testing.assert_array_equal(Cb, C)
    np.testing.assert_allclose(Db @ C, np.eye(6), atol=1e-12)
    S = C.copy()
    S[:, 2] = S[:, 0]
    h = ctypes.c_void_p()
    arr = np.ascontiguousarray(S)
    assert lib.pj_basis_create(ctypes.byref(h), 3, 6, arr.ctypes.data_as(pg._dp)) == SING


def test_basis_argument_errors(lib):
    h = ctypes.c_void_p()
    assert lib.pj_basis_create(None, 0, 8, None) == ARG
    assert lib.pj_basis_create(ctypes.byref(h), 0, 0, None) == ARG
    assert lib.pj_basis_create(ctypes.byref(h), 0, 257, None) == ARG
    assert lib.pj_basis_create(ctypes.byref(h), 1, 6, None) == ARG        # Haar needs a power of two
    assert lib.pj_basis_create(ctypes.byref(h), 3, 4, None) == ARG        # custom needs C
    assert lib.pj_basis_create(ctypes.byref(h), 9, 4, None) == ARG
    assert lib.pj_basis_get(None, None, None) == ARG
    assert lib.pj_basis_destroy(None) == ARG


# ------------------------------------------------------------ sizes

def test_packed_bytes_and_workspace(lib):
    # f32: tiles of 32 rows x 8 indices, 1 KiB each; K = 4096, L = 64 -> G = 64
    assert pg.packed_bytes(1024, 4096, 64, 16, "f32") == (1024 // 32) * (16 * 64 // 8) * 1024
    # ragged: rows padded to 32, groups padded to a multiple of 8
    assert pg.packed_bytes(33, 100, 16, 3, "f32") == 2 * (3 * 8 // 8) * 1024
    # split modes store two planes
    assert pg.packed_bytes(64, 256, 16, 4, "bf16x3") == 2 * pg.packed_bytes(64, 256, 16, 4, "bf16")
    assert pg.packed_bytes(0, 10, 4, 1) == 0 and pg.packed_bytes(4, 10, 4, 5) == 0
    # fp8: 2 KiB tiles of 32 rows x 64 indices plus 64 scale bytes per tile
    assert pg.packed_bytes(32, 64 * 16, 16, 2, "fp8") == 2 * (2048 + 64)
    assert pg.packed_bytes(32, 64 * 16, 16, 2, "fp8x2") == 2 * pg.packed_bytes(32, 64 * 16, 16, 2, "fp8")
    ws = pg.gemm_workspace_bytes(100, 200, 300, 16, 4, "f32")
    assert ws >= pg.packed_bytes(100, 300, 16, 4) + pg.packed_bytes(200, 300, 16, 4)
    assert pg.gemm_workspace_bytes(100, 200, 300, 16, 17, "f32") == 0


# ------------------------------------------------------- proj_gemm errors

def _gemm(lib, b, r=4, ta=b"N", tb=b"N", M=8, W=8, K=32, lda=32, ldb=8, ldr=8, prec=1, ws_bytes=1 << 30,
          A=FAKE, B=FAKE, R=FAKE, ws=FAKE):
    return lib.proj_gemm(b.handle if b is not None else None, r, ta, tb, M, W, K, A, lda, B, ldb, 0.0, R, ldr,
                         prec, ws, ws_bytes, None)


def test_proj_gemm_validation(lib, basis16):
    b = basis16
    assert _gemm(lib, None) == ARG
    assert _gemm(lib, b, A=None) == ARG
    assert _gemm(lib, b, R=None) == ARG
    assert _gemm(lib, b, r=0) == ARG
    assert _gemm(lib, b, r=17) == ARG
    assert _gemm(lib, b, ta=b"X") == ARG
    assert _gemm(lib, b, prec=8) == ARG
    assert _gemm(lib, b, M=0) == SHAPE
    assert _gemm(lib, b, K=-1) == SHAPE
    assert _gemm(lib, b, lda=31) == SHAPE
    assert _gemm(lib, b, ta=b"T", lda=7) == SHAPE          # A stored K x M needs lda >= M
    assert _gemm(lib, b, ldb=7) == SHAPE
    assert _gemm(lib, b, tb=b"T", ldb=31) == SHAPE         # B stored W x K needs ldb >= K
    assert _gemm(lib, b, ldr=7) == SHAPE
    assert _gemm(lib, b, prec=6, r=9) == UNSUP             # FP8 only for r <= 8
    assert _gemm(lib, b, ws_bytes=16) == WS
    assert _gemm(lib, b, ws=None) == WS


def test_valid_call_without_device_reports_hip(lib, basis16):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    assert _gemm(lib, basis16) == HIP


def test_saved_forward_backward_validation(lib, basis16):
    """proj_gemm_save / proj_gemm_backward_saved: the kept projections' size
    (A_hat then B_hat, 256-byte aligned, Gp rounded to the k-block) and the
    argument errors, before any device work."""
    b = basis16
    # f32: K = 150, L = 16 -> G = 10, Gp = 16 (k-blocks of 8); bf16 the same (16)
    a256 = lambda n: -(-n // 256) * 256
    assert pg.gemm_saved_bytes(45, 33, 150, 16, 5, "f32") == a256(45 * 5 * 16 * 4) + a256(33 * 5 * 16 * 4)
    assert pg.gemm_saved_bytes(45, 33, 150, 16, 5, "f64") == a256(45 * 5 * 16 * 8) + a256(33 * 5 * 16 * 8)
    # 16-bit formats round the groups to 16, FP8 to 64
    assert pg.gemm_saved_bytes(45, 33, 150, 16, 5, "bf16") == a256(45 * 5 * 16 * 4) + a256(33 * 5 * 16 * 4)
    assert pg.gemm_saved_bytes(45, 33, 400, 16, 5, "bf16") == a256(45 * 5 * 32 * 4) + a256(33 * 5 * 32 * 4)
    assert pg.gemm_saved_bytes(45, 33, 400, 16, 5, "fp8") == a256(45 * 5 * 64 * 4) + a256(33 * 5 * 64 * 4)
    assert pg.gemm_saved_bytes(45, 33, 150, 16, 17, "f32") == 0
    sv = pg.gemm_saved_bytes(8, 8, 32, 16, 4, "f32")

    def save(r=4, saved=FAKE, saved_bytes=sv, lda=32, ws_bytes=1 << 30):
        return lib.proj_gemm_save(b.handle, r, b"N", b"N", 8, 8, 32, FAKE, lda, FAKE, 8, 0.0, FAKE, 8, 1, FAKE,
                                  ws_bytes, saved, saved_bytes, None)

    assert save(r=17) == ARG
    assert save(saved=None) == ARG
    assert save(lda=31) == SHAPE
    assert save(saved_bytes=sv - 1) == WS
    assert save(ws_bytes=16) == WS
    wb = lib.pj_gemm_backward_saved_workspace_bytes(8, 8, 32, 16, 4, 1)
    assert wb > 0

    def bwd(r=4, saved=FAKE, saved_bytes=sv, dA=FAKE, dB=FAKE, lddr=8, ws_bytes=wb):
        return lib.proj_gemm_backward_saved(b.handle, r, b"N", b"N", 8, 8, 32, saved, saved_bytes, FAKE, lddr,
                                            dA, 32, dB, 8, 1, FAKE, ws_bytes, None)

    assert bwd(saved=None) == ARG
    assert bwd(dA=None, dB=None) == ARG
    assert bwd(r=0) == ARG
    assert bwd(lddr=7) == SHAPE
    assert bwd(saved_bytes=sv - 1) == WS
    assert bwd(ws_bytes=wb - 1) == WS
    import torch
    if not torch.cuda.is_available():
        assert save() == HIP and bwd() == HIP


def test_batched_tiles_workspace(lib):
    """Per-problem tiles: more items (and workspace) with the small tile, the
    library's own choice between the two, NULL flags rejected."""
    import ctypes as ct
    descs = (pg.GemmDesc * 2)(pg.GemmDesc(300, 150, 64, b"N", b"N", FAKE, 64, FAKE, 150, FAKE, 150),
                              pg.GemmDesc(1024, 1024, 64, b"N", b"N", FAKE, 64, FAKE, 1024, FAKE, 1024))
    big = (ct.c_ubyte * 2)(0, 0)
    small = (ct.c_ubyte * 2)(1, 1)
    wb = lib.pj_gemm_batched_tiles_workspace_bytes(2, ct.cast(descs, ct.c_void_p), ct.cast(big, ct.c_void_p), 16, 4,
                                                   1, 0)
    ws = lib.pj_gemm_batched_tiles_workspace_bytes(2, ct.cast(descs, ct.c_void_p), ct.cast(small, ct.c_void_p), 16,
                                                   4, 1, 0)
    wa = lib.pj_gemm_batched_workspace_bytes(2, ct.cast(descs, ct.c_void_p), 16, 4, 1, 0)
    assert 0 < wb < ws and wb <= wa <= ws
    assert lib.pj_gemm_batched_tiles_workspace_bytes(2, ct.cast(descs, ct.c_void_p), None, 16, 4, 1, 0) == 0
    assert lib.proj_gemm_batched_tiles(None, 4, 2, ct.cast(descs, ct.c_void_p), ct.cast(big, ct.c_void_p), 0.0, 1, 0,
                                       FAKE, ws, None) == ARG


def test_pca2d_support_validation(lib):
    """Centring, symmetrisation and distance entry points reject bad
    arguments before any device work; valid calls need a device."""
    assert lib.pj_images_center(3, 16, None, FAKE, FAKE, None) == ARG
    assert lib.pj_images_center(0, 16, FAKE, FAKE, FAKE, None) == SHAPE
    assert lib.pj_images_subtract(2, 16, FAKE, None, FAKE, None) == ARG
    assert lib.pj_images_subtract(2, 0, FAKE, FAKE, FAKE, None) == SHAPE
    assert lib.pj_symmetrize(4, None, 4, None) == ARG
    assert lib.pj_symmetrize(4, FAKE, 3, None) == SHAPE
    assert lib.pj_sq_distances(2, 3, 10, FAKE, 10, None, 10, FAKE, 3, None) == ARG
    assert lib.pj_sq_distances(2, 3, 10, FAKE, 9, FAKE, 10, FAKE, 3, None) == SHAPE
    assert lib.pj_sq_distances(2, 3, 10, FAKE, 10, FAKE, 10, FAKE, 2, None) == SHAPE
    import torch
    if not torch.cuda.is_available():
        assert lib.pj_images_center(3, 16, FAKE, FAKE, FAKE, None) == HIP
        assert lib.pj_sq_distances(2, 3, 10, FAKE, 10, FAKE, 10, FAKE, 3, None) == HIP


def test_noalloc_validation_and_scratch_limit(lib, basis16):
    """proj_gemm_noalloc rejects what proj_gemm rejects, and a request whose
    workspace exceeds the fixed scratch, before any device work."""
    b = basis16

    def call(M=32, W=32, K=64, r=4, prec=1, A=FAKE, lda=None):
        return lib.proj_gemm_noalloc(b.handle, r, b"N", b"N", M, W, K, A, lda or K, FAKE, W, 0.0, FAKE, W,
                                     prec, None)
    assert call(A=None) == ARG
    assert call(r=0) == ARG
    assert call(M=0) == SHAPE
    assert call(lda=3) == SHAPE
    assert call(prec=6, r=9) == UNSUP
    M, W, K, r = 8192, 8192, 4096, 16
    assert pg.gemm_workspace_bytes(M, W, K, 16, r) > pg.NOALLOC_SCRATCH_BYTES
    assert call(M=M, W=W, K=K, r=r) == SCRATCH
    assert pg.NOALLOC_SCRATCH_BYTES == 64 << 20
    text = open(HEADER).read()
    assert "#define PJ_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)" in text


def test_conv_picks_fft_for_long_kernels(lib):
    """proj_conv1d takes the frequency-domain path when its cost model says so
    (its workspace query then returns the FFT path's size): long kernels at
    small L, not short kernels or L = 256 with a few projections."""
    W = 1 << 22
    fft = lambda N, L, r: lib.pj_conv1d_fft_workspace_bytes(W, N, L, r, 1)
    conv = lambda N, L, r: lib.pj_conv1d_workspace_bytes(W, N, L, r, 1)
    assert conv(16384, 16, 16) == fft(16384, 16, 16) > 0
    assert conv(8192, 8, 8) == fft(8192, 8, 8) > 0
    for N, L, r in [(16384, 256, 16), (1024, 256, 1), (600, 2, 1), (64, 4, 4)]:
        assert conv(N, L, r) != fft(N, L, r)
    assert fft(8192, 2, 1) == 0                   # 4097 taps per phase: beyond the transform


def test_pack_and_packed_gemm_validation(lib, basis16):
    b = basis16
    n = pg.packed_bytes(8, 32, 16, 4)
    assert lib.pj_pack_a(b.handle, 0, b"N", 8, 32, FAKE, 32, 1, FAKE, n, None) == ARG
    assert lib.pj_pack_a(b.handle, 4, b"N", 8, 32, FAKE, 31, 1, FAKE, n, None) == SHAPE
    assert lib.pj_pack_a(b.handle, 4, b"N", 8, 32, FAKE, 32, 1, FAKE, n - 1, None) == WS
    assert lib.pj_pack_b(b.handle, 4, b"N", 8, 32, FAKE, 7, 1, FAKE, n, None) == SHAPE
    assert lib.pj_pack_b(b.handle, 4, b"T", 8, 32, FAKE, 31, 1, FAKE, n, None) == SHAPE
    assert lib.pj_pack_b(b.handle, 4, b"Q", 8, 32, FAKE, 32, 1, FAKE, n, None) == ARG
    assert lib.pj_gemm_packed(5, 8, 8, 32, 16, 1, FAKE, 4, n, FAKE, 8, n, 0.0, FAKE, 8, -1, None) == ARG
    assert lib.pj_gemm_packed(4, 8, 8, 32, 16, 1, FAKE, 4, n, FAKE, 4, n, 0.0, FAKE, 7, -1, None) == SHAPE
    assert lib.pj_gemm_packed(4, 8, 8, 32, 16, 1, None, 4, n, FAKE, 4, n, 0.0, FAKE, 8, -1, None) == ARG
    assert lib.pj_gemm_packed(4, 8, 8, 32, 16, 1, FAKE, 4, n - 1, FAKE, 4, n, 0.0, FAKE, 8, -1, None) == WS
    assert lib.pj_gemm_packed(4, 8, 8, 32, 16, 1, FAKE, 4, n, FAKE, 8, n, 0.0, FAKE, 8, -1, None) == WS
    assert lib.pj_gemm_packed(4, 8, 8, 32, 16, 1, FAKE, 4, n, FAKE, 4, n, 0.0, FAKE, 8, 99, None) == ARG
    assert lib.pj_pack_ab(b.handle, 4, b"N", b"X", 8, 8, 32, FAKE, 32, FAKE, 32, 1, FAKE, n, FAKE, n, None) == ARG
    assert lib.pj_pack_ab(b.handle, 4, b"N", b"T", 8, 8, 32, FAKE, 32, FAKE, 32, 1, FAKE, n, FAKE, n - 1, None) == WS


def test_batched_validation(lib, basis16):
    import ctypes as ct
    b = basis16
    D = pg.GemmDesc
    good = D(8, 8, 32, b"N", b"N", 0x1000, 32, 0x1000, 8, 0x1000, 8)
    arr = (D * 2)(good, good)
    n = pg.gemm_batched_workspace_bytes(arr, 16, 4, "f32")
    assert n > 0
    p = ct.cast(arr, ct.c_void_p)
    assert lib.proj_gemm_batched(b.handle, 4, 2, p, 0.0, 1, -1, FAKE, n - 1, None) == WS
    assert lib.proj_gemm_batched(b.handle, 17, 2, p, 0.0, 1, -1, FAKE, n, None) == ARG
    assert lib.proj_gemm_batched(b.handle, 4, 0, p, 0.0, 1, -1, FAKE, n, None) == ARG
    assert lib.proj_gemm_batched(b.handle, 4, 2, p, 0.0, 1, 99, FAKE, n, None) == ARG
    assert lib.proj_gemm_batched(b.handle, 9, 2, p, 0.0, 6, -1, FAKE, n, None) == UNSUP
    bad = (D * 2)(good, D(8, 8, 32, b"N", b"N", 0x1000, 31, 0x1000, 8, 0x1000, 8))
    assert lib.proj_gemm_batched(b.handle, 4, 2, ct.cast(bad, ct.c_void_p), 0.0, 1, -1, FAKE, n, None) == SHAPE
    nul = (D * 2)(good, D(8, 8, 32, b"N", b"N", 0, 32, 0x1000, 8, 0x1000, 8))
    assert lib.proj_gemm_batched(b.handle, 4, 2, ct.cast(nul, ct.c_void_p), 0.0, 1, -1, FAKE, n, None) == ARG
    # the workspace grows with the batch
    assert pg.gemm_batched_workspace_bytes((D * 3)(good, good, good), 16, 4, "f32") > n


def test_conv_validation(lib, basis16):
    """proj_conv1d and proj_conv1d_rate: every argument error is reported
    before any device work; a valid call without a device reports PJ_ERR_HIP."""
    b = basis16
    W, N = 1000, 37
    full = lib.pj_conv1d_workspace_bytes(W, N, 16, 4, 1)
    blk = lib.pj_conv1d_rate_workspace_bytes(W, N, 16, 4, 1, 1)
    assert full > 0 and blk > 0
    assert lib.pj_conv1d_rate_workspace_bytes(W, N, 16, 4, 0, 1) == full
    assert lib.pj_conv1d_rate_workspace_bytes(W, N, 16, 4, 2, 1) == 0          # unknown rate
    assert lib.pj_conv1d_rate_workspace_bytes(W, W + 1, 16, 4, 1, 1) == 0      # N > W
    assert lib.pj_conv1d_rate_workspace_bytes(W, N, 16, 17, 1, 1) == 0         # r > L

    def call(rate, r=4, mode=0, Wc=W, Nc=N, s=FAKE, k=FAKE, y=FAKE, prec=1, ws_bytes=None, h=b.handle):
        n = (full if rate == 0 else blk) if ws_bytes is None else ws_bytes
        return lib.proj_conv1d_rate(h, r, mode, rate, Wc, s, Nc, k, y, prec, FAKE, n, None)

    for rate in (0, 1):
        assert call(rate, h=None) == ARG
        assert call(rate, r=0) == ARG
        assert call(rate, r=17) == ARG
        assert call(rate, mode=2) == ARG
        assert call(rate, s=None) == ARG
        assert call(rate, y=None) == ARG
        assert call(rate, prec=42) == ARG
        assert call(rate, Nc=0) == SHAPE
        assert call(rate, Nc=W + 1) == SHAPE
        assert call(rate, Wc=0, Nc=1) == SHAPE
        assert call(rate, prec=2) == UNSUP
        assert call(rate, ws_bytes=(full if rate == 0 else blk) - 1) == WS
        assert call(rate) == HIP
    assert call(5) == ARG
    assert lib.proj_conv1d(b.handle, 4, 0, W, FAKE, N, FAKE, FAKE, 1, FAKE, full - 1, None) == WS
    assert lib.proj_conv1d(b.handle, 4, 0, W, FAKE, N, FAKE, FAKE, 1, FAKE, full, None) == HIP


@pytest.mark.parametrize("L", [1, 4, 8, 64])
def test_klt_basis_matches_oracle(lib, L):
    """pj_basis_create_klt (host Jacobi) against the oracle's eigenbasis: same
    eigenvalues, orthonormal C with D = C^T, and the same projector Q_r at
    every r past which the eigenvalues are separated."""
    X = np.random.default_rng(L).standard_normal((40, 6 * L)) @ np.diag(np.linspace(1, 3, 6 * L))
    M = oracle.block_moments(X, L)
    b, eig = pg.klt_basis(M)
    C, D = b.matrices()
    Co, Do, wo = oracle.basis_klt(M)
    np.testing.assert_allclose(eig, wo, rtol=1e-10, atol=1e-10 * wo[0])
    np.testing.assert_allclose(C.T @ C, np.eye(L), atol=1e-12)
    np.testing.assert_allclose(D, C.T, atol=0)
    for r in range(1, L + 1):
        if r == L or wo[r - 1] - wo[r] > 1e-6 * wo[0]:
            np.testing.assert_allclose(oracle.q_matrix(C, D, r), oracle.q_matrix(Co, Do, r), atol=1e-9)
    for l in range(L):                                   # sign rule: largest-magnitude entry positive
        assert C[np.argmax(np.abs(C[:, l])), l] > 0


def test_klt_and_moments_validation(lib):
    h = pg._vp()
    M = np.eye(4)
    assert lib.pj_basis_create_klt(None, 4, M.ctypes.data_as(pg._dp), None) == ARG
    assert lib.pj_basis_create_klt(ctypes.byref(h), 4, None, None) == ARG
    assert lib.pj_basis_create_klt(ctypes.byref(h), 0, M.ctypes.data_as(pg._dp), None) == ARG
    assert lib.pj_basis_create_klt(ctypes.byref(h), 257, M.ctypes.data_as(pg._dp), None) == ARG
    bad = np.eye(4); bad[0, 1] = 1.0
    assert lib.pj_basis_create_klt(ctypes.byref(h), 4, bad.ctypes.data_as(pg._dp), None) == ARG
    nan = np.eye(4); nan[2, 2] = np.nan
    assert lib.pj_basis_create_klt(ctypes.byref(h), 4, nan.ctypes.data_as(pg._dp), None) == ARG
    n = lib.pj_block_moments_workspace_bytes(1000, 4096, 64)
    assert n > 0 and lib.pj_block_moments_workspace_bytes(0, 4096, 64) == 0
    assert lib.pj_block_moments(64, 1000, 4096, None, 4096, FAKE, FAKE, n, None) == ARG
    assert lib.pj_block_moments(0, 1000, 4096, FAKE, 4096, FAKE, FAKE, n, None) == ARG
    assert lib.pj_block_moments(64, 1000, 4096, FAKE, 4095, FAKE, FAKE, n, None) == SHAPE
    assert lib.pj_block_moments(64, 0, 4096, FAKE, 4096, FAKE, FAKE, n, None) == SHAPE
    assert lib.pj_block_moments(64, 1000, 4096, FAKE, 4096, FAKE, FAKE, n - 1, None) == WS
    assert lib.pj_block_moments(64, 1000, 4096, FAKE, 4096, FAKE, FAKE, n, None) == HIP


def test_conv_circular_validation(lib, basis16):
    W, N = 1024, 37
    n = lib.pj_conv1d_circular_workspace_bytes(W, N, 16, 4, 1)
    assert n > 0
    assert lib.pj_conv1d_circular_workspace_bytes(1000, N, 16, 4, 1) == 0      # W not a multiple of L
    assert lib.pj_conv1d_circular_workspace_bytes(W, W + 1, 16, 4, 1) == 0
    b = basis16
    call = lambda **kw: lib.proj_conv1d_circular(kw.get("h", b.handle), kw.get("r", 4), kw.get("mode", 0),
                                                 kw.get("W", W), FAKE, kw.get("N", N), FAKE, FAKE, kw.get("prec", 1),
                                                 FAKE, kw.get("ws", n), None)
    assert call(h=None) == ARG
    assert call(r=0) == ARG
    assert call(mode=3) == ARG
    assert call(W=1000) == SHAPE
    assert call(N=W + 1) == SHAPE
    assert call(N=0) == SHAPE
    assert call(prec=0) == UNSUP
    assert call(ws=n - 1) == WS
    assert call() == HIP
