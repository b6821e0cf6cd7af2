"""GPU parity of the projected GEMM (C ABI through the ctypes binding) against
the FP64 oracle, element by element within the derived rounding bound
(tests/_tol.py), on the seeded synthetic inputs.

Paper: Sec. III-A/B, eq. (5)-(8), (15)."""
import numpy as np
import pytest

import oracle
from paper_1411_2860_amd import inputs
from tests import _ref, _tol

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KB = {"f64": 8, "f32": 8, "bf16": 16, "f16": 16, "bf16x3": 16, "f16x3": 16, "fp8": 64, "fp8x2": 64}


@pytest.fixture(scope="module")
def pg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1411_2860_amd import projgemm
    projgemm.lib()
    return projgemm


def _dev(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)


def _run(pg, A, B, basis, r, prec, transA=False, transB=False):
    dt = torch.float64 if prec == "f64" else torch.float32
    Ad = _dev(A.T if transA else A, dt)
    Bd = _dev(B.T if transB else B, dt)
    R = pg.gemm(Ad, Bd, r, basis, prec=prec, transA=transA, transB=transB)
    torch.cuda.synchronize()
    return R.double().cpu().numpy()


def _check(pg, A, B, kind, L, r, prec, transA=False, transB=False, Cc=None):
    basis = pg.Basis(kind, L, Cc)
    C, D = _ref.oracle_basis(kind, L, Cc)
    got = _run(pg, A, B, basis, r, prec, transA, transB)
    ref = oracle.gemm_proj(A, B, C, D, r)
    if prec in ("f32", "f64"):
        # the oracle's own basis gives the same projected product
        Co, Do = (Cc, oracle.invert(Cc)) if kind == "custom" else oracle.basis(kind, L)
        np.testing.assert_allclose(oracle.gemm_proj(A, B, Co, Do, r), ref, rtol=1e-9,
                                   atol=1e-9 * np.abs(ref).max())
    Gp = -(-(-(-A.shape[1] // L)) // KB[prec]) * KB[prec]
    bound = _tol.gemm_bound(prec, L, r, Gp, _tol.magnitude(A, B, C, D, r))
    if prec.startswith("fp8"):
        bound = bound + 4.0 * _tol.fp8_floor(A, B, C, D, r, prec)
    _tol.assert_within(got, ref, bound, f"{kind} L={L} r={r} {prec}")
    return got, ref


# ------------------------------------------- FP64 parity configuration
@pytest.mark.parametrize("r", [1, 2, 4, 8, 16])
def test_fp64_parity_256_dct16(pg, r):
    """M = K = W = 256, L = 16 DCT-II, A a smoothed 0..255 field (sigma 4),
    B ~ N(0, 1); every r."""
    A = inputs.smoothed_field(256, 256, sigma=4.0, seed=inputs.SEED_CFG1_A)
    B = inputs.gaussian_matrix(256, 256, seed=inputs.SEED_CFG1_B)
    got, ref = _check(pg, A, B, "dct2", 16, r, "f64")
    if r == 16:
        assert oracle.rel_fro(got, A @ B) < 1e-13


# ----------------------------------- recognition-shaped GEMM, reduced size
@pytest.fixture(scope="module")
def images():
    A = inputs.image_rows(96, seed_base=inputs.SEED_IMG_BASE)                 # queries
    Bt = inputs.image_rows(160, seed_base=inputs.SEED_IMG_BASE, first=1024)   # database rows
    return A, Bt


@pytest.mark.parametrize("r", [1, 3, 8, 16, 64])
def test_fp32_images_transB(pg, images, r):
    """Queries x database^T with 64x64 images (K = 4096), L = 64 DCT-II."""
    A, Bt = images
    got, ref = _check(pg, A, Bt.T, "dct2", 64, r, "f32", transB=True)
    if r == 64:
        assert oracle.rel_fro(got, A @ Bt.T) < 1e-5


@pytest.mark.parametrize("prec", ["bf16", "bf16x3", "f16", "f16x3"])
@pytest.mark.parametrize("r", [1, 16, 64])
def test_reduced_precision_images(pg, images, prec, r):
    A, Bt = images
    _check(pg, A, Bt.T, "dct2", 64, r, prec, transB=True)


@pytest.mark.parametrize("prec", ["fp8", "fp8x2"])
@pytest.mark.parametrize("r", [1, 2, 8])
def test_fp8_images(pg, images, prec, r):
    """Block-scaled FP8 (one E8M0 scale per 32 projected values), r <= 8."""
    A, Bt = images
    got, ref = _check(pg, A, Bt.T, "dct2", 64, r, prec, transB=True)
    # the split form is markedly closer than the single FP8 rounding
    if prec == "fp8x2":
        assert oracle.rel_fro(got, ref) < 2e-3


@pytest.mark.parametrize("prec", ["fp8", "fp8x2"])
def test_fp8_block_scales_vary(pg, prec):
    """Neighbouring 32-index blocks with magnitudes 2^-12 .. 2^12 apart: a scale
    applied to the wrong block breaks the bound by orders of magnitude."""
    rng = np.random.default_rng(33)
    L, K = 8, 8 * 64 * 4
    A = rng.standard_normal((40, K)) * np.exp2(4.0 * ((np.arange(K) // (L * 8)) % 7 - 3))[None, :]
    B = rng.standard_normal((K, 50)) * np.exp2(-3.0 * ((np.arange(K) // (L * 4)) % 9 - 4))[:, None]
    for r in (1, 2, 8):
        _check(pg, A, B, "haar", L, r, prec)


@pytest.mark.parametrize("prec", ["fp8", "fp8x2"])
def test_fp8_ragged(pg, prec):
    rng = np.random.default_rng(31)
    A = rng.standard_normal((70, 333))
    B = rng.standard_normal((333, 90))
    for r in (1, 3, 8):
        _check(pg, A, B, "dct2", 16, r, prec)


# ------------------------------------------------------ ragged and layouts
@pytest.mark.parametrize("M,K,W,L,kind", [
    (77, 1000, 45, 64, "dct2"),     # K not a multiple of L, ragged M and W
    (33, 65, 31, 16, "haar"),
    (1, 1, 1, 8, "dct2"),           # K < L
    (130, 257, 70, 8, "identity"),
    (64, 96, 96, 3, "custom"),      # L not a power of two
    (300, 512, 129, 256, "dct2"),   # the largest L
])
@pytest.mark.parametrize("prec", ["f32", "f64", "bf16x3"])
def test_ragged_shapes_all_r_edges(pg, M, K, W, L, kind, prec):
    rng = np.random.default_rng(M * 7 + K)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, W))
    Cc = rng.standard_normal((L, L)) + 2 * np.eye(L) if kind == "custom" else None
    for r in sorted({1, max(1, L // 2), L}):
        _check(pg, A, B, kind, L, r, prec, Cc=Cc)


@pytest.mark.parametrize("transA,transB", [(False, False), (True, False), (False, True), (True, True)])
def test_layouts(pg, transA, transB):
    rng = np.random.default_rng(5)
    A = rng.standard_normal((70, 200))
    B = rng.standard_normal((200, 90))
    _check(pg, A, B, "dct2", 16, 5, "f32", transA=transA, transB=transB)


def test_beta_accumulates(pg):
    rng = np.random.default_rng(6)
    A = rng.standard_normal((40, 64)).astype(np.float32)
    B = rng.standard_normal((64, 50)).astype(np.float32)
    R0 = rng.standard_normal((40, 50)).astype(np.float32)
    basis = pg.Basis("dct2", 16)
    C, D = _ref.oracle_basis("dct2", 16)
    out = _dev(R0, torch.float32)
    pg.gemm(_dev(A, torch.float32), _dev(B, torch.float32), 4, basis, beta=0.5, out=out)
    torch.cuda.synchronize()
    ref = 0.5 * R0 + oracle.gemm_proj(A, B, C, D, 4)
    np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=1e-5, atol=1e-4)


def test_packed_once_serves_every_r(pg, images):
    """A buffer packed at rmax gives, at every r <= rmax, exactly the result of
    a pack at r (same kernels, same summation order)."""
    A, Bt = images
    basis = pg.Basis("dct2", 64)
    Ad, Bd = _dev(A, torch.float32), _dev(Bt, torch.float32)
    M, K = A.shape
    W = Bt.shape[0]
    Ap = pg.pack_a(Ad, 32, basis)
    Bp = pg.pack_b(Bd, 32, basis, transB=True)
    for r in (1, 7, 32):
        a = pg.gemm_packed(Ap, Bp, r, M, W, K, 64, 32, 32)
        b = pg.gemm_packed(pg.pack_a(Ad, r, basis), pg.pack_b(Bd, r, basis, transB=True), r, M, W, K, 64, r, r)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


# ----------------------------------------- full recognition size, sampled
@pytest.fixture(scope="module")
def full_images():
    A = inputs.image_rows(1024, seed_base=inputs.SEED_IMG_BASE)
    Bt = inputs.image_rows(8192, seed_base=inputs.SEED_IMG_BASE, first=1024)
    return A, Bt


@pytest.mark.parametrize("r", [1, 2, 4, 7, 16, 64])
def test_full_size_sampled(pg, full_images, r):
    """1024 queries x 8192 database images of 64 x 64, L = 64, FP32, in the
    launch configuration the benchmark times; 48 x 48 sampled outputs
    against the oracle; at r = L the sampled error against the exact product
    is below 1e-5."""
    A, Bt = full_images
    basis = pg.Basis("dct2", 64)
    C, D = _ref.oracle_basis("dct2", 64)
    R = pg.gemm(_dev(A, torch.float32), _dev(Bt, torch.float32), r, basis, transB=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(r)
    rows = np.sort(rng.choice(1024, 48, replace=False))
    cols = np.sort(rng.choice(8192, 48, replace=False))
    got = R[torch.from_numpy(rows).cuda()][:, torch.from_numpy(cols).cuda()].double().cpu().numpy()
    ref = oracle.gemm_proj_block(A, Bt.T, C, D, r, rows, cols)
    mag = oracle.gemm_proj_block(np.abs(A), np.abs(Bt.T), np.abs(C), np.abs(D), r, rows, cols)
    _tol.assert_within(got, ref, _tol.gemm_bound("f32", 64, r, 64, mag), f"full size r={r}")
    if r == 64:
        exact = A[rows] @ Bt[cols].T
        assert oracle.rel_fro(got, exact) < 1e-5


@pytest.mark.parametrize("prec,K,L,r", [("f32", 1500, 64, 7), ("bf16", 5440, 16, 3), ("bf16x3", 5440, 16, 3)])
def test_default_tile_ragged_tail(pg, prec, K, L, r):
    """An output large enough for the library's 256 x 128 default tiles with
    ragged sides (1000 x 8200) and contractions that end in a partial trip of
    the four-stage ring: FP32 21 k-blocks (11 steps of 2), BF16 66 k-blocks
    (33 steps of 2), BF16x3 66 k-blocks (66 steps of 1); the last row and
    column tiles are partly outside.  Sampled outputs (both ends included)
    against the oracle."""
    M, W = 1000, 8200
    rng = np.random.default_rng(K + r)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, W))
    basis = pg.Basis("dct2", L)
    C, D = _ref.oracle_basis("dct2", L)
    R = pg.gemm(_dev(A, torch.float32), _dev(B, torch.float32), r, basis, prec=prec)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([[0, 255, 256, M - 1], rng.choice(M, 40, replace=False)]))
    cols = np.unique(np.concatenate([[0, 127, 128, W - 1], rng.choice(W, 40, replace=False)]))
    got = R[torch.from_numpy(rows).cuda()][:, torch.from_numpy(cols).cuda()].double().cpu().numpy()
    A32 = A.astype(np.float32).astype(np.float64)
    B32 = B.astype(np.float32).astype(np.float64)
    ref = oracle.gemm_proj_block(A32, B32, C, D, r, rows, cols)
    mag = oracle.gemm_proj_block(np.abs(A32), np.abs(B32), np.abs(C), np.abs(D), r, rows, cols)
    Gp = -(-(-(-K // L)) // KB[prec]) * KB[prec]
    _tol.assert_within(got, ref, _tol.gemm_bound(prec, L, r, Gp, mag), f"default tile, ragged tail, {prec}")


_SAMPLE_REF = {}


@pytest.mark.parametrize("prec,r", [("bf16", 16), ("f16", 16), ("bf16x3", 16), ("f16x3", 16), ("bf16", 64),
                                    ("f16", 64), ("bf16x3", 64), ("fp8", 8), ("fp8x2", 8)])
def test_full_size_sampled_reduced_precision_every_tile(pg, full_images, prec, r):
    """The recognition workload (1024 x 8192 outputs, K = 4096, L = 64) in the
    reduced-precision modes, packed once and contracted with EVERY tile
    configuration (so also the one the autotuner picks for the benchmark);
    48 x 48 sampled outputs element by element against the oracle within the
    derived bound of the mode (FP8: plus its subnormal floor)."""
    A, Bt = full_images
    basis = pg.Basis("dct2", 64)
    C, D = _ref.oracle_basis("dct2", 64)
    M, K, W, L = 1024, 4096, 8192, 64
    rng = np.random.default_rng(100 + r)
    rows = np.sort(rng.choice(M, 48, replace=False))
    cols = np.sort(rng.choice(W, 48, replace=False))
    key = (r, tuple(rows), tuple(cols))
    if key not in _SAMPLE_REF:
        _SAMPLE_REF.clear()
        _SAMPLE_REF[key] = (oracle.gemm_proj_block(A, Bt.T, C, D, r, rows, cols),
                            oracle.gemm_proj_block(np.abs(A), np.abs(Bt.T), np.abs(C), np.abs(D), r, rows, cols))
    ref, mag = _SAMPLE_REF[key]
    bound = _tol.gemm_bound(prec, L, r, -(-(K // L) // KB[prec]) * KB[prec], mag)
    if prec.startswith("fp8"):
        bound = bound + 4.0 * _tol.fp8_floor(A[rows], np.ascontiguousarray(Bt[cols].T), C, D, r, prec)
    Ad, Bd = _dev(A, torch.float32), _dev(Bt, torch.float32)
    Ap, Bp = pg.pack_ab(Ad, Bd, r, basis, prec=prec, transB=True)
    R = torch.empty((M, W), dtype=torch.float32, device="cuda")
    ri, ci = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
    for cfg in range(len(pg.tile_configs(prec))):
        R.fill_(float("nan"))
        pg.gemm_packed(Ap, Bp, r, M, W, K, L, r, r, prec=prec, out=R, tile_cfg=cfg)
        torch.cuda.synchronize()
        got = R[ri][:, ci].double().cpu().numpy()
        _tol.assert_within(got, ref, bound, f"full size {prec} r={r} tile_cfg={cfg}")


@pytest.mark.parametrize("prec,r,L,K,beta", [
    ("f32", 1, 16, 65536, 0.0), ("f32", 16, 16, 65536, 0.0), ("f32", 7, 12, 60001, 0.5),
    ("bf16x3", 4, 16, 65536, 0.0), ("f16", 8, 8, 32768, 0.0), ("f64", 3, 8, 32768, -1.0), ("fp8", 8, 16, 65536, 0.0),
])
def test_skinny_output_split_contraction(pg, prec, r, L, K, beta):
    """96 x 96 outputs with a long contraction: the k-blocks are cut into
    contiguous ranges contracted by separate workgroups and summed afterwards
    (highest range first); every output against the oracle, with beta."""
    M = W = 96
    rng = np.random.default_rng(K + r)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, W))
    R0 = rng.standard_normal((M, W))
    basis = pg.Basis("dct2", L)
    C, D = _ref.oracle_basis("dct2", L)
    dt = torch.float64 if prec == "f64" else torch.float32
    Ad, Bd = torch.from_numpy(A).to(dt).cuda(), torch.from_numpy(B).to(dt).cuda()
    R = torch.from_numpy(R0).to(dt).cuda()
    nbytes = pg.gemm_workspace_bytes(M, W, K, L, r, prec)
    assert nbytes > pg.packed_bytes(M, K, L, r, prec) + pg.packed_bytes(W, K, L, r, prec)   # partials included
    pg.gemm(Ad, Bd, r, basis, prec=prec, beta=beta, out=R)
    torch.cuda.synchronize()
    A32 = A.astype(np.float32).astype(np.float64) if prec != "f64" else A
    B32 = B.astype(np.float32).astype(np.float64) if prec != "f64" else B
    R32 = R0.astype(np.float32).astype(np.float64) if prec != "f64" else R0
    ref = oracle.gemm_proj(A32, B32, C, D, r) + beta * R32
    Gp = -(-(-(-K // L)) // KB[prec]) * KB[prec]
    bound = _tol.gemm_bound(prec, L, r, Gp, _tol.magnitude(A32, B32, C, D, r)) + 4 * 2 ** -23 * abs(beta) * np.abs(R32)
    if prec.startswith("fp8"):
        bound = bound + 4.0 * _tol.fp8_floor(A32, B32, C, D, r, prec)
    _tol.assert_within(R.double().cpu().numpy(), ref, bound, f"split {prec} r={r} L={L} K={K}")
