"""GPU test of the allocation-free entry point proj_gemm_noalloc: through the
C ABI, its output equals proj_gemm's (same kernels, same summation order) and
lies within the FP32 rounding bound of the FP64 oracle, on two calls in a
row, the second with a smaller input (the fixed scratch keeps the first
call's contents).  Also a skinny output whose contraction is split into
ranges (the partials live in the scratch too), and the FP64 path.

Paper: Sec. III-A/B, eq. (5)-(8), (15)."""
import numpy as np
import pytest

import oracle
from paper_1411_2860_amd import inputs
from tests import _ref, _tol

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1411_2860_amd import projgemm
    projgemm.lib()
    return projgemm


def _case(M, W, K, seed):
    A = inputs.smoothed_rows(M, K, sigma=4.0, seed=seed)
    B = inputs.gaussian_matrix(K, W, seed=seed + 1)
    return A, B


@pytest.mark.parametrize("prec,kind,L,r,shapes", [
    ("f32", "dct2", 16, 5, [(300, 520, 1000), (64, 96, 200)]),
    ("bf16x3", "haar", 8, 3, [(257, 300, 777), (33, 40, 50)]),
    ("f32", "dct2", 64, 8, [(96, 128, 65536), (40, 64, 4096)]),     # split contraction, then not
    ("f64", "dct2", 16, 4, [(130, 70, 300), (17, 9, 20)]),
])
def test_noalloc_matches_proj_gemm_twice(pg, prec, kind, L, r, shapes):
    basis = pg.Basis(kind, L)
    C, D = _ref.oracle_basis(kind, L)
    dt = torch.float64 if prec == "f64" else torch.float32
    for i, (M, W, K) in enumerate(shapes):
        print(f"noalloc case prec={prec} L={L} r={r} M={M} W={W} K={K} call {i}", flush=True)
        assert pg.gemm_workspace_bytes(M, W, K, L, r, prec) <= pg.NOALLOC_SCRATCH_BYTES
        A, B = _case(M, W, K, seed=900 + 10 * i)
        Ad = torch.from_numpy(A).to(device="cuda", dtype=dt)
        Bd = torch.from_numpy(B).to(device="cuda", dtype=dt)
        ref_lib = pg.gemm(Ad, Bd, r, basis, prec=prec)
        out = torch.full((M, W), float("nan"), dtype=dt, device="cuda")
        pg.gemm_noalloc(Ad, Bd, r, basis, out, prec=prec)
        torch.cuda.synchronize()
        got = out.double().cpu().numpy()
        assert np.array_equal(got, ref_lib.double().cpu().numpy()), "noalloc differs from proj_gemm"
        A64 = Ad.double().cpu().numpy()
        B64 = Bd.double().cpu().numpy()
        ref = oracle.gemm_proj(A64, B64, C, D, r)
        KB = 8 if prec in ("f32", "f64") else 16
        Gp = -(-(-(-K // L)) // KB) * KB
        bound = _tol.gemm_bound(prec, L, r, Gp, _tol.magnitude(A64, B64, C, D, r))
        _tol.assert_within(got, ref, bound, f"noalloc {prec} M={M} W={W} K={K}")


def test_noalloc_beta_and_too_large(pg):
    basis = pg.Basis("dct2", 16)
    M, W, K, r = 64, 80, 160, 6
    A, B = _case(M, W, K, seed=950)
    Ad = torch.from_numpy(A).float().cuda()
    Bd = torch.from_numpy(B).float().cuda()
    R0 = torch.from_numpy(inputs.gaussian_matrix(M, W, seed=951)).float().cuda()
    ref_lib = pg.gemm(Ad, Bd, r, basis, beta=0.5, out=R0.clone())
    out = R0.clone()
    pg.gemm_noalloc(Ad, Bd, r, basis, out, beta=0.5)
    torch.cuda.synchronize()
    assert torch.equal(out, ref_lib)
    big = torch.empty((1, 1), device="cuda")
    with pytest.raises(pg.ProjGemmError, match="PJ_ERR_SCRATCH"):
        # 8192 x 8192 output, K = 4096: packs far beyond the scratch (checked
        # on the host before any device work; the tiny tensors are never read)
        pg.lib()
        rc = pg.lib().proj_gemm_noalloc(basis.handle, 16, b"N", b"N", 8192, 8192, 4096, big.data_ptr(), 4096,
                                        big.data_ptr(), 8192, 0.0, big.data_ptr(), 8192, 1, None)
        pg._check(rc, "proj_gemm_noalloc")
