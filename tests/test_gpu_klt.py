"""GPU parity of the data-adaptive (Karhunen-Loeve) basis path: block second
moments on the device against the FP64 oracle, and the projected GEMM with
the trained basis against the oracle with the same C and D.

Paper: Sec. IV-B footnote and Sec. VI (projection coefficients derived
offline by principal component analysis); Sec. III-B (the projected GEMM)."""
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


@pytest.mark.parametrize("rows,K,L,pad", [
    (1, 1, 1, 0), (3, 10, 4, 0), (37, 300, 16, 5), (64, 4096, 64, 0),
    (200, 1000, 100, 3), (513, 4096, 256, 0), (4096, 4096, 64, 0), (8192, 512, 8, 1),
])
def test_block_moments(pg, rows, K, L, pad):
    """Every entry; FP64 accumulation of exact FP32 products, so the only
    error is FP64 summation order (bounded by gamma_n times the sum of |x x|)."""
    X = inputs.smoothed_rows(rows, K + pad, sigma=3.0, seed=rows + K).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()[:, :K] if pad else torch.from_numpy(X).cuda()
    M = pg.block_moments(Xd, L)
    torch.cuda.synchronize()
    X64 = X[:, :K].astype(np.float64)
    ref = oracle.block_moments(X64, L)
    mag = oracle.block_moments(np.abs(X64), L)
    n = rows * -(-K // L)
    u = 2.0 ** -53
    _tol.assert_within(M.cpu().numpy(), ref, 4 * n * u * mag + 1e-300, f"moments rows={rows} K={K} L={L}")


@pytest.mark.parametrize("r", [1, 2, 4, 8, 16])
def test_projected_gemm_with_trained_basis(pg, r):
    """Train on database-like image rows.  The library's eigenbasis (device
    moments, host eigensolver) spans the same leading subspace as the
    oracle's (its projector is what the method uses, and it is unique where
    the eigenvalues are separated); on the training rows it never loses to
    the DCT-II and its residual is the tail eigenvalue sum (Eckart-Young).
    Then the projected GEMM with the oracle's eigenbasis, given to the
    library as a custom matrix, against the oracle within the FP32 bound."""
    L = 16
    train = inputs.image_rows(256, seed_base=inputs.SEED_IMG_BASE, first=5000).astype(np.float32)
    T = train.astype(np.float64)
    M = pg.block_moments(torch.from_numpy(train).cuda(), L)
    basis, eig = pg.klt_basis(M)
    Cl, Dl = basis.matrices()                      # the library's output, under test
    Co, Do, wo = oracle.basis_klt(oracle.block_moments(T, L))
    np.testing.assert_allclose(eig, wo, rtol=1e-9, atol=1e-12 * wo[0])
    gap = wo[r - 1] - (wo[r] if r < L else 0.0)
    # the projectors differ by about the eigensolver error over the gap
    dq = np.linalg.norm(oracle.q_matrix(Cl, Dl, r) - oracle.q_matrix(Co, Do, r))
    assert dq <= 1e-9 * wo[0] / max(gap, 1e-300) + 1e-12
    Q = oracle.blockdiag(oracle.q_matrix(Cl, Dl, r), T.shape[1] // L)
    Cd, Dd = oracle.basis("dct2", L)
    Qd = oracle.blockdiag(oracle.q_matrix(Cd, Dd, r), T.shape[1] // L)
    res_klt = np.linalg.norm(T - T @ Q) ** 2
    res_dct = np.linalg.norm(T - T @ Qd) ** 2
    assert res_klt <= res_dct * (1 + 1e-9) + 1e-12 * np.linalg.norm(T) ** 2
    np.testing.assert_allclose(res_klt, wo[r:].sum(), rtol=1e-6, atol=1e-9 * wo.sum())

    kb = pg.Basis("custom", L, Co)
    A = inputs.image_rows(64, seed_base=inputs.SEED_IMG_BASE).astype(np.float64)
    B = inputs.gaussian_matrix(4096, 96, seed=77)
    R = pg.gemm(torch.from_numpy(A).float().cuda(), torch.from_numpy(B).float().cuda(), r, kb, prec="f32")
    torch.cuda.synchronize()
    C, D = _ref.oracle_basis("custom", L, Co)
    ref = oracle.gemm_proj(A, B, C, D, r)
    Gp = -(-(4096 // L) // 8) * 8
    bound = _tol.gemm_bound("f32", L, r, Gp, _tol.magnitude(A, B, C, D, r))
    _tol.assert_within(R.double().cpu().numpy(), ref, bound, f"klt r={r}")
