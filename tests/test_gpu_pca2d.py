"""GPU parity of the 2D-PCA pipeline with projected GEMMs (paper Sec. V-A,
eq. (22)-(26)) against the FP64 oracle on synthetic face-like classes."""
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


def _faces(side, per_class=11, n_train=5, n_classes=15):
    imgs, labels, idx = inputs.face_classes(n_classes=n_classes, per_class=per_class, side=side)
    tr = idx < n_train
    return imgs[tr], labels[tr], imgs[~tr], labels[~tr]


def _run(pg, tr, te, L, r, n_axes):
    from paper_1411_2860_amd.pca2d import PCA2D
    basis = pg.Basis("dct2", L)
    model = PCA2D(basis, r, n_axes).fit(torch.from_numpy(tr).float().cuda())
    ft = model.features(torch.from_numpy(te).float().cuda())
    d = model.distances(ft)
    torch.cuda.synchronize()
    return basis, model, ft, d


@pytest.mark.parametrize("L,r", [(8, 1), (8, 8), (12, 1), (16, 2)])
def test_pipeline_small(pg, L, r):
    """96 x 96 images: scatter within the FP32 GEMM bound, the same leading
    eigenvalues, features and distances close to the oracle's, and every
    decision either the oracle's or within rounding of its distance."""
    tr, ltr, te, lte = _faces(96)
    n_axes = 8
    basis, model, ft, d = _run(pg, tr, te, L, r, n_axes)
    C, D = _ref.oracle_basis("dct2", L)
    ref = oracle.pca2d(tr.astype(np.float32).astype(np.float64), te.astype(np.float32).astype(np.float64),
                       C, D, r, n_axes)
    J, m, n = tr.shape
    mean = tr.astype(np.float32).astype(np.float64).mean(0)
    A = (tr - mean).reshape(J * m, n)
    Gp = -(-(J * m // L) // 8) * 8
    bound = _tol.gemm_bound("f32", L, r, Gp, _tol.magnitude(np.ascontiguousarray(A.T), A, C, D, r))
    # the mean image itself carries FP32 rounding: allow its effect on G
    bound = bound + 4 * 2 ** -23 * (np.abs(A).T @ np.abs(A)) * 4
    _tol.assert_within(model.G.double().cpu().numpy(), ref["G"], bound, f"scatter L={L} r={r}")
    np.testing.assert_allclose(model.eig[:n_axes], ref["eig"][:n_axes], rtol=1e-4)
    dist = d.double().cpu().numpy()
    scale = np.abs(ref["dist"]).max()
    np.testing.assert_allclose(dist, ref["dist"], rtol=0, atol=1e-3 * scale)
    gm = dist.argmin(1)
    dm = ref["dist"][np.arange(gm.size), gm]
    assert np.all(dm <= ref["dist"].min(1) + 1e-3 * scale)
    assert np.mean(ltr[gm] == lte) == np.mean(ltr[ref["match"]] == lte)


def test_pipeline_full_size_yale_a_shape(pg):
    """15 classes x 11 images of 288 x 288 (5 training, 6 test per class),
    10 axes, one of 8 DCT-II projections: the recognition decisions agree
    with the oracle's and every class is recognised as well as with all
    projections."""
    tr, ltr, te, lte = _faces(288)
    basis, model, ft, d = _run(pg, tr, te, 8, 1, 10)
    C, D = _ref.oracle_basis("dct2", 8)
    ref = oracle.pca2d(tr.astype(np.float32).astype(np.float64), te.astype(np.float32).astype(np.float64),
                       C, D, 1, 10)
    gm = d.double().cpu().numpy().argmin(1)
    scale = np.abs(ref["dist"]).max()
    dm = ref["dist"][np.arange(gm.size), gm]
    assert np.all(dm <= ref["dist"].min(1) + 1e-3 * scale)
    np.testing.assert_allclose(model.eig[:10], ref["eig"][:10], rtol=1e-4)


def test_support_kernels(pg):
    """The non-GEMM steps against their definitions: mean image and centred
    images (eq. (22)) within the FP32 summation bound, the symmetric part of
    G (exact: one FP32 add and halving), squared distances of eq. (25) within
    the FP32 accumulation bound."""
    rng = np.random.default_rng(81)
    J, m, n = 7, 33, 29
    X = (rng.random((J, m, n)) * 255).astype(np.float32)
    mean, Xc = pg.images_center(torch.from_numpy(X).cuda())
    torch.cuda.synchronize()
    X64 = X.astype(np.float64)
    u = 2.0 ** -24
    mref = X64.mean(0)
    _tol.assert_within(mean.double().cpu().numpy(), mref, 2 * J * u * np.abs(X64).sum(0) / J + 1e-300, "mean")
    _tol.assert_within(Xc.double().cpu().numpy(), X64 - mref, 2 * J * u * np.abs(X64).sum(0) / J + 2 * u * np.abs(X64)
                       + 1e-300, "centred")
    T = 3
    Bt = (rng.random((T, m, n)) * 255).astype(np.float32)
    Bc = pg.images_subtract(torch.from_numpy(Bt).cuda(), mean)
    torch.cuda.synchronize()
    assert np.array_equal(Bc.cpu().numpy(), Bt - mean.cpu().numpy()), "B - mean is one FP32 subtraction"
    G = rng.standard_normal((45, 45)).astype(np.float32)
    Gd = torch.from_numpy(G).cuda()
    pg.symmetrize(Gd)
    torch.cuda.synchronize()
    Gs = ((G + G.T) * np.float32(0.5)).astype(np.float32)
    assert np.array_equal(Gd.cpu().numpy(), Gs)
    d = 1000
    F = rng.standard_normal((5, d)).astype(np.float32)
    Y = rng.standard_normal((6, d)).astype(np.float32)
    D = pg.sq_distances(torch.from_numpy(F).cuda(), torch.from_numpy(Y).cuda())
    torch.cuda.synchronize()
    diff = F.astype(np.float64)[:, None, :] - Y.astype(np.float64)[None, :, :]
    ref = (diff ** 2).sum(-1)
    bound = (d / 64 + 6 + 3) * u * 1.01 * ref + 1e-300
    _tol.assert_within(D.double().cpu().numpy(), ref, 4 * bound, "squared distances")
