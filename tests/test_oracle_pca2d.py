"""Pins of the oracle's 2D-PCA pipeline (paper Sec. V-A, eq. (22)-(26)),
on small synthetic face-like classes."""
import numpy as np
import pytest

import oracle
from paper_1411_2860_amd import inputs


@pytest.fixture(scope="module")
def faces():
    imgs, labels, idx = inputs.face_classes(n_classes=6, per_class=5, side=48, sigma_id=4.0, sigma_var=2.0,
                                            var_weight=0.2)
    tr = idx < 2
    return imgs[tr], labels[tr], imgs[~tr], labels[~tr]


def test_all_projections_equal_the_textbook_2dpca(faces):
    """r = L: the scatter matrix is the per-image sum of A_j^T A_j and the
    features are A_j X, computed image by image (an independent route)."""
    tr, ltr, te, lte = faces
    C, D = oracle.basis("dct2", 8)
    out = oracle.pca2d(tr, te, C, D, 8, 5)
    mean = tr.mean(axis=0)
    G = sum((a - mean).T @ (a - mean) for a in tr)
    np.testing.assert_allclose(out["G"], G, rtol=1e-10, atol=1e-6)
    X = out["X"]
    np.testing.assert_allclose(X.T @ X, np.eye(5), atol=1e-10)
    np.testing.assert_allclose(G @ X, X * out["eig"][:5], rtol=1e-8, atol=1e-6 * out["eig"][0])
    for j, a in enumerate(tr):
        np.testing.assert_allclose(out["Y_set"][j], (a - mean) @ X, rtol=1e-10, atol=1e-7)
    for i, b in enumerate(te):
        np.testing.assert_allclose(out["Y_test"][i], (b - mean) @ X, rtol=1e-10, atol=1e-7)


def test_matching_is_nearest_neighbour_by_brute_force(faces):
    tr, ltr, te, lte = faces
    C, D = oracle.basis("dct2", 8)
    out = oracle.pca2d(tr, te, C, D, 2, 4)
    for i in range(te.shape[0]):
        d = [np.sum((out["Y_test"][i] - out["Y_set"][j]) ** 2) for j in range(tr.shape[0])]
        np.testing.assert_allclose(out["dist"][i], d, rtol=1e-9, atol=1e-6 * max(d))
        assert out["match"][i] == int(np.argmin(d))


@pytest.mark.parametrize("L,r", [(8, 8), (8, 1), (16, 1), (12, 1)])
def test_separable_classes_are_recognised(faces, L, r):
    """Classes whose images share most of their content are recognised
    perfectly, with all projections and with one of L (the claim of Sec. V-A
    that one projection keeps the recognition accuracy, on this synthetic
    stand-in)."""
    tr, ltr, te, lte = faces
    C, D = oracle.basis("dct2", L)
    out = oracle.pca2d(tr, te, C, D, r, 5)
    assert np.all(ltr[out["match"]] == lte)


def test_scatter_is_symmetric_psd_for_every_r(faces):
    """G = A^T Q A-type Gram product: with an orthonormal basis the projected
    scatter is A^T Q_r A = (Q_r A)^T (Q_r A), symmetric positive semidefinite."""
    tr, _, te, _ = faces
    C, D = oracle.basis("dct2", 8)
    for r in (1, 3, 8):
        out = oracle.pca2d(tr, te, C, D, r, 3)
        assert np.all(out["eig"] >= -1e-9 * out["eig"][0])
