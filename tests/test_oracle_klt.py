"""Pins of the oracle's data-adaptive (Karhunen-Loeve / principal component)
basis.  Paper: Sec. IV-B footnote and Sec. VI (projection coefficients
derived offline from training data by principal component analysis, as an
alternative to the fixed DCT / Haar bases of eq. (7))."""
import numpy as np
import pytest

import oracle
from paper_1411_2860_amd import inputs


@pytest.mark.parametrize("rows,K,L", [(3, 8, 4), (2, 10, 4), (5, 7, 8), (1, 1, 2)])
def test_block_moments_equal_brute_force(rows, K, L):
    X = np.random.default_rng(rows * 100 + K).standard_normal((rows, K))
    np.testing.assert_allclose(oracle.block_moments(X, L), oracle.block_moments_brute(X, L), rtol=1e-13, atol=1e-13)


def _training(L=8):
    X = inputs.smoothed_rows(64, 512, sigma=4.0, seed=91)
    return X, oracle.block_moments(X, L)


def test_klt_is_orthonormal_and_diagonalises():
    X, M = _training()
    C, D, w = oracle.basis_klt(M)
    np.testing.assert_allclose(C.T @ C, np.eye(8), atol=1e-12)
    np.testing.assert_allclose(D @ C, np.eye(8), atol=1e-12)
    np.testing.assert_allclose(C @ np.diag(w) @ C.T, M, rtol=1e-10, atol=1e-8 * np.abs(M).max())
    assert np.all(np.diff(w) <= 1e-9 * w[0])           # decreasing
    assert w[-1] >= -1e-9 * w[0]                        # positive semidefinite


@pytest.mark.parametrize("r", [1, 2, 3, 4, 6, 8])
def test_klt_residual_is_tail_energy_and_beats_dct(r):
    """Eckart-Young per block: with the KLT basis the residual energy of the
    training rows, ||X (I - Q_{r,K})||_F^2, equals the sum of the eigenvalues
    past r, and no other orthonormal basis (here the DCT-II) does better."""
    L = 8
    X, M = _training(L)
    C, D, w = oracle.basis_klt(M)
    Q = oracle.blockdiag(oracle.q_matrix(C, D, r), X.shape[1] // L)
    res_klt = np.linalg.norm(X - X @ Q) ** 2
    np.testing.assert_allclose(res_klt, w[r:].sum(), rtol=1e-8, atol=1e-8 * w.sum())
    Cd, Dd = oracle.basis("dct2", L)
    Qd = oracle.blockdiag(oracle.q_matrix(Cd, Dd, r), X.shape[1] // L)
    res_dct = np.linalg.norm(X - X @ Qd) ** 2
    assert res_klt <= res_dct * (1 + 1e-12) + 1e-9


def test_klt_of_rank_one_data():
    """Every block a multiple of one vector v: the first basis vector is
    v / ||v|| (sign fixed), the other eigenvalues vanish, and one projection
    reproduces the data exactly."""
    L = 4
    v = np.array([1.0, -2.0, 0.5, 3.0])
    coef = np.random.default_rng(5).standard_normal((6, 3))
    X = np.concatenate([np.outer(coef[:, j], v) for j in range(3)], axis=1)
    C, D, w = oracle.basis_klt(oracle.block_moments(X, L))
    np.testing.assert_allclose(C[:, 0], v / np.linalg.norm(v), atol=1e-12)
    assert np.all(np.abs(w[1:]) <= 1e-10 * w[0])
    Q = oracle.blockdiag(oracle.q_matrix(C, D, 1), 3)
    np.testing.assert_allclose(X @ Q, X, atol=1e-10)
