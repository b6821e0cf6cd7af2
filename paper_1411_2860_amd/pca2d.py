"""2D-PCA recognition with projected matrix products (paper Sec. V-A,
eq. (22)-(26)).

Training: the training images A_j (m x n, training mean image subtracted) give
the image scatter matrix G = sum_j A_j^T A_j, computed as one projected GEMM
over the vertically stacked images (contraction over the image rows, in
groups of L consecutive rows).  The projection axes X are the eigenvectors of
G for its n_axes largest eigenvalues (the library's host eigensolver).  The
features Y = A X of the training and test images are projected GEMMs over the
stacked images (contraction over the image columns).  Matching picks for each
test image the training image nearest in Frobenius distance (the squared
distances of the flattened features, one wave per pair).  Centring, the
symmetric part of G and the distances run in the library's kernels; torch
only holds the memory.

Scatter orientation: A_j^T A_j (n x n), the one that makes Y = A_j X defined
for non-square images (for square images the printed A_j A_j^T is the other
Gram matrix).  When m is a multiple of L the row groups of the scatter GEMM
never straddle two images.
"""
from __future__ import annotations

import numpy as np

from . import projgemm as pg

__all__ = ["PCA2D"]


class PCA2D:
    """2D-PCA whose three GEMM families (scatter, training features, test
    features) run as projected GEMMs on the first r of L projections."""

    def __init__(self, basis: pg.Basis, r: int, n_axes: int = 10, prec: str = "f32"):
        self.basis, self.r, self.n_axes, self.prec = basis, r, n_axes, prec

    def fit(self, train):
        """train: CUDA float32 tensor J x m x n."""
        import torch
        J, m, n = train.shape
        self.shape = (m, n)
        self.mean, A = pg.images_center(train.contiguous())
        A = A.reshape(J * m, n)
        self.G = pg.symmetrize(pg.gemm(A, A, self.r, self.basis, prec=self.prec, transA=True))
        self.eig, V = pg.sym_eig(self.G)
        self.X = torch.from_numpy(np.ascontiguousarray(V[:, :self.n_axes])).to(train.device, torch.float32)
        self.Y_set = pg.gemm(A, self.X, self.r, self.basis, prec=self.prec).reshape(J, m * self.n_axes)
        return self

    def features(self, images):
        """Y_i = (B_i - mean) X for a CUDA float32 tensor T x m x n: T x (m n_axes)."""
        T = images.shape[0]
        m, n = self.shape
        B = pg.images_subtract(images.contiguous(), self.mean).reshape(T * m, n)
        return pg.gemm(B, self.X, self.r, self.basis, prec=self.prec).reshape(T, m * self.n_axes)

    def distances(self, F_test):
        """Squared Frobenius distances test x training from the features."""
        return pg.sq_distances(F_test.contiguous(), self.Y_set.contiguous())

    def match(self, images):
        """Index of the nearest training image for each test image (eq. (25))."""
        d = self.distances(self.features(images))
        return d.argmin(dim=1)
