"""Oracle-side inputs for the GPU parity tests.

The oracle never takes an input from the library: the projection matrices it
uses are its own (oracle.basis, i.e. eq. (7) unnormalised for the DCT-II and
the +1 / -1 Haar pattern), or a host matrix the test itself wrote.  The
projected result does not depend on the scale of the columns of C (D scales
inversely), so the oracle's unnormalised matrices and the library's
orthonormal ones define the same R_hat, and the rounding bounds built from
|C| and |D| coincide as well.
"""
import numpy as np

import oracle


def oracle_basis(kind: str, L: int, C=None):
    """(C, D) from the oracle for a built-in kind, or (C, C^{-1}) with the
    oracle's own inverse for a caller-written custom matrix."""
    if C is not None:
        C = np.asarray(C, dtype=np.float64)
        return C, oracle.invert(C)
    return oracle.basis(kind, L)
