"""The element-wise parity comparator itself (CPU): a planted NaN, infinity
or out-of-bound value in the result must fail it."""
import numpy as np
import pytest

from tests._tol import assert_within


def _case():
    ref = np.linspace(-1.0, 1.0, 12).reshape(3, 4)
    bound = np.full(ref.shape, 1e-6)
    return ref, bound


def test_accepts_values_within_bound():
    ref, bound = _case()
    assert_within(ref + 5e-7, ref, bound, "within")


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_rejects_non_finite(bad):
    ref, bound = _case()
    got = ref.copy()
    got[1, 2] = bad
    with pytest.raises(AssertionError, match="not finite"):
        assert_within(got, ref, bound, "planted")


def test_rejects_out_of_bound_and_nan_bound():
    ref, bound = _case()
    got = ref.copy()
    got[2, 3] += 1e-5
    with pytest.raises(AssertionError, match="outside bound"):
        assert_within(got, ref, bound, "planted")
    nb = bound.copy()
    nb[0, 0] = np.nan                      # a NaN bound never accepts
    with pytest.raises(AssertionError, match="outside bound"):
        assert_within(ref, ref, nb, "nan bound")


def test_rejects_shape_mismatch():
    ref, bound = _case()
    with pytest.raises(AssertionError, match="shape"):
        assert_within(ref[:2], ref, bound[:2], "shape")
