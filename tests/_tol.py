"""Element-wise rounding-error bounds for comparing the HIP path with the FP64
oracle, derived from the arithmetic each precision mode performs.

Every projected value is an L-term dot product (rounded once to the operand
format), and every output is an n = r * Gp term sum of products accumulated
in FP32 (FP64 for 'f64').  Standard first-order forward error analysis gives,
for each output element,

    |R_gpu - R_hat| <= (2 * gamma_L(u_acc) + 2 * u_op + gamma_n(u_acc)) * Mag

with Mag = sum_{l<r} |A| |C|  (x)  |D| |B|  (the projections of |A| and |B|
with |C| and |D|), u_acc the unit roundoff of the accumulation format and
u_op that of the operand format (0 when operands stay in the accumulation
format).  For the hi + lo split modes the operand term becomes 3 * u_op^2 (the
dropped lo*lo product and the rounding of lo).  The bound is used with a
safety factor of 4 and a floor of the accumulation roundoff.
"""
import numpy as np

import oracle

U = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "bf16": 2.0 ** -8, "f16": 2.0 ** -11, "fp8": 2.0 ** -4}

# FP8 (OCP e4m3) with one power-of-two scale 2^e per 32 values, 2^e <= amax/224:
# values below 2^-6 * 2^e are subnormal, with absolute rounding error up to
# 2^-10 * 2^e <= amax * 2^-10 / 224.
FP8_SUB = 2.0 ** -10 / 224.0

PREC_UNITS = {
    "f64": (U["f64"], 0.0),
    "f32": (U["f32"], 0.0),
    "bf16": (U["f32"], 2 * U["bf16"]),
    "f16": (U["f32"], 2 * U["f16"]),
    "bf16x3": (U["f32"], 3 * U["bf16"] ** 2),
    "f16x3": (U["f32"], 3 * U["f16"] ** 2),
    "fp8": (U["f32"], 2 * U["fp8"] + U["fp8"] ** 2),
    "fp8x2": (U["f32"], 3 * U["fp8"] ** 2 + 2 * U["fp8"] ** 3),
}


def magnitude(A, B, C, D, r):
    """sum_l |A_c^(l)| |B_d^(l)| built from |A|, |B|, |C|, |D| (K x W layout of B)."""
    return oracle.gemm_proj(np.abs(A), np.abs(B), np.abs(C), np.abs(D), r)


def gemm_bound(prec, L, r, Gp, mag, safety=4.0):
    u_acc, op = PREC_UNITS[prec]
    n = r * Gp
    g = lambda m: m * u_acc / (1 - m * u_acc)
    return safety * (2 * g(L) + op + g(n) + u_acc) * mag


def assert_within(got, ref, bound, what=""):
    """|got - ref| <= bound element by element.  Every value of `got` must be
    finite (a NaN or an infinity never passes), and so must `ref`."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    bound = np.broadcast_to(np.asarray(bound, dtype=np.float64), got.shape)
    if got.shape != ref.shape:
        raise AssertionError(f"{what}: shape {got.shape} != reference shape {ref.shape}")
    if not np.isfinite(ref).all():
        raise AssertionError(f"{what}: the reference holds non-finite values")
    nonfinite = ~np.isfinite(got)
    if nonfinite.any():
        i = np.unravel_index(np.argmax(nonfinite), got.shape)
        raise AssertionError(f"{what}: {int(nonfinite.sum())} of {got.size} values not finite; first at {i}: "
                             f"{got[i]!r}")
    err = np.abs(got - ref)
    bad = ~(err <= bound)
    if np.any(bad):
        i = np.unravel_index(np.argmax(np.where(bad, err - bound, -np.inf)), err.shape)
        raise AssertionError(f"{what}: {bad.sum()} of {bad.size} outside bound; worst at {i}: "
                             f"got {got[i]!r} ref {ref[i]!r} err {err[i]:.3e} bound {bound[i]:.3e}")


def fp8_floor(A, B, C, D, r, prec):
    """Absolute term of the FP8 bound from subnormal rounding:
    sum_k (da_k |b_k| + |a_k| db_k) <= FP8_SUB (max|a| sum|b| + sum|a| max|b|)
    per output, over the projected rows of A and columns of B (x2 split: the
    residual's scale is at most 2^-4 of the value's)."""
    Ac = np.abs(oracle.project_a(A, C, r))            # r x M x G
    Bd = np.abs(oracle.project_b(B, D, r))            # r x G x W
    amax = Ac.max(axis=(0, 2))[:, None]
    asum = Ac.sum(axis=(0, 2))[:, None]
    bmax = Bd.max(axis=(0, 1))[None, :]
    bsum = Bd.sum(axis=(0, 1))[None, :]
    f = FP8_SUB * (amax * bsum + asum * bmax)
    return f * (U["fp8"] if prec == "fp8x2" else 1.0)
