"""Seeded synthetic inputs for the projected GEMM / cross-correlation workloads.

This module only makes data: it holds none of the projection method's
arithmetic, so both the HIP path's tests and the CPU oracle may draw inputs
from it.  All generators are NumPy (PCG64 via ``default_rng``) and return
float64 arrays; callers cast as needed.

Stand-ins for the paper's data (the face images of Sec. V-A and the audio of
Sec. V-B are not available):
  * images: independent Gaussian-smoothed white-noise fields (sigma = 4 px),
    min-max scaled to 0..255 and rounded to integers (uint8 range), which
    have the low-frequency energy concentration the DCT-II projection
    exploits (Sec. III-A);
  * signals: a stationary AR(2) process with poles 0.95 and 0.9, whose power
    spectrum is concentrated at low frequencies like audio chroma features;
    template kernels are excerpts of the signal itself.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.ndimage import correlate1d
from scipy.signal import lfilter

__all__ = [
    "gaussian_taps", "smoothed_field", "image_rows", "gaussian_matrix",
    "ar2_signal", "excerpt_kernel", "batched_shapes", "smoothed_rows",
    "SEED_CFG1_A", "SEED_CFG1_B", "SEED_IMG_BASE", "SEED_AR2", "SEED_KERNEL", "SEED_BATCH",
]

SEED_CFG1_A = 14112860
SEED_CFG1_B = 14112861
SEED_IMG_BASE = 2860000
SEED_AR2 = 1411
SEED_KERNEL = 2860
SEED_BATCH = 64


def gaussian_taps(sigma: float) -> np.ndarray:
    """Normalised Gaussian taps of radius ceil(4 sigma)."""
    rad = int(math.ceil(4.0 * sigma))
    x = np.arange(-rad, rad + 1, dtype=np.float64)
    w = np.exp(-0.5 * (x / sigma) ** 2)
    return w / w.sum()


def _to_uint8_range(x: np.ndarray, axes) -> np.ndarray:
    """Min-max scaling to [0, 255], rounded; a constant slice (one sample, or
    equal samples) has no range to scale and becomes the mid value 128."""
    lo = x.min(axis=axes, keepdims=True)
    hi = x.max(axis=axes, keepdims=True)
    span = hi - lo
    flat = span == 0
    scaled = (x - lo) / np.where(flat, 1.0, span) * 255.0
    return np.rint(np.where(flat, 128.0, scaled))


def smoothed_field(rows: int, cols: int, sigma: float = 4.0, seed: int = SEED_CFG1_A) -> np.ndarray:
    """One rows x cols smoothed noise field with integer values in 0..255.

    White noise N(0, 1) on a field padded by the filter radius is filtered
    with a separable Gaussian and cropped (a valid filtering: no boundary
    artefacts), then min-max scaled to [0, 255] and rounded."""
    taps = gaussian_taps(sigma)
    rad = (taps.size - 1) // 2
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((rows + 2 * rad, cols + 2 * rad))
    z = correlate1d(z, taps, axis=0, mode="constant")
    z = correlate1d(z, taps, axis=1, mode="constant")
    z = z[rad:rad + rows, rad:rad + cols]
    return _to_uint8_range(z, axes=None)


def image_rows(n: int, side: int = 64, sigma: float = 4.0, seed_base: int = SEED_IMG_BASE,
               first: int = 0) -> np.ndarray:
    """n images of side x side pixels, image i drawn from seed seed_base + first + i,
    each flattened row-major into one row: returns n x side^2 (values 0..255)."""
    taps = gaussian_taps(sigma)
    rad = (taps.size - 1) // 2
    p = side + 2 * rad
    z = np.empty((n, p, p))
    for i in range(n):
        z[i] = np.random.default_rng(seed_base + first + i).standard_normal((p, p))
    z = correlate1d(z, taps, axis=1, mode="constant")
    z = correlate1d(z, taps, axis=2, mode="constant")
    z = z[:, rad:rad + side, rad:rad + side]
    return _to_uint8_range(z, axes=(1, 2)).reshape(n, side * side)


def smoothed_rows(n: int, length: int, sigma: float = 4.0, seed: int = 0) -> np.ndarray:
    """n independent 1-D smoothed noise sequences of the given length,
    each min-max scaled to 0..255 and rounded: returns n x length."""
    taps = gaussian_taps(sigma)
    rad = (taps.size - 1) // 2
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, length + 2 * rad))
    z = correlate1d(z, taps, axis=1, mode="constant")[:, rad:rad + length]
    return _to_uint8_range(z, axes=1)


def gaussian_matrix(rows: int, cols: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """iid N(0, scale^2) entries."""
    return np.random.default_rng(seed).standard_normal((rows, cols)) * scale


def ar2_signal(n: int, seed: int = SEED_AR2, burn: int = 4096,
               a1: float = 1.85, a2: float = -0.855) -> np.ndarray:
    """s[t] = a1 s[t-1] + a2 s[t-2] + e[t], e ~ N(0, 1); the first `burn`
    samples are dropped.  The defaults put the poles at 0.95 and 0.9."""
    e = np.random.default_rng(seed).standard_normal(n + burn)
    s = lfilter([1.0], [1.0, -a1, -a2], e)
    return s[burn:]


def excerpt_kernel(s: np.ndarray, N: int, seed: int = SEED_KERNEL) -> tuple[np.ndarray, int]:
    """A length-N template cut from the signal at a seeded offset
    o ~ U{0 .. len(s) - N}; returns (kernel, o)."""
    o = int(np.random.default_rng(seed).integers(0, s.size - N + 1))
    return s[o:o + N].copy(), o


def batched_shapes(count: int = 64, lo: int = 128, hi: int = 4096, seed: int = SEED_BATCH):
    """count (M, W, K) triples drawn iid uniform on {lo .. hi}."""
    rng = np.random.default_rng(seed)
    return [tuple(int(v) for v in rng.integers(lo, hi + 1, size=3)) for _ in range(count)]


SEED_FACES = 2205


def face_classes(n_classes: int = 15, per_class: int = 11, side: int = 288, sigma_id: float = 8.0,
                 sigma_var: float = 4.0, var_weight: float = 0.35, seed: int = SEED_FACES):
    """Synthetic stand-in for a face database (Yale-A shape: 15 persons x 11
    images, cropped to 288 x 288).  Class c has an identity field (smoothed
    noise, sigma_id) shared by its images; image i of class c mixes it with
    its own variation field (sigma_var) and a brightness offset:
        img = (1 - var_weight) * id_c + var_weight * var_ci + offset_ci,
    clipped to 0..255.  Returns (images n x side x side float64, labels n,
    index within class n), classes in order."""
    imgs = np.empty((n_classes * per_class, side, side))
    labels = np.empty(n_classes * per_class, dtype=np.int64)
    index = np.empty(n_classes * per_class, dtype=np.int64)
    rng = np.random.default_rng(seed)
    for c in range(n_classes):
        ident = smoothed_field(side, side, sigma=sigma_id, seed=seed * 1000 + c)
        for i in range(per_class):
            var = smoothed_field(side, side, sigma=sigma_var, seed=seed * 100000 + c * 100 + i)
            off = rng.uniform(-20.0, 20.0)
            img = (1.0 - var_weight) * ident + var_weight * var + off
            imgs[c * per_class + i] = np.clip(img, 0.0, 255.0)
            labels[c * per_class + i] = c
            index[c * per_class + i] = i
    return imgs, labels, index
