"""The seeded synthetic generators are deterministic and have the stated
value ranges and spectra."""
import numpy as np

from paper_1411_2860_amd import inputs


def test_images_deterministic_uint8_range():
    a = inputs.image_rows(3, side=64, seed_base=100)
    b = inputs.image_rows(3, side=64, seed_base=100)
    assert a.shape == (3, 4096) and np.array_equal(a, b)
    assert a.min() == 0 and a.max() == 255 and np.all(a == np.rint(a))
    # image i depends only on its own seed
    c = inputs.image_rows(1, side=64, seed_base=100, first=2)
    assert np.array_equal(c[0], a[2])


def test_smoothed_field_is_lowpass():
    f = inputs.smoothed_field(256, 256, sigma=4.0, seed=1)
    assert f.min() == 0 and f.max() == 255
    spec = np.abs(np.fft.fft2(f - f.mean())) ** 2
    low = spec[:32, :32].sum() + spec[-32:, :32].sum() + spec[:32, -32:].sum() + spec[-32:, -32:].sum()
    assert low / spec.sum() > 0.98   # 1/4 of the band per axis holds > 98 % of the energy


def test_ar2_poles_and_kernel_excerpt():
    s = inputs.ar2_signal(1 << 14, seed=5)
    assert s.size == 1 << 14
    # lag-1 autocorrelation of an AR(2) with poles 0.95, 0.9 is a1 / (1 - a2)
    rho1 = np.corrcoef(s[:-1], s[1:])[0, 1]
    assert abs(rho1 - 1.85 / 1.855) < 0.01
    k, o = inputs.excerpt_kernel(s, 1024, seed=7)
    assert np.array_equal(k, s[o:o + 1024])
    assert np.array_equal(inputs.ar2_signal(100, seed=5, burn=10), inputs.ar2_signal(100, seed=5, burn=10))


def test_batched_shapes_range():
    sh = inputs.batched_shapes()
    assert len(sh) == 64 and sh == inputs.batched_shapes()
    assert all(128 <= v <= 4096 for t in sh for v in t)
