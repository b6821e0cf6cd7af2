"""Pins of the oracle's projected cross-correlation / convolution.

Paper: Sec. II-B eq. (3) (convolution; cross-correlation by replacing
k[m - n] with k[m + n]), Sec. III-A eq. (10)-(14) (projected translations,
zero extension for linear xcorr, reversal for convolution, DC-only output),
Sec. III-B (block projection of signal and kernel during blocking).
"""
import numpy as np
import pytest

import oracle
from paper_1411_2860_amd import inputs


def _rand(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


@pytest.mark.parametrize("kind", ["dct2", "haar", "identity"])
@pytest.mark.parametrize("W,N,L", [(100, 16, 4), (257, 33, 8), (64, 64, 16), (50, 1, 2), (130, 7, 1)])
def test_full_r_equals_numpy_correlate(kind, W, N, L):
    C, D = oracle.basis(kind, L)
    s, k = _rand(W, 1), _rand(N, 2)
    ref = np.correlate(s, k, mode="valid")
    np.testing.assert_allclose(oracle.xcorr(s, k), ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.xcorr_proj(s, k, C, D, L), ref, rtol=1e-10, atol=1e-10)


def test_conv_is_xcorr_with_reversed_kernel_and_numpy_convolve():
    s, k = _rand(90, 3), _rand(11, 4)
    np.testing.assert_allclose(oracle.conv(s, k), np.convolve(s, k, mode="valid"), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.conv(s, k), oracle.xcorr(s, k[::-1]), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kind", ["dct2", "haar"])
def test_pipeline_equals_closed_form_every_r(kind):
    """The projected xcorr equals the exact xcorr of the block-projected
    signal (each aligned L-block multiplied by Q_r)."""
    L = 8
    C, D = oracle.basis(kind, L)
    s, k = _rand(203, 5), _rand(29, 6)
    for r in range(1, L + 1):
        np.testing.assert_allclose(oracle.xcorr_proj(s, k, C, D, r), oracle.xcorr_proj_closed(s, k, C, D, r),
                                   rtol=1e-10, atol=1e-10)


def test_brute_force_explicit_block_diagonal():
    """Tiny exhaustive check: s_tilde = Q_{r,W}^T s built from the explicit
    block-diagonal matrix of eq. (15), then the xcorr sum written as
    Python loops."""
    for L in (1, 2, 3, 4):
        C = np.random.default_rng(L).standard_normal((L, L)) + 2 * np.eye(L)
        D = oracle.invert(C)
        for W in (2 * L + 3, 4 * L):
            s, k = _rand(W, W), _rand(L + 1, W + 1)
            nb = -(-W // L)
            for r in range(1, L + 1):
                Q = oracle.blockdiag(C[:, :r] @ D[:r, :], nb)
                sp = np.zeros(nb * L); sp[:W] = s
                st = (sp @ Q)[:W]
                brute = [sum(k[n] * st[m + n] for n in range(k.size)) for m in range(W - k.size + 1)]
                np.testing.assert_allclose(oracle.xcorr_proj(s, k, C, D, r), brute, rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("kind", ["dct2", "haar"])
def test_dc_only_is_block_mean_signal(kind):
    """eq. (14): one projection of the DCT (or Haar) keeps the block DC terms,
    i.e. every aligned L-block of the signal is replaced by its mean."""
    L = 4
    C, D = oracle.basis(kind, L)
    s, k = _rand(61, 7), _rand(9, 8)
    nb = -(-61 // L)
    sp = np.zeros(nb * L); sp[:61] = s
    means = np.repeat(sp.reshape(nb, L).mean(axis=1), L)[:61]
    np.testing.assert_allclose(oracle.xcorr_proj(s, k, C, D, 1), np.correlate(means, k, "valid"),
                               rtol=1e-12, atol=1e-12)


def test_two_readings_agree_on_aligned_outputs():
    """Projecting s in aligned blocks with the kernel projected at every phase,
    and projecting k in blocks with s projected at every offset, give the same
    outputs at m = 0 mod L when N is a multiple of L (Sec. III-A: the
    translated-and-projected inputs); elsewhere they differ."""
    L = 4
    C, D = oracle.basis("dct2", L)
    s, k = _rand(120, 9), _rand(16, 10)
    for r in (1, 2, 3):
        v2 = oracle.xcorr_proj(s, k, C, D, r)
        v1 = oracle.xcorr_proj_sliding(s, k, C, D, r)
        np.testing.assert_allclose(v2[::L], v1[::L], rtol=1e-10, atol=1e-10)
        assert np.max(np.abs(v2 - v1)) > 1e-6


def test_sampled_positions_match_full_output():
    L = 16
    C, D = oracle.basis("dct2", L)
    s = inputs.ar2_signal(1000, seed=11, burn=256)
    k, _ = inputs.excerpt_kernel(s, 64, seed=12)
    ms = np.array([0, 1, 15, 16, 17, 500, 936])
    for r in (1, 4, 16):
        np.testing.assert_allclose(oracle.xcorr_proj_at(s, k, C, D, r, ms), oracle.xcorr_proj(s, k, C, D, r)[ms],
                                   rtol=1e-12, atol=1e-12)


def test_error_decreases_on_ar2_signal():
    """On the low-pass AR(2) stand-in the error shrinks steadily with r
    (energy compaction of the DCT, Sec. III-A); exact at r = L."""
    L = 16
    C, D = oracle.basis("dct2", L)
    s = inputs.ar2_signal(4096, seed=13, burn=512)
    k, _ = inputs.excerpt_kernel(s, 256, seed=14)
    ref = np.correlate(s, k, "valid")
    errs = [oracle.rel_fro(oracle.xcorr_proj(s, k, C, D, r), ref) for r in (1, 2, 4, 8, 16)]
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-12


# ---- block rate (outputs at m = aL, the rest interpolated) ----------------------

@pytest.mark.parametrize("kind,L", [("haar", 2), ("haar", 4), ("dct2", 4), ("dct2", 8)])
@pytest.mark.parametrize("W,N", [(103, 17), (96, 32), (40, 40), (61, 1)])
def test_block_rate_exact_for_affine_output(kind, L, W, N):
    """An affine signal s[n] = alpha n + beta makes the exact cross-correlation
    affine in m; at r = L the computed samples are exact, so the linear
    interpolation between them must reproduce the exact output everywhere
    before the last computed sample, and hold that sample's value after it."""
    C, D = oracle.basis(kind, L)
    s = 0.37 * np.arange(W) - 5.0
    k = _rand(N, 7)
    exact = np.correlate(s, k, mode="valid")
    y = oracle.xcorr_proj_block_rate(s, k, C, D, L)
    nout = W - N + 1
    last = ((nout - 1) // L) * L
    np.testing.assert_allclose(y[:last + 1], exact[:last + 1], rtol=1e-10, atol=1e-9)
    np.testing.assert_allclose(y[last:], np.full(nout - last, exact[last]), rtol=1e-10, atol=1e-9)


@pytest.mark.parametrize("kind,L", [("haar", 2), ("dct2", 4), ("dct2", 16)])
@pytest.mark.parametrize("r", [1, 2])
def test_block_rate_samples_are_the_closed_form(kind, L, r):
    """The computed samples m = aL equal the exact cross-correlation of the
    block-projected signal (an independent route, numpy.correlate) there."""
    C, D = oracle.basis(kind, L)
    s, k = _rand(301, 8), _rand(45, 9)
    y = oracle.xcorr_proj_block_rate(s, k, C, D, r)
    closed = oracle.xcorr_proj_closed(s, k, C, D, r)
    np.testing.assert_allclose(y[::L], closed[::L], rtol=1e-10, atol=1e-10)


def test_block_rate_with_unit_blocks_is_every_output():
    """L = 1: every output is a computed sample, no interpolation."""
    C, D = oracle.basis("identity", 1)
    s, k = _rand(77, 10), _rand(9, 11)
    np.testing.assert_allclose(oracle.xcorr_proj_block_rate(s, k, C, D, 1), np.correlate(s, k, "valid"),
                               rtol=1e-12, atol=1e-12)


def test_block_rate_half_samples_error_is_interpolation_error():
    """L = 2, r = 2 (exact samples): the only error left is the interpolation
    of the odd outputs, which vanishes on the even ones and is bounded by the
    second difference of the exact output on the odd ones."""
    C, D = oracle.basis("haar", 2)
    s = inputs.ar2_signal(4000, seed=12, burn=512)
    k, _ = inputs.excerpt_kernel(s, 200, seed=13)
    exact = np.correlate(s, k, "valid")
    y = oracle.xcorr_proj_block_rate(s, k, C, D, 2)
    np.testing.assert_allclose(y[::2], exact[::2], rtol=1e-9, atol=1e-9)
    odd = np.arange(1, exact.size - 1, 2)
    second = np.abs(exact[odd - 1] - 2 * exact[odd] + exact[odd + 1]) / 2
    assert np.all(np.abs(y[odd] - exact[odd]) <= second + 1e-9)


def test_block_rate_sampled_equals_full():
    C, D = oracle.basis("dct2", 8)
    s, k = _rand(500, 14), _rand(60, 15)
    full = oracle.xcorr_proj_block_rate(s, k, C, D, 3)
    ms = np.array([0, 1, 7, 8, 9, 200, 433, 437, 440])
    np.testing.assert_allclose(oracle.xcorr_proj_block_rate_at(s, k, C, D, 3, ms), full[ms], rtol=0, atol=0)


# ---- circular mode ----------------------------------------------------------------

@pytest.mark.parametrize("kind,L", [("dct2", 4), ("haar", 8), ("identity", 1), ("dct2", 16)])
@pytest.mark.parametrize("W,N", [(64, 5), (128, 128), (48, 1)])
def test_circular_all_projections_is_fft_circular_xcorr(kind, L, W, N):
    """r = L: the exact circular cross-correlation, computed independently in
    the frequency domain (numpy.fft): y = ifft(fft(s) conj(fft(k_padded)))."""
    if W % L:
        pytest.skip("W must be a multiple of L")
    C, D = oracle.basis(kind, L)
    s, k = _rand(W, 20), _rand(N, 21)
    kp = np.zeros(W); kp[:N] = k
    ref = np.real(np.fft.ifft(np.fft.fft(s) * np.conj(np.fft.fft(kp))))
    np.testing.assert_allclose(oracle.xcorr_proj_circular(s, k, C, D, L), ref, rtol=1e-9, atol=1e-9)


def test_circular_brute_force_every_r():
    """Pure loops over the definition with explicit modular indices, on the
    block-projected signal built from the explicit projector Q_r."""
    L, W, N = 4, 24, 7
    C, D = oracle.basis("dct2", L)
    s, k = _rand(W, 22), _rand(N, 23)
    for r in range(1, L + 1):
        Q = oracle.q_matrix(C, D, r)
        st = [sum(s[b * L + t] * Q[t, u] for t in range(L)) for b in range(W // L) for u in range(L)]
        ref = [sum(k[n] * st[(m + n) % W] for n in range(N)) for m in range(W)]
        np.testing.assert_allclose(oracle.xcorr_proj_circular(s, k, C, D, r), ref, rtol=1e-10, atol=1e-10)


def test_circular_agrees_with_linear_away_from_the_wrap():
    """The first W - N + 1 outputs do not wrap: they equal the linear
    projected cross-correlation."""
    C, D = oracle.basis("dct2", 8)
    s, k = _rand(256, 24), _rand(40, 25)
    for r in (1, 3, 8):
        np.testing.assert_allclose(oracle.xcorr_proj_circular(s, k, C, D, r)[:256 - 40 + 1],
                                   oracle.xcorr_proj(s, k, C, D, r), rtol=1e-10, atol=1e-10)
