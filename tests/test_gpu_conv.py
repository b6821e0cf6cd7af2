"""GPU parity of the projected 1-D cross-correlation / convolution against the
FP64 oracle, element by element within a derived rounding bound.

Paper: Sec. II-B eq. (3); Sec. III-A eq. (10)-(14); Sec. III-B (projection
during the blocking of the signal and of the kernel)."""
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


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def conv_bound(L, r, N, mag, safety=4.0):
    """Each output sums r * ncp products of two L-term FP32 dot products,
    accumulated in FP32 (see tests/_tol.py for the derivation)."""
    u = _tol.U["f32"]
    ncp = -(-((N + L - 2) // L + 1) // 8) * 8
    g = lambda m: m * u / (1 - m * u)
    return safety * (2 * g(L) + g(r * ncp) + u) * mag


def _check(pg, s, k, kind, L, r, mode="xcorr"):
    basis = pg.Basis(kind, L)
    C, D = _ref.oracle_basis(kind, L)
    y = pg.conv1d(_dev(s), _dev(k), r, basis, mode=mode)
    torch.cuda.synchronize()
    got = y.double().cpu().numpy()
    kk = k[::-1] if mode == "conv" else k
    ref = oracle.xcorr_proj(s, kk, C, D, r)
    mag = oracle.xcorr_proj(np.abs(s), np.abs(kk), np.abs(C), np.abs(D), r)
    _tol.assert_within(got, ref, conv_bound(L, r, k.size, mag), f"{kind} L={L} r={r} N={k.size} {mode}")
    return got, ref


@pytest.mark.parametrize("r", [1, 2, 5, 16])
def test_small_dct16(pg, r):
    s = inputs.ar2_signal(3000, seed=21, burn=512)
    k, _ = inputs.excerpt_kernel(s, 100, seed=22)
    got, ref = _check(pg, s, k, "dct2", 16, r)
    if r == 16:
        assert oracle.rel_fro(got, np.correlate(s, k, "valid")) < 1e-5


@pytest.mark.parametrize("L", [2, 4])
@pytest.mark.parametrize("N", [600, 1200])
def test_paper_operating_points_haar(pg, L, N):
    """Block of 20000 samples, kernels of 600 / 1200 samples, L = 2 and 4 Haar
    (the CONV and music-matching settings of Sec. IV-A and V-B), one
    projection and all projections."""
    s = inputs.ar2_signal(20000, seed=23)
    k, _ = inputs.excerpt_kernel(s, N, seed=24)
    for r in (1, L):
        _check(pg, s, k, "haar", L, r)


@pytest.mark.parametrize("W,N,L,kind", [
    (1000, 1, 8, "dct2"),       # N = 1
    (257, 257, 16, "dct2"),     # N = W: one output
    (999, 37, 16, "haar"),      # nothing aligned
    (513, 64, 1, "identity"),   # L = 1: plain cross-correlation
    (4099, 300, 256, "dct2"),   # largest L
    (700, 33, 5, "dct2"),       # L not a power of two
])
def test_ragged(pg, W, N, L, kind):
    rng = np.random.default_rng(W + N)
    s, k = rng.standard_normal(W), rng.standard_normal(N)
    for r in sorted({1, max(1, L // 2), L}):
        _check(pg, s, k, kind, L, r)


@pytest.mark.parametrize("L", [16, 32, 64, 128, 256])
def test_few_projection_signal_pass(pg, L):
    """r <= 4 with L a power of two: the signal projection reads 256-sample
    steps across lanes (several blocks per step below L = 256) and the block
    holding a ragged tail (W not a multiple of 4) is recomputed from its
    samples; full and block rate."""
    rng = np.random.default_rng(L)
    for W in (20 * L + 3, 20 * L + 4, 7 * L + 1):
        s, k = rng.standard_normal(W), rng.standard_normal(3 * L + 1)
        for r in (1, 3, 4, 8):
            _check(pg, s, k, "dct2", L, r)
            _check_block(pg, s, k, "dct2", L, r)


@pytest.mark.parametrize("r", [7, 33])
def test_half_kblock_phases(pg, r):
    """12 kernel blocks per projection (N = 500, L = 64): every k-block of 8
    contraction indices after the first spans two projections, and with odd
    r the last one is half empty."""
    s = inputs.ar2_signal(20000, seed=27)
    k, _ = inputs.excerpt_kernel(s, 500, seed=28)
    _check(pg, s, k, "dct2", 64, r)


@pytest.mark.parametrize("r", [1, 3, 8])
def test_convolution_mode(pg, r):
    s = inputs.ar2_signal(5000, seed=25)
    k, _ = inputs.excerpt_kernel(s, 200, seed=26)
    got, _ = _check(pg, s, k, "dct2", 8, r, mode="conv")
    if r == 8:
        assert oracle.rel_fro(got, np.convolve(s, k, "valid")) < 1e-5


@pytest.fixture(scope="module")
def long_signal():
    return inputs.ar2_signal(1 << 22, seed=inputs.SEED_AR2)


@pytest.mark.parametrize("N", [1024, 4096, 16384])
@pytest.mark.parametrize("r", [1, 16, 256])
def test_full_size_sampled(pg, long_signal, N, r):
    """2^22-sample AR(2) signal, kernel excerpts of 1024 / 4096 / 16384
    samples, L = 256 DCT-II; 512 sampled outputs (including both ends)
    against the oracle; exact at r = L."""
    s = long_signal
    k, o = inputs.excerpt_kernel(s, N, seed=inputs.SEED_KERNEL)
    basis = pg.Basis("dct2", 256)
    C, D = _ref.oracle_basis("dct2", 256)
    y = pg.conv1d(_dev(s), _dev(k), r, basis)
    torch.cuda.synchronize()
    nout = s.size - N + 1
    rng = np.random.default_rng(N + r)
    ms = np.unique(np.concatenate([[0, 1, 255, 256, nout - 1, o], rng.integers(0, nout, 506)]))
    got = y[torch.from_numpy(ms).cuda()].double().cpu().numpy()
    ref = oracle.xcorr_proj_at(s, k, C, D, r, ms)
    mag = oracle.xcorr_proj_at(np.abs(s), np.abs(k), np.abs(C), np.abs(D), r, ms)
    _tol.assert_within(got, ref, conv_bound(256, r, N, mag), f"full size N={N} r={r}")
    if r == 256:
        exact = np.array([np.dot(k, s[m:m + N]) for m in ms])
        assert oracle.rel_fro(got, exact) < 1e-5


@pytest.mark.parametrize("W,N,L,r", [
    (65536, 4096, 64, 20),      # two projection ranges
    (65536, 4096, 64, 64),      # nine uneven ranges over 64 projections
    (1 << 18, 8192, 256, 64),   # five ranges, 256-phase tiles
])
def test_split_contraction_every_output(pg, W, N, L, r):
    """Long contractions are cut into contiguous projection ranges that run
    as separate workgroups and are summed afterwards; every output checked."""
    s = inputs.ar2_signal(W, seed=27)
    k, _ = inputs.excerpt_kernel(s, N, seed=28)
    _check(pg, s, k, "dct2", L, r)


# ---- block rate: outputs at m = aL, the rest interpolated ----------------------

def _check_block(pg, s, k, kind, L, r, mode="xcorr"):
    basis = pg.Basis(kind, L)
    C, D = _ref.oracle_basis(kind, L)
    y = pg.conv1d(_dev(s), _dev(k), r, basis, mode=mode, rate="block")
    torch.cuda.synchronize()
    got = y.double().cpu().numpy()
    kk = k[::-1] if mode == "conv" else k
    ref = oracle.xcorr_proj_block_rate(s, kk, C, D, r)
    mag = oracle.xcorr_proj_block_rate(np.abs(s), np.abs(kk), np.abs(C), np.abs(D), r)
    _tol.assert_within(got, ref, block_bound(L, r, k.size, mag), f"block {kind} L={L} r={r} N={k.size} {mode}")
    return got, ref


def block_bound(L, r, N, mag, safety=4.0):
    """The computed samples sum either r * ceil(N / L) products of two L-term
    FP32 dot products (projected signal against projected kernel blocks) or
    L * ceil(N / L) products of a signal sample with a kernel value rebuilt
    from its projections (an L-term and an r-term dot product); the bound
    takes the longer sum.  The interpolation is a convex combination of two
    computed samples (its own three roundings add at most 3u of the
    magnitude).  The magnitude sum_l |s C| |D k| is the same for both
    groupings."""
    u = _tol.U["f32"]
    g = lambda m: m * u / (1 - m * u)
    return safety * (2 * g(L) + g(L * -(-N // L)) + 4 * u) * mag


@pytest.mark.parametrize("L", [2, 4])
@pytest.mark.parametrize("N", [600, 1200])
def test_block_rate_paper_operating_points(pg, L, N):
    """Block of 20000 samples, kernels of 600 / 1200 samples, Haar L = 2 and 4:
    one projection at the block rate (half the sampling rate for L = 2,
    missing samples interpolated) and all projections at the block rate."""
    s = inputs.ar2_signal(20000, seed=23)
    k, _ = inputs.excerpt_kernel(s, N, seed=24)
    for r in (1, L):
        _check_block(pg, s, k, "haar", L, r)


@pytest.mark.parametrize("W,N,L,kind", [
    (1000, 1, 8, "dct2"),       # N = 1
    (257, 257, 16, "dct2"),     # one output
    (999, 37, 16, "haar"),      # nothing aligned
    (513, 64, 1, "identity"),   # L = 1: every output computed
    (4099, 300, 256, "dct2"),   # largest L
    (700, 33, 5, "dct2"),       # L not a power of two
    (2001, 97, 10, "dct2"),     # L not a multiple of 4: the rebuilt taps pad L and r to 12 (at r = L)
])
def test_block_rate_ragged(pg, W, N, L, kind):
    rng = np.random.default_rng(W + N + 1)
    s, k = rng.standard_normal(W), rng.standard_normal(N)
    for r in sorted({1, max(1, L // 2), L}):
        _check_block(pg, s, k, kind, L, r)


def test_block_rate_convolution_mode(pg):
    s = inputs.ar2_signal(5000, seed=29)
    k, _ = inputs.excerpt_kernel(s, 200, seed=30)
    _check_block(pg, s, k, "haar", 2, 1, mode="conv")


@pytest.mark.parametrize("r", [16, 256])
def test_block_rate_full_size_sampled(pg, long_signal, r):
    """2^22 samples, N = 16384, L = 256: sampled outputs (computed ones,
    interpolated ones and the held tail) against the oracle."""
    s = long_signal
    N = 16384
    k, o = inputs.excerpt_kernel(s, N, seed=inputs.SEED_KERNEL)
    basis = pg.Basis("dct2", 256)
    C, D = _ref.oracle_basis("dct2", 256)
    y = pg.conv1d(_dev(s), _dev(k), r, basis, rate="block")
    torch.cuda.synchronize()
    nout = s.size - N + 1
    rng = np.random.default_rng(r + 7)
    ms = np.unique(np.concatenate([[0, 1, 255, 256, 257, nout - 1, nout - 2, o], rng.integers(0, nout, 200)]))
    got = y[torch.from_numpy(ms).cuda()].double().cpu().numpy()
    ref = oracle.xcorr_proj_block_rate_at(s, k, C, D, r, ms)
    mag = oracle.xcorr_proj_block_rate_at(np.abs(s), np.abs(k), np.abs(C), np.abs(D), r, ms)
    _tol.assert_within(got, ref, block_bound(256, r, N, mag), f"block full size r={r}")


# ---- circular mode -----------------------------------------------------------------

def _check_circular(pg, s, k, kind, L, r, mode="xcorr"):
    basis = pg.Basis(kind, L)
    C, D = _ref.oracle_basis(kind, L)
    y = pg.conv1d_circular(_dev(s), _dev(k), r, basis, mode=mode)
    torch.cuda.synchronize()
    got = y.double().cpu().numpy()
    kk = k[::-1] if mode == "conv" else k
    ref = oracle.xcorr_proj_circular(s, kk, C, D, r)
    mag = oracle.xcorr_proj_circular(np.abs(s), np.abs(kk), np.abs(C), np.abs(D), r)
    _tol.assert_within(got, ref, conv_bound(L, r, k.size, mag), f"circular {kind} L={L} r={r} N={k.size} {mode}")
    return got, ref


@pytest.mark.parametrize("W,N,L,kind", [
    (4096, 300, 16, "dct2"),
    (4096, 4096, 16, "haar"),     # N = W: every output wraps
    (1024, 1, 8, "dct2"),
    (768, 100, 1, "identity"),    # L = 1: exact circular cross-correlation
    (65536, 2000, 256, "dct2"),
    (700, 33, 5, "dct2"),         # L not a power of two
])
def test_circular(pg, W, N, L, kind):
    s = inputs.ar2_signal(W, seed=31)
    k, _ = inputs.excerpt_kernel(s, N, seed=32)
    for r in sorted({1, max(1, L // 3), L}):
        got, _ = _check_circular(pg, s, k, kind, L, r)
        if r == L:
            kp = np.zeros(W); kp[:N] = k
            exact = np.real(np.fft.ifft(np.fft.fft(s) * np.conj(np.fft.fft(kp))))
            assert oracle.rel_fro(got, exact) < 1e-5


def test_circular_convolution_mode(pg):
    s = inputs.ar2_signal(2048, seed=33)
    k, _ = inputs.excerpt_kernel(s, 150, seed=34)
    _check_circular(pg, s, k, "dct2", 8, 3, mode="conv")


@pytest.mark.parametrize("r", [16, 256])
def test_circular_full_size_sampled(pg, long_signal, r):
    """2^22 samples, N = 16384, L = 256: sampled outputs on both sides of
    the wrap against the linear oracle run on the periodic extension (padded
    to whole blocks, so every block is a copy of one of the signal's)."""
    s = long_signal
    N, L, W = 16384, 256, s.size
    k, _ = inputs.excerpt_kernel(s, N, seed=inputs.SEED_KERNEL)
    basis = pg.Basis("dct2", L)
    C, D = _ref.oracle_basis("dct2", L)
    y = pg.conv1d_circular(_dev(s), _dev(k), r, basis)
    torch.cuda.synchronize()
    rng = np.random.default_rng(r + 11)
    ms = np.unique(np.concatenate([[0, W - N, W - N + 1, W - 1], rng.integers(0, W, 100),
                                   rng.integers(W - N, W, 100)]))
    got = y[torch.from_numpy(ms).cuda()].double().cpu().numpy()
    ext = np.concatenate([s, s[:-(-(N - 1) // L) * L]])
    ref = oracle.xcorr_proj_at(ext, k, C, D, r, ms)
    mag = oracle.xcorr_proj_at(np.abs(ext), np.abs(k), np.abs(C), np.abs(D), r, ms)
    _tol.assert_within(got, ref, conv_bound(L, r, N, mag), f"circular full size r={r}")


# ---- frequency domain (FFT) realisation of the full rate ----------------------

def _fft_geom(W, N, L):
    T = (N + L - 2) // L + 1
    F = 512
    while F < 4096 and 4 * (F - T + 1) < 3 * F:
        F *= 2
    return T, F, F - T + 1


def fft_bound(s, k, C, D, L, r, mag):
    """Rounding of the FFT path per output m = (sP + a)L + b: the projected
    signal rows and kernel taps carry their L-term FP32 dot products (as in
    the direct path), and the F-point transforms of segment s and taps
    h_{l,b}, their product and the inverse transform add about
    u log2(F) ||x_{l,s}||_2 ||h_{l,b}||_1 per projection (the DFT is unitary
    up to sqrt(F), |H| <= ||h||_1); used with a safety factor of 8."""
    u = _tol.U["f32"]
    g = lambda m: m * u / (1 - m * u)
    W, N = s.size, k.size
    T, F, P = _fft_geom(W, N, L)
    nout = W - N + 1
    rows = -(-nout // L)
    nseg = -(-rows // P)
    nb = nseg * P + F
    sc = np.zeros((r, nb))
    pj = oracle.project_signal(s, C, r)
    sc[:, :min(nb, pj.shape[1])] = pj[:, :nb]
    seg = np.array([[np.linalg.norm(sc[l, i * P:i * P + F]) for i in range(nseg)] for l in range(r)])
    kd = oracle.project_kernel(k, D, r)                  # kd[l][q + L - 1], q = -(L - 1) .. N - 1
    h1 = np.zeros((r, L))
    for b in range(L):
        q = np.arange(T) * L - b + L - 1
        ok = (q >= 0) & (q < kd.shape[1])
        h1[:, b] = np.abs(kd[:, q[ok]]).sum(axis=1)
    m = np.arange(nout)
    sidx, b = (m // L) // P, m % L
    fftpart = 8.0 * u * (3 * np.log2(F) + 4) * (seg[:, sidx] * h1[:, b]).sum(axis=0)
    return fftpart + 4.0 * (2 * g(L) + u) * mag


def _check_fft(pg, s, k, kind, L, r, mode="xcorr"):
    basis = pg.Basis(kind, L)
    C, D = _ref.oracle_basis(kind, L)
    y = pg.conv1d_fft(_dev(s), _dev(k), r, basis, mode=mode)
    torch.cuda.synchronize()
    got = y.double().cpu().numpy()
    kk = k[::-1] if mode == "conv" else k
    ref = oracle.xcorr_proj(s, kk, C, D, r)
    mag = oracle.xcorr_proj(np.abs(s), np.abs(kk), np.abs(C), np.abs(D), r)
    _tol.assert_within(got, ref, fft_bound(s, kk, C, D, L, r, mag), f"fft {kind} L={L} r={r} N={k.size} {mode}")
    return got, ref


@pytest.mark.parametrize("r", [1, 4, 16])
def test_fft_long_kernel(pg, r):
    """N / L = 1024 (L = 16, N = 16384 on 2^18 samples of the AR(2) process):
    every output against the oracle; 4096-point transforms, 3072 rows per
    segment (86 segments); at r = L the exact cross-correlation within 1e-5."""
    s = inputs.ar2_signal(1 << 18, seed=31)
    k, _ = inputs.excerpt_kernel(s, 16384, seed=32)
    got, ref = _check_fft(pg, s, k, "dct2", 16, r)
    if r == 16:
        assert oracle.rel_fro(got, np.correlate(s, k, "valid")) < 1e-5


@pytest.mark.parametrize("W,N,L,kind,r", [
    (3000, 100, 4, "haar", 2),       # 512-point transforms, many segments, ragged end
    (5000, 777, 5, "dct2", 3),       # L not a power of two
    (4096, 4096, 8, "dct2", 8),      # one output
    (2049, 2048, 1, "identity", 1),  # L = 1: the plain correlation, 2048 taps
    (70000, 30000, 32, "dct2", 7),   # 938 taps per phase
])
def test_fft_ragged(pg, W, N, L, kind, r):
    rng = np.random.default_rng(W + N)
    s, k = rng.standard_normal(W), rng.standard_normal(N)
    _check_fft(pg, s, k, kind, L, r)


def test_fft_convolution_mode_and_direct_path_agree(pg):
    s = inputs.ar2_signal(20000, seed=33)
    k, _ = inputs.excerpt_kernel(s, 1200, seed=34)
    got, ref = _check_fft(pg, s, k, "haar", 2, 1, mode="conv")
    basis = pg.Basis("haar", 2)
    direct = pg.conv1d(_dev(s), _dev(k), 1, basis, mode="conv")
    torch.cuda.synchronize()
    assert oracle.rel_fro(got, direct.double().cpu().numpy()) < 1e-5


def test_fft_rejects_taps_beyond_transform(pg):
    basis = pg.Basis("dct2", 2)
    assert pg.conv1d_fft_workspace_bytes(1 << 16, 8192, 2, 1) == 0       # 4097 taps per phase
    with pytest.raises(pg.ProjGemmError, match="UNSUPPORTED"):
        s = torch.zeros(1 << 16, device="cuda")
        pg.conv1d_fft(s, torch.zeros(8192, device="cuda"), 1, basis, workspace=torch.empty(256, dtype=torch.uint8,
                                                                                           device="cuda"))


def test_auto_picks_fft_and_direct_still_exact(pg):
    """L = 16, N = 16384 on 2^18 samples, r = 4: the library's choice is the
    frequency-domain path (bit for bit the proj_conv1d_fft result); the direct
    contraction, asked for explicitly, stays within its own bound."""
    s = inputs.ar2_signal(1 << 18, seed=35)
    k, _ = inputs.excerpt_kernel(s, 16384, seed=36)
    L, r = 16, 4
    basis = pg.Basis("dct2", L)
    C, D = _ref.oracle_basis("dct2", L)
    sd, kd = _dev(s), _dev(k)
    auto = pg.conv1d(sd, kd, r, basis)
    fft = pg.conv1d_fft(sd, kd, r, basis)
    direct = pg.conv1d_method(sd, kd, r, basis, method="direct")
    torch.cuda.synchronize()
    assert torch.equal(auto, fft)
    ref = oracle.xcorr_proj(s, k, C, D, r)
    mag = oracle.xcorr_proj(np.abs(s), np.abs(k), np.abs(C), np.abs(D), r)
    _tol.assert_within(direct.double().cpu().numpy(), ref, conv_bound(L, r, k.size, mag), "direct at N/L = 1024")


@pytest.mark.parametrize("L", [12, 24, 32, 48, 64, 96, 128, 200])
def test_direct_phase_tiles_mid_L(pg, L):
    """The direct contraction's phase tile follows L (32, 64, 128 or 256 phases
    per tile, 256 or 128 rows): every output against the oracle, L not
    necessarily a power of two, for r = 1, L / 2 and L."""
    rng = np.random.default_rng(L)
    W, N = 7 * L * 37 + 5, 5 * L + 3
    s, k = rng.standard_normal(W), rng.standard_normal(N)
    basis = pg.Basis("dct2", L)
    C, D = _ref.oracle_basis("dct2", L)
    for r in sorted({1, L // 2, L}):
        y = pg.conv1d_method(_dev(s), _dev(k), r, basis, method="direct")
        torch.cuda.synchronize()
        ref = oracle.xcorr_proj(s, k, C, D, r)
        mag = oracle.xcorr_proj(np.abs(s), np.abs(k), np.abs(C), np.abs(D), r)
        _tol.assert_within(y.double().cpu().numpy(), ref, conv_bound(L, r, N, mag), f"direct L={L} r={r}")
