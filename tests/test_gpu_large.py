"""GPU parity at maximum sizes: 64-bit indexing past 2^31 elements / bytes in
the packed operands, the output and the projected signal.

Paper: Sec. III-B (projected GEMM and CONV).  The operands are seeded
Gaussian data drawn on the device with torch's generator (independent of the
library); the oracle evaluates sampled outputs on the host."""
import numpy as np
import pytest

import oracle
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


def test_gemm_output_and_packs_past_2_31(pg):
    """M = W = 48000 (R has 2.3e9 elements), K = 16384, L = 64, r = 64: the
    packed operands (3.1 GB each) and R (9.2 GB) are indexed past 2^31;
    sampled rows / columns include the last ones."""
    M = W = 48000
    K, L, r = 16384, 64, 64
    g = torch.Generator(device="cuda").manual_seed(4800)
    A = torch.randn((M, K), device="cuda", generator=g)
    Bt = torch.randn((W, K), device="cuda", generator=g)
    basis = pg.Basis("dct2", L)
    C, D = _ref.oracle_basis("dct2", L)
    R = pg.gemm(A, Bt, r, basis, prec="f32", transB=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(48)
    rows = np.unique(np.concatenate([[0, M - 1, M - 2], rng.integers(0, M, 13)]))
    cols = np.unique(np.concatenate([[0, W - 1], rng.integers(0, W, 13)]))
    assert rows.max() < M and cols.max() < W
    got = R[torch.from_numpy(rows).cuda()][:, torch.from_numpy(cols).cuda()].double().cpu().numpy()
    A64 = A[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    B64 = Bt[torch.from_numpy(cols).cuda()].double().cpu().numpy().T.copy()
    del A, Bt, R
    torch.cuda.empty_cache()
    ref = oracle.gemm_proj(A64, B64, C, D, r)
    Gp = -(-(K // L) // 8) * 8
    bound = _tol.gemm_bound("f32", L, r, Gp, _tol.magnitude(A64, B64, C, D, r))
    _tol.assert_within(got, ref, bound, "gemm 48000^2")


def test_conv_signal_past_2_30(pg):
    """W = 2^30 + 123 samples (4.3 GB), N = 1000, L = 256, r = 8: sampled
    outputs, including the last, each checked by the oracle on a local window
    that starts on a block boundary (the projected blocks it touches are the
    same as in the whole signal)."""
    W, N, L, r = (1 << 30) + 123, 1000, 256, 8
    g = torch.Generator(device="cuda").manual_seed(1 << 10)
    s = torch.randn(W, device="cuda", generator=g)
    k = torch.randn(N, device="cuda", generator=g)
    basis = pg.Basis("dct2", L)
    C, D = _ref.oracle_basis("dct2", L)
    y = pg.conv1d(s, k, r, basis)
    torch.cuda.synchronize()
    nout = W - N + 1
    rng = np.random.default_rng(30)
    ms = np.unique(np.concatenate([[0, nout - 1, nout - 2, nout - 900], rng.integers(0, nout, 12)]))
    assert ms.min() >= 0 and ms.max() < nout          # checked on the host before the device gather
    got = y[torch.from_numpy(ms).cuda()].double().cpu().numpy()
    kh = k.double().cpu().numpy()
    ref, mag = [], []
    for m in ms:
        base = (int(m) // L) * L
        end = min(W, -(-(int(m) + N) // L) * L + L)
        win = s[base:end].double().cpu().numpy()
        ref.append(oracle.xcorr_proj_at(win, kh, C, D, r, [int(m) - base])[0])
        mag.append(oracle.xcorr_proj_at(np.abs(win), np.abs(kh), np.abs(C), np.abs(D), r, [int(m) - base])[0])
    del s, y
    torch.cuda.empty_cache()
    u = _tol.U["f32"]
    ncp = -(-((N + L - 2) // L + 1) // 8) * 8
    gm = lambda n: n * u / (1 - n * u)
    bound = 4.0 * (2 * gm(L) + gm(r * ncp) + u) * np.array(mag)
    _tol.assert_within(got, np.array(ref), bound, "conv 2^30")
