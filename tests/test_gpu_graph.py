"""The library's calls replayed from a captured HIP graph (stream capture of
the caller's stream): proj_gemm, proj_gemm_noalloc and proj_conv1d at both
output rates enqueue kernels only, so a captured call must give, on every
replay, exactly the result of the eager call.  Each replay starts from a
cleared output, with eager work and a synchronisation between replays.

Paper: Sec. III-B (GEMM), Sec. III-A eq. (10)-(14) (CONV); the graph
replay itself is a property of this library, not of the paper."""
import numpy as np
import pytest

from paper_1411_2860_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1411_2860_amd import projgemm
    projgemm.lib()
    return projgemm


def _replays_match(call, out, replays=4):
    call()
    torch.cuda.synchronize()
    ref = out.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    for i in range(replays):
        out.fill_(float("nan"))
        scratch = torch.randn(1 << 16, device="cuda")      # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {i} differs from the eager call"
        del scratch
    return ref


@pytest.mark.parametrize("prec", ["f32", "bf16", "bf16x3"])
def test_gemm_replays(pg, prec):
    rng = np.random.default_rng(11)
    M, W, K, L, r = 300, 520, 1000, 16, 5
    A = torch.from_numpy(rng.standard_normal((M, K))).float().cuda()
    B = torch.from_numpy(rng.standard_normal((K, W))).float().cuda()
    basis = pg.Basis("dct2", L)
    R = torch.empty(M, W, device="cuda")
    ws = torch.empty(pg.gemm_workspace_bytes(M, W, K, L, r, prec), dtype=torch.uint8, device="cuda")
    ref = _replays_match(lambda: pg.gemm(A, B, r, basis, prec=prec, out=R, workspace=ws), R)
    assert torch.isfinite(ref).all()


def test_gemm_noalloc_replays(pg):
    rng = np.random.default_rng(12)
    M, W, K, L, r = 256, 384, 640, 16, 8
    A = torch.from_numpy(rng.standard_normal((M, K))).float().cuda()
    B = torch.from_numpy(rng.standard_normal((W, K))).float().cuda()
    basis = pg.Basis("haar", L)
    R = torch.empty(M, W, device="cuda")
    ref = _replays_match(lambda: pg.gemm_noalloc(A, B, r, basis, R, transB=True), R)
    R2 = pg.gemm(A, B, r, basis, transB=True)
    torch.cuda.synchronize()
    assert torch.equal(ref, R2)


@pytest.mark.parametrize("L,r,rate", [(256, 1, "full"), (256, 16, "full"), (64, 4, "block"), (256, 256, "block"),
                                      (2, 1, "block"), (4, 4, "full")])
def test_conv_replays(pg, L, r, rate):
    """Full rate with one launch for both projections (r <= 4), the split
    signal pass, and both block-rate groupings; Haar blocks of 2 and 4."""
    W, N = 40003, 1500
    s = inputs.ar2_signal(W, seed=31)
    k, _ = inputs.excerpt_kernel(s, N, seed=32)
    sd = torch.from_numpy(s.astype(np.float32)).cuda()
    kd = torch.from_numpy(k.astype(np.float32)).cuda()
    basis = pg.Basis("haar" if L <= 4 else "dct2", L)
    y = torch.empty(W - N + 1, device="cuda")
    ws = torch.empty(max(1, pg.conv1d_workspace_bytes(W, N, L, r, rate=rate)), dtype=torch.uint8, device="cuda")
    ref = _replays_match(lambda: pg.conv1d(sd, kd, r, basis, out=y, workspace=ws, rate=rate), y)
    assert torch.isfinite(ref).all()
