"""GPU parity of the batched projected GEMM (one grouped pack launch and one
persistent GEMM launch for many uneven problems) against the FP64 oracle.

Paper: Sec. III-B (the projected GEMM, applied to every problem); the batch,
its persistent schedule and its tile choice are this library's own."""
import numpy as np
import pytest

import oracle
from paper_1411_2860_amd import inputs
from tests import _ref, _tol

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KB = {"f32": 8, "bf16": 16, "bf16x3": 16, "f16": 16, "f16x3": 16, "fp8": 64, "fp8x2": 64}


@pytest.fixture(scope="module")
def pg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1411_2860_amd import projgemm
    projgemm.lib()
    return projgemm


def _bound(prec, A, B, C, D, r, L, mag=None):
    K = A.shape[1]
    Gp = -(-(-(-K // L)) // KB[prec]) * KB[prec]
    if mag is None:
        mag = _tol.magnitude(A, B, C, D, r)
    b = _tol.gemm_bound(prec, L, r, Gp, mag)
    if prec.startswith("fp8"):
        b = b + 4.0 * _tol.fp8_floor(A, B, C, D, r, prec)
    return b


def _small_batch(seed=3):
    rng = np.random.default_rng(seed)
    shapes = [(1, 1, 1), (5, 7, 3), (33, 40, 65), (64, 64, 64), (100, 31, 17), (129, 257, 300),
              (2, 300, 48), (300, 2, 100), (77, 77, 1000), (31, 129, 16)]
    As = [rng.standard_normal((m, k)) for m, w, k in shapes]
    Bs = [rng.standard_normal((k, w)) for m, w, k in shapes]
    return As, Bs


@pytest.mark.parametrize("prec,r", [("f32", 1), ("f32", 7), ("f32", 16), ("bf16", 4), ("bf16x3", 16),
                                    ("f16x3", 8), ("fp8", 1), ("fp8", 8), ("fp8x2", 4)])
def test_small_uneven_batch(pg, prec, r):
    As, Bs = _small_batch()
    L = 16
    basis = pg.Basis("dct2", L)
    C, D = _ref.oracle_basis("dct2", L)
    outs = pg.gemm_batched([torch.from_numpy(a).float().cuda() for a in As],
                           [torch.from_numpy(b).float().cuda() for b in Bs], r, basis, prec=prec)
    torch.cuda.synchronize()
    for i, (A, B, R) in enumerate(zip(As, Bs, outs)):
        ref = oracle.gemm_proj(A, B, C, D, r)
        _tol.assert_within(R.double().cpu().numpy(), ref, _bound(prec, A, B, C, D, r, L), f"problem {i} {prec} r={r}")


@pytest.mark.parametrize("cfg", range(19))
def test_every_tile_config_and_layouts(pg, cfg):
    """Each workgroup tile configuration of the persistent launch, with mixed
    layouts: A stored transposed, B stored transposed."""
    As, Bs = _small_batch(seed=4)
    L, r = 8, 3
    basis = pg.Basis("haar", L)
    C, D = _ref.oracle_basis("haar", L)
    Ad = [torch.from_numpy(np.ascontiguousarray(a.T)).float().cuda() for a in As]
    Bd = [torch.from_numpy(np.ascontiguousarray(b.T)).float().cuda() for b in Bs]
    assert cfg < len(pg.tile_configs("f32"))
    for prec in ("f32", "bf16x3"):
        outs = pg.gemm_batched(Ad, Bd, r, basis, prec=prec, transA=True, transB=True, tile_cfg=cfg)
        torch.cuda.synchronize()
        for i, (A, B, R) in enumerate(zip(As, Bs, outs)):
            ref = oracle.gemm_proj(A, B, C, D, r)
            _tol.assert_within(R.double().cpu().numpy(), ref, _bound(prec, A, B, C, D, r, L),
                               f"cfg {cfg} {prec} problem {i}")


@pytest.mark.parametrize("cfg", [0, 6, 9, 13, 16, 17])
def test_mixed_per_problem_tiles(pg, cfg):
    """One persistent launch running some problems in the configuration's
    tile and the others in its small tile (alternating, and the library's own
    choice), both layouts of B."""
    As, Bs = _small_batch(seed=6)
    L, r = 16, 5
    basis = pg.Basis("dct2", L)
    C, D = _ref.oracle_basis("dct2", L)
    Ad = [torch.from_numpy(a).float().cuda() for a in As]
    for transB in (False, True):
        Bd = [torch.from_numpy(np.ascontiguousarray(b.T if transB else b)).float().cuda() for b in Bs]
        for small in ([i % 2 == 0 for i in range(len(As))], [True] * len(As), None):
            for prec in ("f32", "bf16"):
                outs = pg.gemm_batched(Ad, Bd, r, basis, prec=prec, transB=transB, tile_cfg=cfg, small=small)
                torch.cuda.synchronize()
                for i, (A, B, R) in enumerate(zip(As, Bs, outs)):
                    ref = oracle.gemm_proj(A, B, C, D, r)
                    _tol.assert_within(R.double().cpu().numpy(), ref, _bound(prec, A, B, C, D, r, L),
                                       f"cfg {cfg} {prec} small={small} transB={transB} problem {i}")


def test_batched_equals_single_calls(pg):
    """The batch computes what proj_gemm computes: the same basis, the same
    contraction order; B sides stored K x W are projected column-wise in the
    batch, so the packed values may differ from the single call's in their
    FP32 rounding, and the two results agree within twice the rounding bound
    of one (identical where the packs are).  A stored transposed goes
    column-wise too; with B stored W x K both paths pack identically."""
    As, Bs = _small_batch(seed=5)
    L, r = 16, 5
    basis = pg.Basis("dct2", L)
    C, D = _ref.oracle_basis("dct2", L)
    Ad = [torch.from_numpy(a).float().cuda() for a in As]
    for transB in (False, True):
        Bd = [torch.from_numpy(np.ascontiguousarray(b.T if transB else b)).float().cuda() for b in Bs]
        outs = pg.gemm_batched(Ad, Bd, r, basis, prec="bf16x3", transB=transB, tile_cfg=0, small=[False] * len(As))
        for i, (A, B, Ag, Bg, R) in enumerate(zip(As, Bs, Ad, Bd, outs)):
            R1 = pg.gemm(Ag, Bg, r, basis, prec="bf16x3", transB=transB)
            torch.cuda.synchronize()
            if transB:
                assert torch.equal(R, R1), f"problem {i}: same packs, same tile, different result"
            else:
                _tol.assert_within(R.double().cpu().numpy(), R1.double().cpu().numpy(),
                                   2.0 * _bound("bf16x3", A, B, C, D, r, L), f"problem {i} batch vs single")


@pytest.fixture(scope="module")
def batch64():
    """64 problems with (M, W, K) uniform on 128..4096; A rows are 1-D smoothed
    sequences (sigma 4) in 0..255, B iid N(0, 1)."""
    shapes = inputs.batched_shapes()
    As, Bs = [], []
    for i, (m, w, k) in enumerate(shapes):
        As.append(inputs.smoothed_rows(m, k, sigma=4.0, seed=6400 + i).astype(np.float32))
        Bs.append(inputs.gaussian_matrix(k, w, seed=64000 + i).astype(np.float32))
    return shapes, As, Bs


@pytest.mark.parametrize("prec,r,cfg", [("bf16x3", 4, -1), ("bf16", 16, -1), ("fp8", 8, -1), ("f16x3", 1, -1),
                                         ("bf16x3", 4, 16), ("bf16", 16, 16), ("bf16x3", 1, 17)])
def test_batch64_sampled(pg, batch64, prec, r, cfg):
    """The 64-problem workload, sampled outputs of every problem, in the
    library's default tile and in the tiles the autotuner picks for the
    timed run."""
    shapes, As, Bs = batch64
    L = 16
    basis = pg.Basis("dct2", L)
    C, D = _ref.oracle_basis("dct2", L)
    outs = pg.gemm_batched([torch.from_numpy(a).cuda() for a in As], [torch.from_numpy(b).cuda() for b in Bs],
                           r, basis, prec=prec, tile_cfg=cfg)
    torch.cuda.synchronize()
    rng = np.random.default_rng(r)
    for i, ((m, w, k), A, B, R) in enumerate(zip(shapes, As, Bs, outs)):
        rows = np.sort(rng.choice(m, min(m, 12), replace=False))
        cols = np.sort(rng.choice(w, min(w, 12), replace=False))
        got = R.cpu().numpy().astype(np.float64)[np.ix_(rows, cols)]
        A64, B64 = A.astype(np.float64), B.astype(np.float64)
        ref = oracle.gemm_proj_block(A64, B64, C, D, r, rows, cols)
        mag = oracle.gemm_proj_block(np.abs(A64), np.abs(B64), np.abs(C), np.abs(D), r, rows, cols)
        bound = _bound(prec, A64[rows], B64[:, cols], C, D, r, L, mag=mag)
        _tol.assert_within(got, ref, bound, f"batch64 problem {i} {(m, w, k)} {prec} r={r} cfg={cfg}")
