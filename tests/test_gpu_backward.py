"""GPU parity of the hand-written backward of the projected GEMM and of the
autograd.Function built on it, against the FP64 oracle (closed-form
gradients dA = dR (Q B)^T, dB = (A Q)^T dR), finite differences, and the exact
GEMM gradient at r = L.  Upstream gradients are seeded synthetic inputs."""
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


def _dev(x, dt=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dt)


def _grad_bounds(A, B, C, D, r, dR, prec, L):
    """Rounding bound: the projections (L terms), one contraction over W (dA)
    or M (dB) in the operand format with FP32 (FP64) accumulation, and the
    synthesis (r terms); magnitudes from the gradients of |A|, |B|, |C|, |D|
    and |dR|."""
    u_acc, op = _tol.PREC_UNITS[prec]
    M, W = dR.shape
    g = lambda m: m * u_acc / (1 - m * u_acc)
    mA, mB = oracle.gemm_proj_grad(np.abs(A), np.abs(B), np.abs(C), np.abs(D), r, np.abs(dR))
    bA = 4.0 * (2 * g(L) + g(r) + op + g(W + 4) + u_acc) * mA
    bB = 4.0 * (2 * g(L) + g(r) + op + g(M + 4) + u_acc) * mB
    return bA, bB


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "bf16"])
@pytest.mark.parametrize("transA,transB", [(False, False), (True, True), (False, True)])
def test_backward_parity(pg, prec, transA, transB):
    rng = np.random.default_rng(51)
    M, K, W, L = 37, 150, 29, 16
    A, B, dR = rng.standard_normal((M, K)), rng.standard_normal((K, W)), rng.standard_normal((M, W))
    basis = pg.Basis("dct2", L)
    C, D = _ref.oracle_basis("dct2", L)
    dt = torch.float64 if prec == "f64" else torch.float32
    for r in (1, 5, 16):
        dA, dB = pg.gemm_backward(_dev(A.T if transA else A, dt), _dev(B.T if transB else B, dt), _dev(dR, dt), r,
                                  basis, prec=prec, transA=transA, transB=transB)
        torch.cuda.synchronize()
        gA = dA.double().cpu().numpy()
        gB = dB.double().cpu().numpy()
        gA = gA.T if transA else gA
        gB = gB.T if transB else gB
        rA, rB = oracle.gemm_proj_grad(A, B, C, D, r, dR)
        bA, bB = _grad_bounds(A, B, C, D, r, dR, prec, L)
        _tol.assert_within(gA, rA, bA, f"dA {prec} r={r}")
        _tol.assert_within(gB, rB, bB, f"dB {prec} r={r}")


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "bf16"])
@pytest.mark.parametrize("transA,transB", [(False, False), (True, True), (False, True)])
def test_saved_forward_and_backward(pg, prec, transA, transB):
    """proj_gemm_save: R identical to proj_gemm's, kept projections equal to
    the oracle's A_c and B_d (paper Sec. III-B) within the projection bound;
    proj_gemm_backward_saved within the gradient bound of the oracle's.  The
    library's DCT-II is the orthonormal one, so the kept projections are the
    oracle's with the columns of eq. (7)'s basis scaled to unit length (and
    the rows of D = C^-1 scaled inversely); the product is the same."""
    rng = np.random.default_rng(53)
    M, K, W, L = 45, 150, 33, 16
    A, B, dR = rng.standard_normal((M, K)), rng.standard_normal((K, W)), rng.standard_normal((M, W))
    basis = pg.Basis("dct2", L)
    C, D = _ref.oracle_basis("dct2", L)
    dt = torch.float64 if prec == "f64" else torch.float32
    Ad, Bd = _dev(A.T if transA else A, dt), _dev(B.T if transB else B, dt)
    G = -(-K // L)
    kb = 8 if prec in ("f64", "f32") else 16
    Gp = -(-G // kb) * kb
    u_acc = _tol.PREC_UNITS["f64" if prec == "f64" else "f32"][0]
    for r in (1, 5, 16):
        R, saved = pg.gemm_save(Ad, Bd, r, basis, prec=prec, transA=transA, transB=transB)
        R0 = pg.gemm(Ad, Bd, r, basis, prec=prec, transA=transA, transB=transB)
        torch.cuda.synchronize()
        assert torch.equal(R, R0), f"{prec} r={r}: saved forward differs from proj_gemm"
        assert saved.numel() == pg.gemm_saved_bytes(M, W, K, L, r, prec)
        esz = 8 if prec == "f64" else 4
        nbh = -(-(M * r * Gp * esz) // 256) * 256
        flat = saved.cpu().numpy()
        npdt = np.float64 if prec == "f64" else np.float32
        ah = flat[:M * r * Gp * esz].view(npdt).reshape(M, r, Gp).astype(np.float64)
        bh = flat[nbh:nbh + W * r * Gp * esz].view(npdt).reshape(W, r, Gp).astype(np.float64)
        nrm = np.linalg.norm(C, axis=0)
        Cn, Dn = C / nrm, D * nrm[:, None]
        pa = oracle.project_a(A, Cn, r)                    # r x M x G
        pb = oracle.project_b(B, Dn, r)                    # r x G x W
        ba = 4.0 * L * u_acc * oracle.project_a(np.abs(A), np.abs(Cn), r) + 1e-300
        bb = 4.0 * L * u_acc * oracle.project_b(np.abs(B), np.abs(Dn), r) + 1e-300
        _tol.assert_within(ah[:, :, :G], pa.transpose(1, 0, 2), ba.transpose(1, 0, 2), f"A_hat {prec} r={r}")
        _tol.assert_within(bh[:, :, :G], pb.transpose(2, 0, 1), bb.transpose(2, 0, 1), f"B_hat {prec} r={r}")
        assert not ah[:, :, G:].any() and not bh[:, :, G:].any(), "padded groups must be zero"
        dA, dB = pg.gemm_backward_saved(saved, _dev(dR, dt), r, basis, M, W, K, prec=prec, transA=transA,
                                        transB=transB)
        torch.cuda.synchronize()
        gA = dA.double().cpu().numpy()
        gB = dB.double().cpu().numpy()
        gA = gA.T if transA else gA
        gB = gB.T if transB else gB
        rA, rB = oracle.gemm_proj_grad(A, B, C, D, r, dR)
        bA, bB = _grad_bounds(A, B, C, D, r, dR, prec, L)
        _tol.assert_within(gA, rA, bA, f"saved dA {prec} r={r}")
        _tol.assert_within(gB, rB, bB, f"saved dB {prec} r={r}")


def test_gradcheck_f64(pg):
    """Finite differences of the library's own FP64 forward against its
    backward (torch.autograd.gradcheck)."""
    from paper_1411_2860_amd.autograd import ProjGemmFn
    basis = pg.Basis("haar", 4)
    rng = np.random.default_rng(52)
    A = _dev(rng.standard_normal((5, 10)), torch.float64).requires_grad_()
    B = _dev(rng.standard_normal((10, 3)), torch.float64).requires_grad_()
    for r in (1, 2, 4):
        assert torch.autograd.gradcheck(lambda a, b: ProjGemmFn.apply(a, b, r, basis, "f64"), (A, B),
                                        eps=1e-6, atol=1e-8, rtol=1e-6)


def test_full_r_is_exact_gradient(pg):
    from paper_1411_2860_amd.autograd import proj_matmul
    rng = np.random.default_rng(53)
    A = rng.standard_normal((64, 128))
    B = rng.standard_normal((128, 48))
    dR = rng.standard_normal((64, 48))
    basis = pg.Basis("dct2", 32)
    Ad = _dev(A).requires_grad_()
    Bd = _dev(B).requires_grad_()
    R = proj_matmul(Ad, Bd, 32, basis, "f32")
    R.backward(_dev(dR))
    assert oracle.rel_fro(Ad.grad.double().cpu().numpy(), dR @ B.T) < 1e-5
    assert oracle.rel_fro(Bd.grad.double().cpu().numpy(), A.T @ dR) < 1e-5


def _gelu(x):
    return 0.5 * x * (1.0 + np.tanh(0.7978845608028654 * (x + 0.044715 * x ** 3)))


def _gelu_grad(x):
    t = np.tanh(0.7978845608028654 * (x + 0.044715 * x ** 3))
    return 0.5 * (1 + t) + 0.5 * x * (1 - t * t) * 0.7978845608028654 * (1 + 3 * 0.044715 * x * x)


@pytest.mark.parametrize("r1,r2", [(16, 64), (8, 16)])
def test_mlp_small_end_to_end(pg, r1, r2):
    """Two-layer MLP y = gelu(X Q1 W1) Q2 W2 with loss 1/2 mean((y - T)^2):
    loss and weight gradients against an FP64 reference built from the
    oracle's projected GEMM and its closed-form gradients (BF16 x3 here)."""
    from paper_1411_2860_amd.autograd import proj_matmul
    L = 64
    X = inputs.image_rows(96, seed_base=7000) / 255.0
    W1 = inputs.gaussian_matrix(4096, 256, seed=6, scale=1 / 64.0)
    W2 = inputs.gaussian_matrix(256, 64, seed=7, scale=1 / 16.0)
    T = inputs.gaussian_matrix(96, 64, seed=8)
    C, D = oracle.basis("dct2", L)
    # FP64 reference
    H0 = oracle.gemm_proj(X, W1, C, D, r1)
    H = _gelu(H0)
    Y = oracle.gemm_proj(H, W2, C, D, r2)
    n = Y.size
    loss_ref = 0.5 * np.mean((Y - T) ** 2)
    dY = (Y - T) / n
    dH, dW2_ref = oracle.gemm_proj_grad(H, W2, C, D, r2, dY)
    _, dW1_ref = oracle.gemm_proj_grad(X, W1, C, D, r1, dH * _gelu_grad(H0))
    # GPU
    basis = pg.Basis("dct2", L)
    Xd = _dev(X)
    W1d = _dev(W1).requires_grad_()
    W2d = _dev(W2).requires_grad_()
    Hd = torch.nn.functional.gelu(proj_matmul(Xd, W1d, r1, basis, "bf16x3"), approximate="tanh")
    Yd = proj_matmul(Hd, W2d, r2, basis, "bf16x3")
    loss = 0.5 * torch.mean((Yd - _dev(T)) ** 2)
    loss.backward()
    assert abs(loss.item() - loss_ref) < 1e-4 * loss_ref
    assert oracle.rel_fro(W1d.grad.double().cpu().numpy(), dW1_ref) < 1e-3
    assert oracle.rel_fro(W2d.grad.double().cpu().numpy(), dW2_ref) < 1e-3


def test_mlp_full_size_layer_gradients_sampled(pg):
    """Layer shapes of the 4096 -> 4096 -> 1024 MLP at batch 4096, BF16: the
    backward of each projected layer with a seeded upstream gradient, sampled
    entries against the oracle; the r = L gradient against the exact one."""
    L = 64
    X = inputs.image_rows(4096, seed_base=8000) / 255.0
    W1 = inputs.gaussian_matrix(4096, 4096, seed=5, scale=1 / 64.0)
    dH = inputs.gaussian_matrix(4096, 4096, seed=9, scale=1e-3)
    basis = pg.Basis("dct2", L)
    C, D = _ref.oracle_basis("dct2", L)
    rng = np.random.default_rng(54)
    ra, ca = np.sort(rng.choice(4096, 24, replace=False)), np.sort(rng.choice(4096, 24, replace=False))
    rb, cb = np.sort(rng.choice(4096, 24, replace=False)), np.sort(rng.choice(4096, 24, replace=False))
    for r in (16, 64):
        dA, dB = pg.gemm_backward(_dev(X), _dev(W1), _dev(dH), r, basis, prec="bf16")
        torch.cuda.synchronize()
        gA = dA.double().cpu().numpy()[np.ix_(ra, ca)]
        gB = dB.double().cpu().numpy()[np.ix_(rb, cb)]
        refA, refB = oracle.gemm_proj_grad_block(X, W1, C, D, r, dH, ra, ca, rb, cb)
        magA, magB = oracle.gemm_proj_grad_block(np.abs(X), np.abs(W1), np.abs(C), np.abs(D), r, np.abs(dH),
                                                 ra, ca, rb, cb)
        # Each gradient entry: the projected operand is an L-term FP32 sum, both
        # operands of the reduced contraction are rounded to BF16 once, the
        # contraction accumulates n = 4096 terms in FP32, and the synthesis is
        # an r-term FP32 sum: first-order bound with the usual safety factor.
        u, ub = 2.0 ** -24, 2.0 ** -8
        g = lambda m: m * u / (1 - m * u)
        rel = 4.0 * (g(L) + 2 * ub + g(4096) + g(r) + u)
        _tol.assert_within(gA, refA, rel * magA, f"MLP layer dA r={r}")
        _tol.assert_within(gB, refB, rel * magB, f"MLP layer dB r={r}")
        del dA, dB
