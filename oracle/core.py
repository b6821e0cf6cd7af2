"""ctypes front end of oracle.c plus small pure-NumPy / pure-Python forms.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Three independent routes to the projected GEMM are provided:
  * ``gemm_proj``      -- the C pipeline: project A, project B, accumulate
                          (Sec. III-A/B, eq. (5)-(8));
  * ``gemm_proj_closed`` -- the closed form A Q_{r,K} B with Q_r = C[:, :r] D[:r, :]
                          via numpy.matmul (a library primitive as one step);
  * ``gemm_proj_brute``  -- pure-Python loops over the explicit block-diagonal
                          C_N, S_r, D_N of eq. (15), for tiny shapes.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

__all__ = [
    "build", "lib_path", "threads", "set_threads",
    "basis_dct2", "basis_haar", "basis_identity", "basis", "invert",
    "gemm", "xcorr", "conv",
    "project_a", "project_b", "gemm_proj", "gemm_proj_block", "gemm_proj_grad",
    "gemm_proj_closed", "gemm_proj_brute", "q_matrix", "blockdiag", "gemm_proj_grad_block",
    "project_signal", "project_kernel", "xcorr_proj", "xcorr_proj_at",
    "xcorr_proj_closed", "xcorr_proj_sliding", "xcorr_proj_block_rate", "xcorr_proj_block_rate_at", "xcorr_proj_circular",
    "block_moments", "block_moments_brute", "basis_klt", "pca2d",
    "rel_fro", "snr_db", "work_gemm_plain", "work_gemm_proj",
    "work_conv_plain_time", "work_conv_proj_time", "work_conv_plain_freq", "work_conv_proj_freq",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (no fast-math: the natural
    summation order of the source is kept)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=False)
            lib = ctypes.CDLL(_LIB)
            d = ctypes.POINTER(ctypes.c_double)
            i64 = ctypes.c_int64
            p64 = ctypes.POINTER(ctypes.c_int64)
            ci = ctypes.c_int
            sig = {
                "or_set_threads": (None, [ci]),
                "or_basis_dct2": (None, [ci, d]),
                "or_basis_haar": (ci, [ci, d]),
                "or_basis_identity": (None, [ci, d]),
                "or_invert": (ci, [ci, d, d]),
                "or_gemm": (None, [i64, i64, i64, d, d, d]),
                "or_xcorr": (None, [i64, d, i64, d, d]),
                "or_conv": (None, [i64, d, i64, d, d]),
                "or_project_a": (None, [i64, i64, ci, ci, d, d, d]),
                "or_project_b": (None, [i64, i64, ci, ci, d, d, d]),
                "or_accumulate": (None, [i64, i64, i64, ci, d, d, d]),
                "or_gemm_proj": (ci, [i64, i64, i64, ci, ci, d, d, d, d, d]),
                "or_gemm_proj_block": (ci, [i64, i64, i64, ci, ci, d, d, d, d, i64, p64, i64, p64, d]),
                "or_gemm_proj_grad": (ci, [i64, i64, i64, ci, ci, d, d, d, d, d, d, d]),
                "or_project_signal": (None, [i64, ci, ci, d, d, i64, d]),
                "or_project_kernel": (None, [i64, ci, ci, d, d, d]),
                "or_xcorr_proj_at": (ci, [i64, d, i64, d, ci, ci, d, d, i64, p64, d]),
                "or_xcorr_proj": (ci, [i64, d, i64, d, ci, ci, d, d, d]),
            }
            for name, (res, args) in sig.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


_threads = None


def threads() -> int:
    """Number of OpenMP threads the oracle runs with."""
    if _threads is not None:
        return _threads
    n = os.environ.get("OMP_NUM_THREADS")
    return int(n) if n and n.isdigit() else (os.cpu_count() or 1)


def set_threads(n: int) -> None:
    """Runs the following oracle calls on n OpenMP threads (timing only; the
    results do not depend on it: every parallel loop writes disjoint outputs)."""
    global _threads
    _load().or_set_threads(int(n))
    _threads = int(n)


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _p(x: np.ndarray):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pi(x: np.ndarray):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _ok(rc, what):
    if rc is not None and rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


# ------------------------------------------------------------------- bases

def basis_dct2(L: int) -> np.ndarray:
    """Unnormalised DCT-II of eq. (7): C[i, j] = cos(pi/L (i + 1/2) j)."""
    C = np.empty((L, L))
    _load().or_basis_dct2(L, _p(C))
    return C


def basis_haar(L: int) -> np.ndarray:
    """Unnormalised Haar decomposition basis (+1/-1/0), columns: scaling
    function, then wavelets coarse to fine, shifts ascending."""
    C = np.empty((L, L))
    _ok(_load().or_basis_haar(L, _p(C)), "haar (L must be a power of two)")
    return C


def basis_identity(L: int) -> np.ndarray:
    C = np.empty((L, L))
    _load().or_basis_identity(L, _p(C))
    return C


def invert(C) -> np.ndarray:
    """D = C^{-1} by Gauss-Jordan with partial pivoting (eq. (5): D = C^{-1})."""
    C = _f64(C)
    L = C.shape[0]
    D = np.empty((L, L))
    rc = _load().or_invert(L, _p(C), _p(D))
    if rc == -1:
        raise np.linalg.LinAlgError("singular projection matrix")
    _ok(rc, "invert")
    return D


def basis(kind: str, L: int):
    """(C, D) for kind in {'dct2', 'haar', 'identity'}; D = C^{-1}."""
    C = {"dct2": basis_dct2, "haar": basis_haar, "identity": basis_identity}[kind](L)
    return C, invert(C)


# ---------------------------------------------------------------- exact

def gemm(A, B) -> np.ndarray:
    A, B = _f64(A), _f64(B)
    M, K = A.shape
    K2, W = B.shape
    assert K == K2
    R = np.empty((M, W))
    _load().or_gemm(M, K, W, _p(A), _p(B), _p(R))
    return R


def xcorr(s, k) -> np.ndarray:
    """Valid cross-correlation y[m] = sum_n k[n] s[m+n], m = 0..W-N."""
    s, k = _f64(s), _f64(k)
    y = np.empty(s.size - k.size + 1)
    _load().or_xcorr(s.size, _p(s), k.size, _p(k), _p(y))
    return y


def conv(s, k) -> np.ndarray:
    """Valid convolution (eq. (3)), output index starting where the kernel is
    fully inside the signal."""
    s, k = _f64(s), _f64(k)
    y = np.empty(s.size - k.size + 1)
    _load().or_conv(s.size, _p(s), k.size, _p(k), _p(y))
    return y


# ------------------------------------------------------------ projected GEMM

def project_a(A, C, r: int) -> np.ndarray:
    """A_c^{(l)}[i, j] = sum_t A[i, jL+t] c[t, l]; returns r x M x G."""
    A, C = _f64(A), _f64(C)
    M, K = A.shape
    L = C.shape[0]
    G = -(-K // L)
    out = np.empty((r, M, G))
    _load().or_project_a(M, K, L, r, _p(A), _p(C), _p(out))
    return out


def project_b(B, D, r: int) -> np.ndarray:
    """B_d^{(l)}[j, w] = sum_u d[l, u] B[jL+u, w]; returns r x G x W."""
    B, D = _f64(B), _f64(D)
    K, W = B.shape
    L = D.shape[0]
    G = -(-K // L)
    out = np.empty((r, G, W))
    _load().or_project_b(K, W, L, r, _p(B), _p(D), _p(out))
    return out


def gemm_proj(A, B, C, D, r: int) -> np.ndarray:
    """Projected GEMM, pipeline form: project, project, accumulate."""
    A, B, C, D = _f64(A), _f64(B), _f64(C), _f64(D)
    M, K = A.shape
    W = B.shape[1]
    L = C.shape[0]
    assert 1 <= r <= L and B.shape[0] == K
    R = np.empty((M, W))
    _ok(_load().or_gemm_proj(M, K, W, L, r, _p(A), _p(B), _p(C), _p(D), _p(R)), "gemm_proj")
    return R


def gemm_proj_block(A, B, C, D, r: int, rows, cols) -> np.ndarray:
    """R_hat[rows][:, cols] of the projected GEMM (same pipeline, restricted)."""
    A, B, C, D = _f64(A), _f64(B), _f64(C), _f64(D)
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    cols = np.ascontiguousarray(np.asarray(cols, dtype=np.int64))
    M, K = A.shape
    W = B.shape[1]
    L = C.shape[0]
    out = np.empty((rows.size, cols.size))
    _ok(_load().or_gemm_proj_block(M, K, W, L, r, _p(A), _p(B), _p(C), _p(D),
                                   rows.size, _pi(rows), cols.size, _pi(cols), _p(out)), "gemm_proj_block")
    return out


def gemm_proj_grad(A, B, C, D, r: int, dR):
    """(dA, dB) of R = A Q_{r,K} B for upstream gradient dR."""
    A, B, C, D, dR = _f64(A), _f64(B), _f64(C), _f64(D), _f64(dR)
    M, K = A.shape
    W = B.shape[1]
    L = C.shape[0]
    dA = np.empty((M, K))
    dB = np.empty((K, W))
    _ok(_load().or_gemm_proj_grad(M, K, W, L, r, _p(A), _p(B), _p(C), _p(D), _p(dR), _p(dA), _p(dB)),
        "gemm_proj_grad")
    return dA, dB


def gemm_proj_grad_block(A, B, C, D, r: int, dR, rows_a, cols_a, rows_b, cols_b):
    """Selected gradient entries of R = A Q_{r,K} B: dA[rows_a][:, cols_a] and
    dB[rows_b][:, cols_b], from the definitions dA = dR (Q B)^T and
    dB = (A Q)^T dR with Q = blockdiag(C[:, :r] D[:r, :]) (K zero-extended).
    Each needed row of Q B / column of A Q is formed from its own group."""
    A, B, dR = _f64(A), _f64(B), _f64(dR)
    K = A.shape[1]
    L = _f64(C).shape[0]
    Q = q_matrix(C, D, r)

    def group(k):
        j, t = divmod(int(k), L)
        idx = np.arange(j * L, j * L + L)
        return t, idx, idx < K

    dA = np.empty((len(rows_a), len(cols_a)))
    for b_, k in enumerate(cols_a):
        t, idx, ok = group(k)
        qb = Q[t, ok] @ B[idx[ok], :]                    # row k of Q B
        for a_, i in enumerate(rows_a):
            dA[a_, b_] = float(np.dot(dR[i, :], qb))
    dB = np.empty((len(rows_b), len(cols_b)))
    for a_, k in enumerate(rows_b):
        t, idx, ok = group(k)
        aq = A[:, idx[ok]] @ Q[ok, t]                    # column k of A Q
        for b_, w in enumerate(cols_b):
            dB[a_, b_] = float(np.dot(aq, dR[:, w]))
    return dA, dB


def q_matrix(C, D, r: int) -> np.ndarray:
    """Q_r = C[:, :r] D[:r, :] (L x L)."""
    C, D = _f64(C), _f64(D)
    return C[:, :r] @ D[:r, :]


def blockdiag(X, groups: int) -> np.ndarray:
    """The block-diagonal matrix of eq. (15) with `groups` copies of X."""
    X = _f64(X)
    L = X.shape[0]
    out = np.zeros((groups * L, groups * L))
    for g in range(groups):
        out[g * L:(g + 1) * L, g * L:(g + 1) * L] = X
    return out


def gemm_proj_closed(A, B, C, D, r: int) -> np.ndarray:
    """Closed form A Q_{r,K} B (K zero-extended to a multiple of L)."""
    A, B = _f64(A), _f64(B)
    M, K = A.shape
    L = _f64(C).shape[0]
    G = -(-K // L)
    Ap = np.zeros((M, G * L)); Ap[:, :K] = A
    Bp = np.zeros((G * L, B.shape[1])); Bp[:K] = B
    return Ap @ blockdiag(q_matrix(C, D, r), G) @ Bp


def gemm_proj_brute(A, B, C, D, r: int) -> np.ndarray:
    """Pure-Python loops over the explicit C_N, S_r, D_N of eq. (15):
    R = A C_N S_r D_N B with S_r = blockdiag(diag(1 x r, 0 x (L - r))).
    For tiny shapes only."""
    A, B, C, D = _f64(A).tolist(), _f64(B).tolist(), _f64(C).tolist(), _f64(D).tolist()
    M, K, W, L = len(A), len(A[0]), len(B[0]), len(C)
    G = -(-K // L)
    Kp = G * L
    CN = [[0.0] * Kp for _ in range(Kp)]
    DN = [[0.0] * Kp for _ in range(Kp)]
    S = [[0.0] * Kp for _ in range(Kp)]
    for g in range(G):
        for a in range(L):
            S[g * L + a][g * L + a] = 1.0 if a < r else 0.0
            for b in range(L):
                CN[g * L + a][g * L + b] = C[a][b]
                DN[g * L + a][g * L + b] = D[a][b]
    Ap = [row + [0.0] * (Kp - K) for row in A]
    Bp = B + [[0.0] * W for _ in range(Kp - K)]

    def mm(X, Y):
        n, m, p = len(X), len(Y), len(Y[0])
        return [[sum(X[i][k] * Y[k][j] for k in range(m)) for j in range(p)] for i in range(n)]

    return np.array(mm(mm(mm(mm(Ap, CN), S), DN), Bp))


# ------------------------------------------------------- projected xcorr

def project_signal(s, C, r: int, nb: int | None = None) -> np.ndarray:
    """s_c[l][i] = sum_t s[iL+t] c[t, l]; returns r x nb (default ceil(W/L)+1)."""
    s, C = _f64(s), _f64(C)
    L = C.shape[0]
    if nb is None:
        nb = -(-s.size // L) + 1
    out = np.empty((r, nb))
    _load().or_project_signal(s.size, L, r, _p(s), _p(C), nb, _p(out))
    return out


def project_kernel(k, D, r: int) -> np.ndarray:
    """k_d[l][q + L - 1] = sum_u d[l, u] k[q + u], q = -(L-1)..N-1."""
    k, D = _f64(k), _f64(D)
    L = D.shape[0]
    out = np.empty((r, k.size + L - 1))
    _load().or_project_kernel(k.size, L, r, _p(k), _p(D), _p(out))
    return out


def xcorr_proj(s, k, C, D, r: int) -> np.ndarray:
    """Projected valid cross-correlation, all outputs m = 0..W-N."""
    s, k, C, D = _f64(s), _f64(k), _f64(C), _f64(D)
    L = C.shape[0]
    assert 1 <= r <= L and k.size <= s.size
    y = np.empty(s.size - k.size + 1)
    _ok(_load().or_xcorr_proj(s.size, _p(s), k.size, _p(k), L, r, _p(C), _p(D), _p(y)), "xcorr_proj")
    return y


def xcorr_proj_at(s, k, C, D, r: int, ms) -> np.ndarray:
    """Projected valid cross-correlation at the output positions ms."""
    s, k, C, D = _f64(s), _f64(k), _f64(C), _f64(D)
    ms = np.ascontiguousarray(np.asarray(ms, dtype=np.int64))
    L = C.shape[0]
    y = np.empty(ms.size)
    _ok(_load().or_xcorr_proj_at(s.size, _p(s), k.size, _p(k), L, r, _p(C), _p(D), ms.size, _pi(ms), _p(y)),
        "xcorr_proj_at")
    return y


def xcorr_proj_closed(s, k, C, D, r: int) -> np.ndarray:
    """Closed form: exact valid xcorr of the block-projected signal
    s_tilde (each aligned L-block multiplied by Q_r), via numpy.correlate."""
    s, k = _f64(s), _f64(k)
    L = _f64(C).shape[0]
    nb = -(-s.size // L)
    sp = np.zeros(nb * L); sp[:s.size] = s
    st = (sp.reshape(nb, L) @ q_matrix(C, D, r)).reshape(-1)[:s.size]
    return np.correlate(st, k, mode="valid")


def xcorr_proj_sliding(s, k, C, D, r: int) -> np.ndarray:
    """The other reading of the full-rate projected CONV: the kernel is
    block-projected once and the signal is projected at every offset, i.e.
    the exact xcorr of s with the block-projected kernel.  Used only to show
    that both readings agree at outputs m = 0 mod L when N is a multiple of
    L."""
    s, k = _f64(s), _f64(k)
    L = _f64(C).shape[0]
    nb = -(-k.size // L)
    kp = np.zeros(nb * L); kp[:k.size] = k
    # k enters on the D side: each block k_b becomes Q_r k_b (column form),
    # i.e. k_b Q_r^T as a row.
    kt = (kp.reshape(nb, L) @ q_matrix(C, D, r).T).reshape(-1)
    sp = np.zeros(s.size + nb * L - k.size); sp[:s.size] = s
    return np.correlate(sp, kt, mode="valid")[: s.size - k.size + 1]


def xcorr_proj_circular(s, k, C, D, r: int) -> np.ndarray:
    """Projected circular cross-correlation (Sec. II-B eq. (4): the signal is
    periodic with period W; Sec. III-A: cyclic translations).  W must be a
    multiple of L so that the aligned L-blocks of the periodic signal repeat;
    every block of s is replaced by its reconstruction from the first r
    projections (s_tilde, as in the linear case) and
        y[m] = sum_{n<N} k[n] s_tilde[(m + n) mod W],  m = 0 .. W - 1,
    i.e. the valid cross-correlation of s_tilde extended periodically by N - 1
    samples (numpy.correlate as one step)."""
    s, k = _f64(s), _f64(k)
    L = _f64(C).shape[0]
    W, N = s.size, k.size
    assert W % L == 0 and 1 <= N <= W
    st = (s.reshape(W // L, L) @ q_matrix(C, D, r)).reshape(-1)
    ext = np.concatenate([st, st[:N - 1]])
    return np.correlate(ext, k, mode="valid")


def _interpolate_block_rate(yd, m, L: int) -> np.ndarray:
    """Outputs at positions m from the computed samples yd[a] = y[aL]: exact
    at m = aL, linear between two computed samples, held after the last."""
    nd = yd.size
    a, f = m // L, m % L
    nxt = np.minimum(a + 1, nd - 1)
    y = yd[a] + (f / L) * (yd[nxt] - yd[a])
    return np.where(a + 1 < nd, y, yd[a])


def xcorr_proj_block_rate(s, k, C, D, r: int) -> np.ndarray:
    """Block-rate projected valid cross-correlation (Sec. III-A: results may be
    omitted and interpolated from their neighbours; Sec. IV-A: one projection
    at half the sampling rate for L = 2).  Only the outputs m = aL are computed
    -- aligned signal blocks against aligned kernel blocks, i.e. the projected
    cross-correlation at those positions.  An output aL + f (0 < f < L) lying
    before the next computed output is the linear interpolation
    y[aL] + (f / L) (y[(a+1)L] - y[aL]) (for L = 2 the average of the two
    neighbours); past the last computed output its value is held."""
    s, k = _f64(s), _f64(k)
    L = _f64(C).shape[0]
    nout = s.size - k.size + 1
    nd = (nout - 1) // L + 1
    yd = xcorr_proj_at(s, k, C, D, r, np.arange(nd, dtype=np.int64) * L)
    return _interpolate_block_rate(yd, np.arange(nout), L)


def xcorr_proj_block_rate_at(s, k, C, D, r: int, ms) -> np.ndarray:
    """xcorr_proj_block_rate at the output positions ms only (the computed
    samples they need are evaluated one by one)."""
    s, k = _f64(s), _f64(k)
    L = _f64(C).shape[0]
    nout = s.size - k.size + 1
    nd = (nout - 1) // L + 1
    ms = np.asarray(ms, dtype=np.int64)
    need = np.unique(np.concatenate([ms // L, np.minimum(ms // L + 1, nd - 1)]))
    vals = xcorr_proj_at(s, k, C, D, r, need * L)
    yd = np.zeros(nd)
    yd[need] = vals
    return _interpolate_block_rate(yd, ms, L)


# ------------------------------------------------ data-adaptive (KLT) basis

def block_moments(X, L: int) -> np.ndarray:
    """Second-moment matrix of the aligned L-blocks of the rows of X (K
    zero-extended to a multiple of L): M[t, u] = sum_i sum_j X[i, jL+t] X[i, jL+u].
    One library product (numpy.matmul) over the stacked blocks."""
    X = _f64(X)
    rows, K = X.shape
    G = -(-K // L)
    Xp = np.zeros((rows, G * L))
    Xp[:, :K] = X
    Xb = Xp.reshape(rows * G, L)
    return Xb.T @ Xb


def block_moments_brute(X, L: int) -> np.ndarray:
    """block_moments by plain Python loops (tiny inputs)."""
    X = np.asarray(X, dtype=np.float64)
    rows, K = X.shape
    G = -(-K // L)
    M = [[0.0] * L for _ in range(L)]
    for i in range(rows):
        for j in range(G):
            blk = [X[i, j * L + t] if j * L + t < K else 0.0 for t in range(L)]
            for t in range(L):
                for u in range(L):
                    M[t][u] += blk[t] * blk[u]
    return np.array(M)


def basis_klt(M):
    """Karhunen-Loeve (principal component) basis of a symmetric positive
    semidefinite L x L second-moment matrix: the columns of C are its
    eigenvectors ordered by decreasing eigenvalue (numpy.linalg.eigh), each
    with its largest-magnitude entry made positive; C is orthonormal, so
    D = C^{-1} = C^T.  Returns (C, D, eigenvalues)."""
    M = _f64(M)
    M = (M + M.T) / 2
    w, V = np.linalg.eigh(M)
    order = np.argsort(-w, kind="stable")
    w, V = w[order], V[:, order]
    for j in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, j])))
        if V[i, j] < 0:
            V[:, j] = -V[:, j]
    return V, V.T.copy(), w


# ------------------------------------------------------------------ 2D-PCA

def pca2d(train, test, C, D, r: int, n_axes: int):
    """2D-PCA with every matrix product of eq. (22)-(24) projected (Sec. V-A):
      * training images A_j (m x n) and test images B_i have the training
        mean image subtracted;
      * scatter matrix G = sum_j A_j^T A_j (n x n; the orientation that makes
        Y = A X well defined), one projected GEMM over the vertically stacked
        training images (contraction over the image rows);
      * projection axes X = the eigenvectors of G for its n_axes largest
        eigenvalues (numpy.linalg.eigh, sign rule of basis_klt);
      * features Y_set,j = A_j X and Y_test,i = B_i X, projected GEMMs over the
        stacked images (contraction over the image columns);
      * matching (eq. (25)): nearest training image in Frobenius distance,
        computed exactly.
    Returns dict with G, X, eigenvalues, Y_set (J x m x D), Y_test, dist
    (tests x train squared distances) and match (index of the nearest
    training image per test image, first index on ties)."""
    train, test = _f64(train), _f64(test)
    J, m, n = train.shape
    T = test.shape[0]
    mean = train.mean(axis=0)
    A = (train - mean).reshape(J * m, n)
    B = (test - mean).reshape(T * m, n)
    G = gemm_proj(np.ascontiguousarray(A.T), A, C, D, r)
    G = (G + G.T) / 2
    Vx, _, w = basis_klt(G)
    X = np.ascontiguousarray(Vx[:, :n_axes])
    Ys = gemm_proj(A, X, C, D, r).reshape(J, m, n_axes)
    Yt = gemm_proj(B, X, C, D, r).reshape(T, m, n_axes)
    Fs, Ft = Ys.reshape(J, -1), Yt.reshape(T, -1)
    dist = (Ft * Ft).sum(1)[:, None] + (Fs * Fs).sum(1)[None, :] - 2.0 * (Ft @ Fs.T)
    return {"G": G, "X": X, "eig": w, "Y_set": Ys, "Y_test": Yt, "dist": dist,
            "match": np.argmin(dist, axis=1)}


# -------------------------------------------------------- metrics and counts

def rel_fro(X, ref) -> float:
    """||X - ref||_F / ||ref||_F."""
    X, ref = np.asarray(X, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(X - ref) / den) if den > 0 else float(np.linalg.norm(X - ref))


def snr_db(ref, approx) -> float:
    """eq. (9): 10 log10( sum r^2 / sum (r - r_hat)^2 )."""
    ref, approx = np.asarray(ref, dtype=np.float64), np.asarray(approx, dtype=np.float64)
    num = float(np.sum(ref * ref))
    den = float(np.sum((ref - approx) ** 2))
    return math.inf if den == 0.0 else 10.0 * math.log10(num / den)


def work_gemm_plain(N: int) -> int:
    """eq. (16): MACs of one N x N by N x N subblock product."""
    return N ** 3


def work_gemm_proj(N: int, l: int, L: int) -> float:
    """eq. (17): 2(l+1)N^2 projection MACs + (l+1)/L N^3 product MACs + l N^2
    accumulations, for l+1 projections of L coefficients."""
    return N * N * ((l + 1) / L * N + 3 * l + 2)


def work_conv_plain_time(N: int) -> int:
    """eq. (18): time-domain CONV MACs for the minimum block W = 3N + 1."""
    return 2 * N * N


def work_conv_proj_time(N: int, l: int, L: int) -> int:
    """eq. (20): projection MACs plus the reduced time-domain CONVs."""
    return (l + 1) * (4 * N + 1) + 2 * (l + 1) * (-(-N // L)) ** 2


def work_conv_plain_freq(N: int) -> float:
    """eq. (19): approximate MACs of an FFT-based CONV of a kernel of N
    samples on the minimum overlap-save block of 3N + 1 samples."""
    return (45 * N + 15) * math.log2(3 * N + 1) + 3 * N + 1


def work_conv_proj_freq(N: int, l: int, L: int) -> float:
    """eq. (21): projection MACs plus l + 1 FFT-based CONVs of the
    down-sampled signal and kernel (ceil(N / L) samples each)."""
    n = -(-N // L)
    return (l + 1) * (4 * N + 1) + (l + 1) * ((45 * n + 15) * math.log2(3 * n + 1) + 3 * n + 1)
