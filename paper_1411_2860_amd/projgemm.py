"""Thin ctypes binding of libprojgemm.so (include/projgemm.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI.  PyTorch supplies device memory (tensors, the
workspace) and the current stream.  If the library is not built, every call
raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

__all__ = [
    "ProjGemmError", "lib", "lib_path", "Basis", "PREC", "BASIS",
    "gemm", "gemm_noalloc", "pack_a", "pack_b", "pack_ab", "tile_configs", "gemm_packed", "packed_bytes", "gemm_workspace_bytes",
    "conv1d", "conv1d_workspace_bytes", "conv1d_fft", "conv1d_fft_workspace_bytes", "conv1d_method",
    "conv1d_method_workspace_bytes", "gemm_backward", "gemm_save", "gemm_saved_bytes",
    "gemm_backward_saved", "GemmDesc", "gemm_batched", "gemm_batched_workspace_bytes",
    "images_center", "images_subtract", "symmetrize", "sq_distances", "status_str",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libprojgemm.so")
_lock = threading.Lock()
_lib = None

PREC = {"f64": 0, "f32": 1, "bf16": 2, "bf16x3": 3, "f16": 4, "f16x3": 5, "fp8": 6, "fp8x2": 7}
BASIS = {"dct2": 0, "haar": 1, "identity": 2, "custom": 3}
STATUS = {0: "PJ_OK", -1: "PJ_ERR_ARG", -2: "PJ_ERR_SHAPE", -3: "PJ_ERR_UNSUPPORTED",
          -4: "PJ_ERR_WORKSPACE", -5: "PJ_ERR_SINGULAR", -6: "PJ_ERR_HIP", -7: "PJ_ERR_SCRATCH"}
NOALLOC_SCRATCH_BYTES = 64 << 20      # PJ_NOALLOC_SCRATCH_BYTES of the header


class ProjGemmError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {STATUS.get(code, code)} ({status_str(code)})")


def lib_path() -> str:
    return _LIB_PATH


_vp = ctypes.c_void_p
_i = ctypes.c_int
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t
_ch = ctypes.c_char
_f = ctypes.c_float
_dp = ctypes.POINTER(ctypes.c_double)

_SIGNATURES = {
    "pj_status_str": (ctypes.c_char_p, [_i]),
    "pj_basis_create": (_i, [ctypes.POINTER(_vp), _i, _i, _dp]),
    "pj_basis_get": (_i, [_vp, _dp, _dp]),
    "pj_basis_L": (_i, [_vp]),
    "pj_basis_destroy": (_i, [_vp]),
    "pj_gemm_workspace_bytes": (_sz, [_i, _i, _i, _i, _i, _i]),
    "pj_packed_bytes": (_sz, [_i, _i, _i, _i, _i]),
    "proj_gemm": (_i, [_vp, _i, _ch, _ch, _i, _i, _i, _vp, _i64, _vp, _i64, _f, _vp, _i64, _i, _vp, _sz, _vp]),
    "proj_gemm_noalloc": (_i, [_vp, _i, _ch, _ch, _i, _i, _i, _vp, _i64, _vp, _i64, _f, _vp, _i64, _i, _vp]),
    "pj_pack_a": (_i, [_vp, _i, _ch, _i, _i, _vp, _i64, _i, _vp, _sz, _vp]),
    "pj_pack_b": (_i, [_vp, _i, _ch, _i, _i, _vp, _i64, _i, _vp, _sz, _vp]),
    "pj_gemm_packed": (_i, [_i, _i, _i, _i, _i, _i, _vp, _i, _sz, _vp, _i, _sz, _f, _vp, _i64, _i, _vp]),
    "pj_pack_ab": (_i, [_vp, _i, _ch, _ch, _i, _i, _i, _vp, _i64, _vp, _i64, _i, _vp, _sz, _vp, _sz, _vp]),
    "pj_gemm_tile_configs": (_i, [_i, ctypes.POINTER(_i), ctypes.POINTER(_i), _i]),
    "pj_conv1d_workspace_bytes": (_sz, [_i64, _i, _i, _i, _i]),
    "pj_gemm_batched_workspace_bytes": (_sz, [_i, _vp, _i, _i, _i, _i]),
    "proj_gemm_batched": (_i, [_vp, _i, _i, _vp, _f, _i, _i, _vp, _sz, _vp]),
    "pj_gemm_batched_tiles_workspace_bytes": (_sz, [_i, _vp, _vp, _i, _i, _i, _i]),
    "proj_gemm_batched_tiles": (_i, [_vp, _i, _i, _vp, _vp, _f, _i, _i, _vp, _sz, _vp]),
    "pj_gemm_backward_workspace_bytes": (_sz, [_i, _i, _i, _i, _i, _i]),
    "proj_gemm_backward": (_i, [_vp, _i, _ch, _ch, _i, _i, _i, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp,
                                _i64, _i, _vp, _sz, _vp]),
    "pj_images_center": (_i, [_i, _i64, _vp, _vp, _vp, _vp]),
    "pj_images_subtract": (_i, [_i, _i64, _vp, _vp, _vp, _vp]),
    "pj_symmetrize": (_i, [_i, _vp, _i64, _vp]),
    "pj_sq_distances": (_i, [_i, _i, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp]),
    "pj_gemm_saved_bytes": (_sz, [_i, _i, _i, _i, _i, _i]),
    "proj_gemm_save": (_i, [_vp, _i, _ch, _ch, _i, _i, _i, _vp, _i64, _vp, _i64, _f, _vp, _i64, _i, _vp, _sz, _vp,
                            _sz, _vp]),
    "pj_gemm_backward_saved_workspace_bytes": (_sz, [_i, _i, _i, _i, _i, _i]),
    "proj_gemm_backward_saved": (_i, [_vp, _i, _ch, _ch, _i, _i, _i, _vp, _sz, _vp, _i64, _vp, _i64, _vp, _i64, _i,
                                      _vp, _sz, _vp]),
    "proj_conv1d": (_i, [_vp, _i, _i, _i64, _vp, _i, _vp, _vp, _i, _vp, _sz, _vp]),
    "pj_conv1d_rate_workspace_bytes": (_sz, [_i64, _i, _i, _i, _i, _i]),
    "pj_conv1d_circular_workspace_bytes": (_sz, [_i64, _i, _i, _i, _i]),
    "proj_conv1d_circular": (_i, [_vp, _i, _i, _i64, _vp, _i, _vp, _vp, _i, _vp, _sz, _vp]),
    "pj_block_moments_workspace_bytes": (_sz, [_i64, _i64, _i]),
    "pj_block_moments": (_i, [_i, _i64, _i64, _vp, _i64, _vp, _vp, _sz, _vp]),
    "pj_basis_create_klt": (_i, [ctypes.POINTER(_vp), _i, _dp, _dp]),
    "pj_sym_eig": (_i, [_i, _dp, _dp, _dp]),
    "proj_conv1d_rate": (_i, [_vp, _i, _i, _i, _i64, _vp, _i, _vp, _vp, _i, _vp, _sz, _vp]),
    "pj_conv1d_fft_workspace_bytes": (_sz, [_i64, _i, _i, _i, _i]),
    "pj_conv1d_method_workspace_bytes": (_sz, [_i64, _i, _i, _i, _i, _i]),
    "proj_conv1d_method": (_i, [_vp, _i, _i, _i, _i64, _vp, _i, _vp, _vp, _i, _vp, _sz, _vp]),
    "proj_conv1d_fft": (_i, [_vp, _i, _i, _i64, _vp, _i, _vp, _vp, _i, _vp, _sz, _vp]),
}


def lib():
    """The loaded library; raises if libprojgemm.so has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                                   "`python -m paper_1411_2860_amd.build` (no fallback exists)")
            L = ctypes.CDLL(_LIB_PATH)
            for name, (res, args) in _SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def status_str(code: int) -> str:
    try:
        return lib().pj_status_str(code).decode()
    except Exception:  # the library itself may be what is missing
        return "?"


def _check(code: int, what: str):
    if code != 0:
        raise ProjGemmError(code, what)


def _prec(p) -> int:
    return PREC[p] if isinstance(p, str) else int(p)


def _stream(stream=None) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _ptr(t) -> int:
    return int(t.data_ptr())


class Basis:
    """An L x L projection basis C with D = C^{-1} (eq. (5)-(7)), built in FP64
    by the library and uploaded to the current device."""

    def __init__(self, kind: str = "dct2", L: int = 8, C=None):
        self._h = _vp()
        arr = None
        if C is not None:
            arr = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
            if arr.shape != (L, L):
                raise ValueError("custom basis must be L x L")
        cp = arr.ctypes.data_as(_dp) if arr is not None else None
        _check(lib().pj_basis_create(ctypes.byref(self._h), BASIS[kind], L, cp), "pj_basis_create")
        self.kind, self.L = kind, L

    @property
    def handle(self):
        return self._h

    def matrices(self):
        """FP64 (C, D) as stored by the library."""
        C = np.empty((self.L, self.L))
        D = np.empty((self.L, self.L))
        _check(lib().pj_basis_get(self._h, C.ctypes.data_as(_dp), D.ctypes.data_as(_dp)), "pj_basis_get")
        return C, D

    def close(self):
        if self._h and self._h.value:
            lib().pj_basis_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def block_moments(X, L: int, stream=None):
    """FP64 L x L second moments of the aligned L-blocks of the rows of the
    FP32 CUDA matrix X (pj_block_moments), as a CUDA float64 tensor."""
    import torch
    if X.dtype != torch.float32 or X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a 2-D float32 tensor with unit column stride")
    rows, K = X.shape
    M = torch.empty((L, L), dtype=torch.float64, device=X.device)
    ws = _byte_buffer(int(lib().pj_block_moments_workspace_bytes(rows, K, L)), X.device)
    _check(lib().pj_block_moments(L, rows, K, _ptr(X), X.stride(0), _ptr(M), _ptr(ws), ws.numel(), _stream(stream)),
           "pj_block_moments")
    return M


def klt_basis(M):
    """(Basis, eigenvalues) of the orthonormal eigenbasis of the symmetric
    positive semidefinite L x L matrix M (numpy array or tensor; pj_basis_create_klt)."""
    if hasattr(M, "detach"):
        M = M.detach().double().cpu().numpy()
    arr = np.ascontiguousarray(np.asarray(M, dtype=np.float64))
    L = arr.shape[0]
    if arr.shape != (L, L):
        raise ValueError("M must be square")
    b = Basis.__new__(Basis)
    b._h = _vp()
    eig = np.empty(L)
    _check(lib().pj_basis_create_klt(ctypes.byref(b._h), L, arr.ctypes.data_as(_dp), eig.ctypes.data_as(_dp)),
           "pj_basis_create_klt")
    b.kind, b.L = "klt", L
    return b, eig


def images_center(X, out=None, stream=None):
    """(mean, centred) of J images X (CUDA float32, J x m x n, contiguous):
    mean over the images and every image minus it (pj_images_center)."""
    import torch
    if X.dtype != torch.float32 or not X.is_contiguous():
        raise TypeError("X must be a contiguous float32 tensor")
    J = X.shape[0]
    mn = X[0].numel()
    mean = torch.empty(X.shape[1:], dtype=torch.float32, device=X.device)
    if out is None:
        out = torch.empty_like(X)
    _check(lib().pj_images_center(J, mn, _ptr(X), _ptr(mean), _ptr(out), _stream(stream)), "pj_images_center")
    return mean, out


def images_subtract(X, mean, out=None, stream=None):
    """X minus the image `mean` for T images X (CUDA float32, T x m x n,
    contiguous; pj_images_subtract)."""
    import torch
    if X.dtype != torch.float32 or not X.is_contiguous() or not mean.is_contiguous():
        raise TypeError("X and mean must be contiguous float32 tensors")
    if out is None:
        out = torch.empty_like(X)
    _check(lib().pj_images_subtract(X.shape[0], X[0].numel(), _ptr(X), _ptr(mean), _ptr(out), _stream(stream)),
           "pj_images_subtract")
    return out


def symmetrize(G, stream=None):
    """G <- (G + G^T) / 2 in place (CUDA float32 square matrix, pj_symmetrize)."""
    n = G.shape[0]
    if G.shape != (n, n) or G.stride(1) != 1:
        raise ValueError("G must be square with unit column stride")
    _check(lib().pj_symmetrize(n, _ptr(G), G.stride(0), _stream(stream)), "pj_symmetrize")
    return G


def sq_distances(F, Y, out=None, stream=None):
    """out[i, j] = ||F_i - Y_j||^2 for the rows of F (T x d) and Y (J x d),
    CUDA float32 (pj_sq_distances)."""
    import torch
    T, d = F.shape
    J, d2 = Y.shape
    if d2 != d or F.stride(1) != 1 or Y.stride(1) != 1:
        raise ValueError("F and Y need the same row length and unit column stride")
    if out is None:
        out = torch.empty((T, J), dtype=torch.float32, device=F.device)
    _check(lib().pj_sq_distances(T, J, d, _ptr(F), F.stride(0), _ptr(Y), Y.stride(0), _ptr(out), out.stride(0),
                                 _stream(stream)), "pj_sq_distances")
    return out


def sym_eig(A):
    """(w, V) of the symmetric matrix A (numpy or tensor, moved to the host):
    eigenvalues in decreasing order, unit eigenvectors as the columns of V
    (pj_sym_eig)."""
    if hasattr(A, "detach"):
        A = A.detach().double().cpu().numpy()
    a = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    n = a.shape[0]
    if a.shape != (n, n):
        raise ValueError("A must be square")
    w = np.empty(n)
    V = np.empty((n, n))
    _check(lib().pj_sym_eig(n, a.ctypes.data_as(_dp), w.ctypes.data_as(_dp), V.ctypes.data_as(_dp)), "pj_sym_eig")
    return w, V


def packed_bytes(rows: int, K: int, L: int, rmax: int, prec="f32") -> int:
    return int(lib().pj_packed_bytes(rows, K, L, rmax, _prec(prec)))


def gemm_workspace_bytes(M: int, W: int, K: int, L: int, r: int, prec="f32") -> int:
    return int(lib().pj_gemm_workspace_bytes(M, W, K, L, r, _prec(prec)))


def _byte_buffer(nbytes: int, device):
    import torch
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def gemm(A, B, r: int, basis: Basis, prec="f32", transA=False, transB=False, beta=0.0, out=None,
         workspace=None, stream=None):
    """R = A Q_{r,K} B (+ beta R).  A is M x K (K x M if transA), B is K x W
    (W x K if transB); row-major CUDA tensors of float32 (float64 for 'f64')."""
    import torch
    p = _prec(prec)
    if transA:
        K, M = A.shape
    else:
        M, K = A.shape
    if transB:
        W, K2 = B.shape
    else:
        K2, W = B.shape
    if K2 != K:
        raise ValueError(f"contraction mismatch {K} vs {K2}")
    dt = torch.float64 if p == PREC["f64"] else torch.float32
    if A.dtype != dt or B.dtype != dt:
        raise TypeError(f"A and B must be {dt}")
    if A.stride(1) != 1 or B.stride(1) != 1:
        raise ValueError("A and B need unit stride along their last dimension")
    if out is None:
        out = torch.empty((M, W), dtype=dt, device=A.device)
        if beta != 0.0:
            raise ValueError("beta != 0 needs `out`")
    need = gemm_workspace_bytes(M, W, K, basis.L, r, p)
    if workspace is None:
        workspace = _byte_buffer(need, A.device)
    _check(lib().proj_gemm(basis.handle, r, b"T" if transA else b"N", b"T" if transB else b"N", M, W, K,
                           _ptr(A), A.stride(0), _ptr(B), B.stride(0), float(beta), _ptr(out), out.stride(0), p,
                           _ptr(workspace), workspace.numel() * workspace.element_size(), _stream(stream)),
           "proj_gemm")
    return out


def gemm_noalloc(A, B, r: int, basis: Basis, out, prec="f32", transA=False, transB=False, beta=0.0, stream=None):
    """proj_gemm_noalloc: the same product as gemm() on the library's fixed
    per-device scratch, with no workspace; `out` (M x W) is the caller's."""
    p = _prec(prec)
    if transA:
        K, M = A.shape
    else:
        M, K = A.shape
    if transB:
        W, K2 = B.shape
    else:
        K2, W = B.shape
    if K2 != K:
        raise ValueError(f"contraction mismatch {K} vs {K2}")
    if A.stride(1) != 1 or B.stride(1) != 1 or out.stride(1) != 1:
        raise ValueError("A, B and out need unit stride along their last dimension")
    if tuple(out.shape) != (M, W):
        raise ValueError(f"out must be {M} x {W}")
    _check(lib().proj_gemm_noalloc(basis.handle, r, b"T" if transA else b"N", b"T" if transB else b"N", M, W, K,
                                   _ptr(A), A.stride(0), _ptr(B), B.stride(0), float(beta), _ptr(out),
                                   out.stride(0), p, _stream(stream)),
           "proj_gemm_noalloc")
    return out


def pack_a(A, rmax: int, basis: Basis, prec="f32", transA=False, out=None, stream=None):
    """Projects and packs the A side at rmax projections; returns a byte tensor."""
    p = _prec(prec)
    if transA:
        K, M = A.shape
    else:
        M, K = A.shape
    n = packed_bytes(M, K, basis.L, rmax, p)
    if out is None:
        out = _byte_buffer(n, A.device)
    _check(lib().pj_pack_a(basis.handle, rmax, b"T" if transA else b"N", M, K, _ptr(A), A.stride(0), p,
                           _ptr(out), out.numel(), _stream(stream)), "pj_pack_a")
    return out


def pack_b(B, rmax: int, basis: Basis, prec="f32", transB=False, out=None, stream=None):
    """Projects and packs the B side at rmax projections; returns a byte tensor."""
    p = _prec(prec)
    if transB:
        W, K = B.shape
    else:
        K, W = B.shape
    n = packed_bytes(W, K, basis.L, rmax, p)
    if out is None:
        out = _byte_buffer(n, B.device)
    _check(lib().pj_pack_b(basis.handle, rmax, b"T" if transB else b"N", W, K, _ptr(B), B.stride(0), p,
                           _ptr(out), out.numel(), _stream(stream)), "pj_pack_b")
    return out


def pack_ab(A, B, rmax: int, basis: Basis, prec="f32", transA=False, transB=False, out_a=None, out_b=None,
            stream=None):
    """Projects and packs both sides in one launch; returns (Ap, Bp)."""
    p = _prec(prec)
    M, K = (A.shape[1], A.shape[0]) if transA else tuple(A.shape)
    W = B.shape[0] if transB else B.shape[1]
    if out_a is None:
        out_a = _byte_buffer(packed_bytes(M, K, basis.L, rmax, p), A.device)
    if out_b is None:
        out_b = _byte_buffer(packed_bytes(W, K, basis.L, rmax, p), B.device)
    _check(lib().pj_pack_ab(basis.handle, rmax, b"T" if transA else b"N", b"T" if transB else b"N", M, W, K,
                            _ptr(A), A.stride(0), _ptr(B), B.stride(0), p, _ptr(out_a), out_a.numel(),
                            _ptr(out_b), out_b.numel(), _stream(stream)), "pj_pack_ab")
    return out_a, out_b


def tile_configs(prec="f32"):
    """[(tile_m, tile_n)] of the reduced-contraction tile configurations."""
    n = lib().pj_gemm_tile_configs(_prec(prec), None, None, 0)
    tm = (_i * n)()
    tn = (_i * n)()
    lib().pj_gemm_tile_configs(_prec(prec), tm, tn, n)
    return list(zip(tm, tn))


def gemm_packed(Ap, Bp, r: int, M: int, W: int, K: int, L: int, rmax_a: int, rmax_b: int, prec="f32",
                beta=0.0, out=None, tile_cfg=-1, stream=None):
    """R = sum_{l<r} A_c^{(l)} B_d^{(l)} (+ beta R) from packed operands."""
    import torch
    p = _prec(prec)
    dt = torch.float64 if p == PREC["f64"] else torch.float32
    if out is None:
        out = torch.empty((M, W), dtype=dt, device=Ap.device)
    _check(lib().pj_gemm_packed(r, M, W, K, L, p, _ptr(Ap), rmax_a, Ap.numel(), _ptr(Bp), rmax_b, Bp.numel(),
                                float(beta), _ptr(out), out.stride(0), int(tile_cfg), _stream(stream)),
           "pj_gemm_packed")
    return out


_RATES = {"full": 0, "block": 1}


def conv1d_workspace_bytes(W: int, N: int, L: int, r: int, prec="f32", rate="full") -> int:
    return int(lib().pj_conv1d_rate_workspace_bytes(W, N, L, r, _RATES[rate], _prec(prec)))


def conv1d(s, k, r: int, basis: Basis, mode="xcorr", prec="f32", out=None, workspace=None, stream=None, rate="full"):
    """Projected valid cross-correlation (mode 'xcorr') or convolution
    ('conv') of the 1-D float32 CUDA tensors s (W) and k (N): W - N + 1 outputs.
    rate 'full' computes every output; 'block' computes the outputs at m = aL
    and interpolates the others linearly (proj_conv1d_rate)."""
    import torch
    Wn, N = s.numel(), k.numel()
    if s.dtype != torch.float32 or k.dtype != torch.float32:
        raise TypeError("s and k must be float32")
    if not (s.is_contiguous() and k.is_contiguous()):
        raise ValueError("s and k must be contiguous")
    if out is None:
        out = torch.empty(max(Wn - N + 1, 1), dtype=torch.float32, device=s.device)
    need = conv1d_workspace_bytes(Wn, N, basis.L, r, prec, rate)
    if workspace is None:
        workspace = _byte_buffer(need, s.device)
    _check(lib().proj_conv1d_rate(basis.handle, r, {"xcorr": 0, "conv": 1}[mode], _RATES[rate], Wn, _ptr(s), N,
                                  _ptr(k), _ptr(out), _prec(prec), _ptr(workspace), workspace.numel(),
                                  _stream(stream)), "proj_conv1d_rate")
    return out


METHODS = {"auto": 0, "direct": 1, "fft": 2}


def conv1d_method_workspace_bytes(W: int, N: int, L: int, r: int, method="auto", prec="f32") -> int:
    return int(lib().pj_conv1d_method_workspace_bytes(W, N, L, r, METHODS[method], _prec(prec)))


def conv1d_method(s, k, r: int, basis: Basis, method="auto", mode="xcorr", prec="f32", out=None, workspace=None,
                  stream=None):
    """conv1d (full rate) with the realisation chosen: 'auto' (the library's
    cost model), 'direct' or 'fft' (proj_conv1d_method)."""
    import torch
    Wn, N = s.numel(), k.numel()
    if s.dtype != torch.float32 or k.dtype != torch.float32:
        raise TypeError("s and k must be float32")
    if not (s.is_contiguous() and k.is_contiguous()):
        raise ValueError("s and k must be contiguous")
    if out is None:
        out = torch.empty(max(Wn - N + 1, 1), dtype=torch.float32, device=s.device)
    if workspace is None:
        workspace = _byte_buffer(conv1d_method_workspace_bytes(Wn, N, basis.L, r, method, prec), s.device)
    _check(lib().proj_conv1d_method(basis.handle, r, {"xcorr": 0, "conv": 1}[mode], METHODS[method], Wn, _ptr(s), N,
                                    _ptr(k), _ptr(out), _prec(prec), _ptr(workspace), workspace.numel(),
                                    _stream(stream)), "proj_conv1d_method")
    return out


def conv1d_fft_workspace_bytes(W: int, N: int, L: int, r: int, prec="f32") -> int:
    return int(lib().pj_conv1d_fft_workspace_bytes(W, N, L, r, _prec(prec)))


def conv1d_fft(s, k, r: int, basis: Basis, mode="xcorr", prec="f32", out=None, workspace=None, stream=None):
    """conv1d (full rate) through FFTs of the projected signal segments and
    the projected kernel phases (proj_conv1d_fft)."""
    import torch
    Wn, N = s.numel(), k.numel()
    if s.dtype != torch.float32 or k.dtype != torch.float32:
        raise TypeError("s and k must be float32")
    if not (s.is_contiguous() and k.is_contiguous()):
        raise ValueError("s and k must be contiguous")
    if out is None:
        out = torch.empty(max(Wn - N + 1, 1), dtype=torch.float32, device=s.device)
    if workspace is None:
        workspace = _byte_buffer(conv1d_fft_workspace_bytes(Wn, N, basis.L, r, prec), s.device)
    _check(lib().proj_conv1d_fft(basis.handle, r, {"xcorr": 0, "conv": 1}[mode], Wn, _ptr(s), N, _ptr(k), _ptr(out),
                                 _prec(prec), _ptr(workspace), workspace.numel(), _stream(stream)), "proj_conv1d_fft")
    return out


def conv1d_circular(s, k, r: int, basis: Basis, mode="xcorr", prec="f32", out=None, workspace=None, stream=None):
    """Projected circular cross-correlation / convolution of the periodic
    float32 CUDA signal s (period W, a multiple of L) with k (N <= W): W
    outputs (proj_conv1d_circular)."""
    import torch
    Wn, N = s.numel(), k.numel()
    if s.dtype != torch.float32 or k.dtype != torch.float32:
        raise TypeError("s and k must be float32")
    if not (s.is_contiguous() and k.is_contiguous()):
        raise ValueError("s and k must be contiguous")
    if out is None:
        out = torch.empty(Wn, dtype=torch.float32, device=s.device)
    if workspace is None:
        workspace = _byte_buffer(int(lib().pj_conv1d_circular_workspace_bytes(Wn, N, basis.L, r, _prec(prec))),
                                 s.device)
    _check(lib().proj_conv1d_circular(basis.handle, r, {"xcorr": 0, "conv": 1}[mode], Wn, _ptr(s), N, _ptr(k),
                                      _ptr(out), _prec(prec), _ptr(workspace), workspace.numel(), _stream(stream)),
           "proj_conv1d_circular")
    return out


class GemmDesc(ctypes.Structure):
    """pj_gemm_desc: one problem of a batched call."""
    _fields_ = [("M", _i), ("W", _i), ("K", _i), ("transA", _ch), ("transB", _ch),
                ("A", _vp), ("lda", _i64), ("B", _vp), ("ldb", _i64), ("R", _vp), ("ldr", _i64)]


def _descs(As, Bs, Rs, transA=False, transB=False):
    n = len(As)
    arr = (GemmDesc * n)()
    for i, (A, B, R) in enumerate(zip(As, Bs, Rs)):
        M, K = (A.shape[1], A.shape[0]) if transA else tuple(A.shape)
        W = B.shape[0] if transB else B.shape[1]
        arr[i] = GemmDesc(M, W, K, b"T" if transA else b"N", b"T" if transB else b"N", _ptr(A), A.stride(0),
                          _ptr(B), B.stride(0), _ptr(R), R.stride(0))
    return arr


def _small_arr(small, n):
    if small is None:
        return None
    if len(small) != n:
        raise ValueError(f"small needs one flag per problem ({n})")
    return (ctypes.c_ubyte * n)(*[1 if f else 0 for f in small])


def gemm_batched_workspace_bytes(descs, L: int, r: int, prec="f32", tile_cfg=-1, small=None) -> int:
    sm = _small_arr(small, len(descs))
    if sm is None:
        return int(lib().pj_gemm_batched_workspace_bytes(len(descs), ctypes.cast(descs, _vp), L, r, _prec(prec),
                                                         int(tile_cfg)))
    return int(lib().pj_gemm_batched_tiles_workspace_bytes(len(descs), ctypes.cast(descs, _vp), ctypes.cast(sm, _vp),
                                                           L, r, _prec(prec), int(tile_cfg)))


def gemm_batched(As, Bs, r: int, basis: Basis, prec="bf16", transA=False, transB=False, outs=None, beta=0.0,
                 tile_cfg=-1, workspace=None, stream=None, small=None):
    """R_i = A_i Q_{r,K_i} B_i for every problem i, in grouped pack launches
    (one per operand staging mode) and one persistent GEMM launch.  `small`
    (one flag per problem) picks each problem's tile: the configuration's, or
    its small one; None lets the library choose.  Returns the outputs."""
    import torch
    if outs is None:
        outs = []
        for A, B in zip(As, Bs):
            M = A.shape[1] if transA else A.shape[0]
            W = B.shape[0] if transB else B.shape[1]
            outs.append(torch.empty((M, W), dtype=torch.float32, device=A.device))
    descs = _descs(As, Bs, outs, transA, transB)
    need = gemm_batched_workspace_bytes(descs, basis.L, r, prec, tile_cfg, small)
    if need == 0:
        raise ProjGemmError(-1, "pj_gemm_batched_workspace_bytes")
    if workspace is None:
        workspace = _byte_buffer(need, As[0].device)
    sm = _small_arr(small, len(As))
    if sm is None:
        _check(lib().proj_gemm_batched(basis.handle, r, len(As), ctypes.cast(descs, _vp), float(beta), _prec(prec),
                                       int(tile_cfg), _ptr(workspace), workspace.numel(), _stream(stream)),
               "proj_gemm_batched")
    else:
        _check(lib().proj_gemm_batched_tiles(basis.handle, r, len(As), ctypes.cast(descs, _vp), ctypes.cast(sm, _vp),
                                             float(beta), _prec(prec), int(tile_cfg), _ptr(workspace),
                                             workspace.numel(), _stream(stream)),
               "proj_gemm_batched_tiles")
    return outs


def gemm_backward(A, B, dR, r: int, basis: Basis, prec="f32", transA=False, transB=False, need_dA=True,
                  need_dB=True, workspace=None, stream=None):
    """(dA, dB) of R = A Q_{r,K} B for upstream dR; dA has A's layout, dB B's."""
    import torch
    p = _prec(prec)
    M, K = (A.shape[1], A.shape[0]) if transA else tuple(A.shape)
    W = B.shape[0] if transB else B.shape[1]
    dA = torch.empty_like(A) if need_dA else None
    dB = torch.empty_like(B) if need_dB else None
    if dR.stride(1) != 1:
        dR = dR.contiguous()
    need = int(lib().pj_gemm_backward_workspace_bytes(M, W, K, basis.L, r, p))
    if workspace is None:
        workspace = _byte_buffer(need, A.device)
    _check(lib().proj_gemm_backward(basis.handle, r, b"T" if transA else b"N", b"T" if transB else b"N", M, W, K,
                                    _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(dR), dR.stride(0),
                                    _ptr(dA) if dA is not None else None, dA.stride(0) if dA is not None else 1,
                                    _ptr(dB) if dB is not None else None, dB.stride(0) if dB is not None else 1,
                                    p, _ptr(workspace), workspace.numel(), _stream(stream)), "proj_gemm_backward")
    return dA, dB


def gemm_saved_bytes(M: int, W: int, K: int, L: int, r: int, prec="f32") -> int:
    return int(lib().pj_gemm_saved_bytes(M, W, K, L, r, _prec(prec)))


def gemm_save(A, B, r: int, basis: Basis, prec="f32", transA=False, transB=False, out=None, workspace=None,
              saved=None, stream=None):
    """(R, saved): gemm() that also keeps the plain projections of A and B
    (a byte tensor) for gemm_backward_saved."""
    import torch
    p = _prec(prec)
    M, K = (A.shape[1], A.shape[0]) if transA else tuple(A.shape)
    K2, W = (B.shape[1], B.shape[0]) if transB else tuple(B.shape)
    if K2 != K:
        raise ValueError(f"contraction mismatch {K} vs {K2}")
    dt = torch.float64 if p == PREC["f64"] else torch.float32
    if A.dtype != dt or B.dtype != dt:
        raise TypeError(f"A and B must be {dt}")
    if A.stride(1) != 1 or B.stride(1) != 1:
        raise ValueError("A and B need unit stride along their last dimension")
    if out is None:
        out = torch.empty((M, W), dtype=dt, device=A.device)
    if workspace is None:
        workspace = _byte_buffer(gemm_workspace_bytes(M, W, K, basis.L, r, p), A.device)
    if saved is None:
        saved = _byte_buffer(gemm_saved_bytes(M, W, K, basis.L, r, p), A.device)
    _check(lib().proj_gemm_save(basis.handle, r, b"T" if transA else b"N", b"T" if transB else b"N", M, W, K,
                                _ptr(A), A.stride(0), _ptr(B), B.stride(0), 0.0, _ptr(out), out.stride(0), p,
                                _ptr(workspace), workspace.numel(), _ptr(saved), saved.numel(), _stream(stream)),
           "proj_gemm_save")
    return out, saved


def gemm_backward_saved(saved, dR, r: int, basis: Basis, M: int, W: int, K: int, prec="f32", transA=False,
                        transB=False, need_dA=True, need_dB=True, dtype=None, workspace=None, stream=None):
    """(dA, dB) from the projections gemm_save kept; dA has the layout of A
    (M x K, K x M if transA), dB that of B (K x W, W x K if transB)."""
    import torch
    p = _prec(prec)
    dt = dtype or (torch.float64 if p == PREC["f64"] else torch.float32)
    dev = dR.device
    dA = torch.empty((K, M) if transA else (M, K), dtype=dt, device=dev) if need_dA else None
    dB = torch.empty((W, K) if transB else (K, W), dtype=dt, device=dev) if need_dB else None
    if dR.stride(1) != 1:
        dR = dR.contiguous()
    need = int(lib().pj_gemm_backward_saved_workspace_bytes(M, W, K, basis.L, r, p))
    if workspace is None:
        workspace = _byte_buffer(need, dev)
    _check(lib().proj_gemm_backward_saved(basis.handle, r, b"T" if transA else b"N", b"T" if transB else b"N", M, W,
                                          K, _ptr(saved), saved.numel(), _ptr(dR), dR.stride(0),
                                          _ptr(dA) if dA is not None else None, dA.stride(0) if dA is not None else 1,
                                          _ptr(dB) if dB is not None else None, dB.stride(0) if dB is not None else 1,
                                          p, _ptr(workspace), workspace.numel(), _stream(stream)),
           "proj_gemm_backward_saved")
    return dA, dB
