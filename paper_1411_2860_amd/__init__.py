"""Projection-based precision-scalable GEMM and 1-D cross-correlation for
AMD MI355X (gfx950).

Method: Anam, Whatmough, Andreopoulos, "Precision-Energy-Throughput Scaling of
Generic Matrix Multiplication and Convolution Kernels via Linear Projections",
IEEE TCSVT 24(11), 2014.  Input blocks of L consecutive contraction indices are
projected onto an L x L basis C (B side: D = C^{-1}); GEMM or cross-correlation
then runs on the first r projections only and the partial products are
accumulated, so r trades precision for throughput.

The compute path is the C-ABI library ``libprojgemm.so`` (HIP kernels for
gfx950, declared in include/projgemm.h).  The submodule ``projgemm`` is a thin
ctypes binding; it is imported lazily so that ``inputs`` (synthetic data only)
can be used without the library.
"""
import importlib

__all__ = ["inputs", "projgemm", "autograd"]


def __getattr__(name):
    if name in ("projgemm", "autograd", "inputs"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
