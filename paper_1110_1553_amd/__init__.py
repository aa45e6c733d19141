"""Tiled hierarchical Householder QR on AMD MI355X (gfx950).

The product path is the HIP library ``libhqr.so`` (C ABI in ``include/hqr.h``);
this package only marshals arguments to it:

* :func:`factor` -- QR of a column-major float64 device matrix through one
  persistent GPU launch driven by a hierarchical elimination tree;
* :func:`elimlist`, :func:`validate`, :func:`dag_stats` -- the elimination
  lists and task graphs the library builds on the host.

PyTorch supplies device memory and streams only.
"""
from . import _lib
from ._lib import (BINARY, CHAIN, FIBONACCI, FLAT, GREEDY, OPS, Exec, HQRError, Params, dag_stats, elimlist,
                   make_exec, make_params, release_plans, validate, version, workspace_size)

__all__ = ["FLAT", "BINARY", "GREEDY", "FIBONACCI", "CHAIN", "OPS", "Params", "Exec", "HQRError", "make_params",
           "make_exec", "elimlist", "validate", "dag_stats", "workspace_size", "factor", "colmajor", "r_of",
           "Workspace", "status", "release_plans", "version"]


def colmajor(t):
    """A column-major copy of a 2-D tensor: shape (M, N), strides (1, M)."""
    return t.t().contiguous().t()


class Workspace:
    """Device workspace for :func:`factor` (a torch uint8 buffer)."""

    def __init__(self, M, N, params, device="cuda"):
        import torch

        self.bytes = workspace_size(M, N, params)
        self.buf = torch.empty(self.bytes, dtype=torch.uint8, device=device)

    @property
    def ptr(self):
        return self.buf.data_ptr()


def factor(A, params, exec_=None, work=None, stream=None, check=True, timeout_s=0.0):
    """In-place QR of the column-major float64 CUDA tensor ``A`` (M x N,
    strides (1, lda)).  Returns the workspace (it holds the T factors)."""
    import torch

    if A.dtype != torch.float64 or not A.is_cuda or A.dim() != 2:
        raise ValueError("A must be a 2-D float64 CUDA tensor")
    M, N = A.shape
    if A.stride(0) != 1:
        raise ValueError("A must be column-major (stride(0) == 1); use colmajor()")
    lda = A.stride(1) if N > 1 else max(M, 1)
    if work is None:
        work = Workspace(M, N, params, device=A.device)
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    _lib.factor_ptr(A.data_ptr(), M, N, lda, params, exec_, work.ptr, work.bytes, s.cuda_stream)
    if check:
        st, info = _lib.status(work.ptr, s.cuda_stream, timeout_s=timeout_s, detail=True)
        if st != 0:
            err = HQRError("hqr_factor (device)", st)
            err.detail = info
            raise RuntimeError("%s; task %d waited on counter %d for %d, last saw %d" % ((err,) + tuple(info)))
    return work


def status(work, stream=None):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return _lib.status(work.ptr, s.cuda_stream)


def r_of(A):
    """Upper-triangular R (N x N) from a factored column-major tensor, on the host as numpy."""
    import numpy as np

    M, N = A.shape
    Rt = A[:N, :N].detach().cpu().numpy()
    return np.triu(Rt)
