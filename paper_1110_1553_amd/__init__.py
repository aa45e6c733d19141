"""Tiled hierarchical Householder QR on AMD MI355X (gfx950).

The product path is the HIP library ``libhqr.so`` (C ABI in ``include/hqr.h``);
this package only marshals arguments to it:

* :func:`factor` -- QR of a column-major float64 device matrix through one
  persistent GPU launch driven by a hierarchical elimination tree;
* :func:`apply_qt`, :func:`apply_q` -- B <- Q^T B and B <- Q B with a
  finished factorization; :func:`lstsq` -- least squares through both;
* :func:`lstsq_ir` -- least squares with an FP32 factorization refined to
  FP64 accuracy (augmented-system iterative refinement);
* :func:`lstsq_batched`, :class:`BatchedLstsq` -- many independent small
  least-squares problems (or factorizations) in one persistent launch;
* :func:`elimlist`, :func:`validate`, :func:`dag_stats` -- the elimination
  lists and task graphs the library builds on the host.

PyTorch supplies device memory and streams only.
"""
from . import _lib
from ._lib import (BINARY, CHAIN, FIBONACCI, FLAT, GREEDY, OPS, Exec, Factors, HQRError, Params,
                   apply_workspace_size, dag_stats, elimlist, lstsq_workspace_size, make_exec, make_params,
                   release_plans, validate, version, workspace_size)

__all__ = ["FLAT", "BINARY", "GREEDY", "FIBONACCI", "CHAIN", "OPS", "Params", "Exec", "Factors", "HQRError",
           "make_params",
           "make_exec", "elimlist", "validate", "dag_stats", "workspace_size", "apply_workspace_size",
           "lstsq_workspace_size", "factor",
           "apply_qt", "apply_q", "solve", "lstsq", "factors_run", "lstsq_ir", "lstsq_batched", "BatchedLstsq", "colmajor", "r_of", "Workspace", "ApplyWorkspace", "status",
           "release_plans", "version"]


def colmajor(t):
    """A column-major copy of a 2-D tensor: shape (M, N), strides (1, M)."""
    return t.t().contiguous().t()


class Workspace:
    """Device workspace for :func:`factor` (a torch uint8 buffer); with
    ``nrhs`` > 0 the larger one of :func:`lstsq`; with ``f32`` the one of a
    float32 factorization."""

    def __init__(self, M, N, params, device="cuda", nrhs=0, f32=False):
        import torch

        if f32:
            self.bytes = _lib.workspace_size_f32(M, N, params)
        else:
            self.bytes = lstsq_workspace_size(M, N, nrhs, params) if nrhs > 0 else workspace_size(M, N, params)
        self.buf = torch.empty(self.bytes, dtype=torch.uint8, device=device)

    @property
    def ptr(self):
        return self.buf.data_ptr()


class ApplyWorkspace:
    """Device workspace for :func:`apply_qt` and :func:`apply_q`."""

    def __init__(self, M, nrhs, params, device="cuda"):
        import torch

        self.bytes = apply_workspace_size(M, nrhs, params)
        self.buf = torch.empty(self.bytes, dtype=torch.uint8, device=device)

    @property
    def ptr(self):
        return self.buf.data_ptr()


def _colmajor_args(X, name):
    import torch

    if X.dtype != torch.float64 or not X.is_cuda or X.dim() != 2:
        raise ValueError("%s must be a 2-D float64 CUDA tensor" % name)
    if X.stride(0) != 1:
        raise ValueError("%s must be column-major (stride(0) == 1); use colmajor()" % name)
    M, N = X.shape
    return M, N, (X.stride(1) if N > 1 else max(M, 1))


def _device_status(work, s, what, timeout_s=0.0):
    st, info = _lib.status(work.ptr, s.cuda_stream, timeout_s=timeout_s, detail=True)
    if st != 0:
        err = HQRError(what + " (device)", st)
        err.detail = info
        raise err
    return st


def factor(A, params, exec_=None, work=None, stream=None, check=True, timeout_s=0.0, handle=False):
    """In-place QR of the column-major float64 (or float32: FP32 tile
    kernels) CUDA tensor ``A`` (M x N, strides (1, lda)).  Returns the
    workspace (it holds the T factors), or (workspace, :class:`Factors`)
    with ``handle``."""
    import torch

    if A.dtype not in (torch.float64, torch.float32) or not A.is_cuda or A.dim() != 2:
        raise ValueError("A must be a 2-D float64 or float32 CUDA tensor")
    f32 = A.dtype == torch.float32
    M, N = A.shape
    if A.stride(0) != 1:
        raise ValueError("A must be column-major (stride(0) == 1); use colmajor()")
    lda = A.stride(1) if N > 1 else max(M, 1)
    if work is None:
        work = Workspace(M, N, params, device=A.device, f32=f32)
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    fn = _lib.factor_f32_ptr if f32 else _lib.factor_ptr
    fac = fn(A.data_ptr(), M, N, lda, params, exec_, work.ptr, work.bytes, s.cuda_stream, handle=handle)
    if check:
        st, info = _lib.status(work.ptr, s.cuda_stream, timeout_s=timeout_s, detail=True)
        if st != 0:
            err = HQRError("hqr_factor (device)", st)
            err.detail = info
            raise RuntimeError("%s; task %d waited on counter %d for %d, last saw %d" % ((err,) + tuple(info)))
    return (work, fac) if handle else work


def _apply(trans, B, M, N, params, work, exec_, bwork, stream, check):
    import torch

    MB, nrhs, ldb = _colmajor_args(B, "B")
    if MB != M:
        raise ValueError("B must have M = %d rows" % M)
    if bwork is None:
        bwork = ApplyWorkspace(M, nrhs, params, device=B.device)
    s = stream if stream is not None else torch.cuda.current_stream(B.device)
    _lib.apply_ptr(trans, M, N, params, exec_, work.ptr, work.bytes, B.data_ptr(), ldb, nrhs, bwork.ptr, bwork.bytes,
                   s.cuda_stream)
    if check:
        _device_status(bwork, s, "hqr_apply_qt" if trans else "hqr_apply_q")
    return bwork


def apply_qt(B, M, N, params, work, exec_=None, bwork=None, stream=None, check=True):
    """B <- Q^T B in place (B column-major M x nrhs) with the factorization
    of an M x N matrix held in ``work`` (returned by :func:`factor`)."""
    return _apply(True, B, M, N, params, work, exec_, bwork, stream, check)


def apply_q(B, M, N, params, work, exec_=None, bwork=None, stream=None, check=True):
    """B <- Q B in place; see :func:`apply_qt`."""
    return _apply(False, B, M, N, params, work, exec_, bwork, stream, check)


def solve(B, M, N, params, work, exec_=None, bwork=None, stream=None, check=True):
    """Least squares with the finished factorization of an M x N matrix held
    in ``work``: B (column-major M x nrhs) is overwritten by x in its first N
    rows and the residual components of Q^T B below (hqr_solve)."""
    import torch

    MB, nrhs, ldb = _colmajor_args(B, "B")
    if MB != M:
        raise ValueError("B must have M = %d rows" % M)
    if bwork is None:
        bwork = ApplyWorkspace(M, nrhs, params, device=B.device)
    s = stream if stream is not None else torch.cuda.current_stream(B.device)
    _lib.solve_ptr(M, N, params, exec_, work.ptr, work.bytes, B.data_ptr(), ldb, nrhs, bwork.ptr, bwork.bytes,
                   s.cuda_stream)
    if check:
        _device_status(bwork, s, "hqr_solve")
    return bwork


def lstsq(A, B, params, exec_=None, work=None, stream=None, check=True, handle=False):
    """Least squares min ||A X - B|| in place: A (M x N) is overwritten by its
    factorization, B (M x nrhs) by X in its first N rows and the residual
    components of Q^T B below.  Returns the workspace (it also holds the
    factors for :func:`apply_qt`), or (workspace, :class:`Factors`) with
    ``handle``."""
    import torch

    M, N, lda = _colmajor_args(A, "A")
    MB, nrhs, ldb = _colmajor_args(B, "B")
    if MB != M:
        raise ValueError("B must have M = %d rows" % M)
    if work is None:
        work = Workspace(M, N, params, device=A.device, nrhs=nrhs)
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    fac = _lib.lstsq_ptr(A.data_ptr(), M, N, lda, B.data_ptr(), ldb, nrhs, params, exec_, work.ptr, work.bytes,
                         s.cuda_stream, handle=handle)
    if check:
        _device_status(work, s, "hqr_lstsq")
    return (work, fac) if handle else work


class _Buf:
    """A device byte buffer with the ``ptr``/``bytes`` of a workspace."""

    def __init__(self, nbytes, device):
        import torch

        self.bytes = nbytes
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)

    @property
    def ptr(self):
        return self.buf.data_ptr()


def factors_run(fac, op, B, exec_=None, bwork=None, stream=None, check=True):
    """B <- Q^T B (op "apply_qt"), Q B ("apply_q") or the least-squares
    solution ("solve") with the factorization of the handle ``fac``
    (hqr_factors_*); B is a column-major float64 CUDA tensor with M rows."""
    import torch

    M = fac.query()[0]
    MB, nrhs, ldb = _colmajor_args(B, "B")
    if MB != M:
        raise ValueError("B must have M = %d rows" % M)
    if bwork is None:
        bwork = _Buf(fac.apply_workspace_size(nrhs), B.device)
    s = stream if stream is not None else torch.cuda.current_stream(B.device)
    getattr(fac, op)(B.data_ptr(), ldb, nrhs, bwork.ptr, bwork.bytes, s.cuda_stream, exec_)
    if check:
        _device_status(bwork, s, "hqr_factors_" + op)
    return bwork


def lstsq_ir(A, b, params, exec_=None, max_iter=30, tol=1e-12, stream=None, residual=False):
    """min ||A x - b|| for a column-major float64 CUDA matrix A (M x N) and
    vector b (M): FP32 factorization plus FP64 refinement (hqr_lstsq_ir).
    A and b are not modified.  Returns (x, info) or (x, r, info) with
    ``residual``; info has iterations, converged, eta and history."""
    import torch

    M, N, lda = _colmajor_args(A, "A")
    b = b.reshape(-1)
    if b.dtype != torch.float64 or not b.is_cuda or b.numel() != M or not b.is_contiguous():
        raise ValueError("b must be a contiguous float64 CUDA vector of length M")
    x = torch.empty(N, dtype=torch.float64, device=A.device)
    r = torch.empty(M, dtype=torch.float64, device=A.device) if residual else None
    nbytes = _lib.lstsq_ir_workspace_size(M, N, params)
    work = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    info = _lib.lstsq_ir_ptr(A.data_ptr(), M, N, lda, b.data_ptr(), x.data_ptr(), r.data_ptr() if residual else 0,
                             params, exec_, max_iter, tol, work.data_ptr(), nbytes, s.cuda_stream)
    out = {"iterations": info.iterations, "converged": bool(info.converged), "eta": info.eta,
           "history": list(info.history[: info.history_len])}
    return (x, r, out) if residual else (x, out)


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


class BatchedLstsq:
    """Independent least-squares problems min ||A_q X_q - B_q|| (or, with
    ``Bs`` None, factorizations of the A_q) on fixed device buffers, run as
    one batch: planned and bound to the buffers once, then :meth:`run` any
    number of times.  ``run`` enqueues kernel launches only (it can be
    captured in a graph); every run starts again from the current contents
    of the A_q and B_q and overwrites them as :func:`lstsq` does."""

    def __init__(self, As, Bs, params, exec_=None, stream=None):
        import torch

        shapes = [_colmajor_args(A, "A[%d]" % q) for q, A in enumerate(As)]
        rhs = [_colmajor_args(B, "B[%d]" % q) for q, B in enumerate(Bs)] if Bs is not None else None
        if rhs is not None:
            if len(rhs) != len(shapes):
                raise ValueError("As and Bs differ in length")
            for q, (sa, sb) in enumerate(zip(shapes, rhs)):
                if sa[0] != sb[0]:
                    raise ValueError("B[%d] must have %d rows" % (q, sa[0]))
        self.As, self.Bs = list(As), (list(Bs) if Bs is not None else None)
        M = [sh[0] for sh in shapes]
        N = [sh[1] for sh in shapes]
        nrhs = [sb[1] for sb in rhs] if rhs is not None else None
        self.batch = _lib.Batch(M, N, nrhs, params, exec_)
        self.bytes = self.batch.workspace_size()
        device = As[0].device
        self.work = torch.empty(self.bytes, dtype=torch.uint8, device=device)
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self.batch.bind([A.data_ptr() for A in As], [sh[2] for sh in shapes],
                        [B.data_ptr() for B in Bs] if Bs is not None else None,
                        [sb[2] for sb in rhs] if rhs is not None else None,
                        self.work.data_ptr(), self.bytes, s.cuda_stream)

    def run(self, stream=None):
        import torch

        s = stream if stream is not None else torch.cuda.current_stream(self.work.device)
        self.batch.run(self.work.data_ptr(), self.bytes, s.cuda_stream)

    def status(self, stream=None, timeout_s=0.0):
        """(status word, per problem the first zero diagonal index of R or -1)."""
        import torch

        s = stream if stream is not None else torch.cuda.current_stream(self.work.device)
        return self.batch.status(self.work.data_ptr(), s.cuda_stream, timeout_s)


def lstsq_batched(As, Bs, params, exec_=None, stream=None, check=True):
    """Solves every problem of a batch in place (see :class:`BatchedLstsq`)
    and returns, per problem, the index of the first zero diagonal entry of
    R or -1.  With ``check`` a watchdog abort raises HQRError."""
    solver = BatchedLstsq(As, Bs, params, exec_, stream)
    solver.run(stream)
    st, first_zero = solver.status(stream)
    if check and st not in (0, _lib.ERR_SINGULAR):
        raise HQRError("hqr_batch_run (device)", st)
    return first_zero
