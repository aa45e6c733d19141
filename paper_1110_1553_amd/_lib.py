"""ctypes binding of ``libhqr.so`` (argument marshalling only).

Every function here forwards to the C ABI declared in ``include/hqr.h``;
no step of the factorization runs in Python.  Importing this module fails
loudly when the HIP library has not been built.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhqr.so")

FLAT, BINARY, GREEDY, FIBONACCI, CHAIN = 0, 1, 2, 3, 4
TREES = {"flat": FLAT, "binary": BINARY, "greedy": GREEDY, "fibonacci": FIBONACCI, "chain": CHAIN}
OPS = ("GEQRT", "UNMQR", "TSQRT", "TSMQR", "TTQRT", "TTMQR")

ERR_WATCHDOG = 2
ERR_TIMEOUT = 7
ERR_SINGULAR = 8
ERR_FACTORS = 9
PREC_FP64, PREC_FP32, PREC_BF16 = 0, 1, 2
PRECISIONS = {"fp64": PREC_FP64, "fp32": PREC_FP32, "bf16": PREC_BF16}


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("nb", "ib", "p", "a", "low", "high", "coupling", "domino", "precision")]


class Exec(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int32), ("order", ctypes.c_int32), ("spin_limit", ctypes.c_int64),
                ("ev_begin", ctypes.c_void_p), ("ev_end", ctypes.c_void_p)]


class Elim(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("k", "victim", "killer", "kind", "level", "round")]


class DagInfo(ctypes.Structure):
    _fields_ = [("eliminations", ctypes.c_int64), ("tasks", ctypes.c_int64), ("count", ctypes.c_int64 * 6),
                ("weight", ctypes.c_int64), ("critical_path", ctypes.c_int64), ("device_tasks", ctypes.c_int64)]


class IrInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("eta", ctypes.c_double),
                ("history", ctypes.c_double * 32), ("history_len", ctypes.c_int32)]


TASK_DTYPE = np.dtype([("op", "u1"), ("chunk", "u1"), ("row", "<u2"), ("killer", "<u2"), ("k", "<u2"),
                       ("j", "<u2"), ("pad", "<u2"), ("v", "<u4", (3,))])

EXPORTS = ("hqr_elimlist", "hqr_plan_tasks", "hqr_elimlist_validate", "hqr_dag_stats", "hqr_workspace_size", "hqr_factor",
           "hqr_workspace_size_f32", "hqr_factor_f32", "hqr_lstsq_ir_workspace_size", "hqr_lstsq_ir",
           "hqr_apply_workspace_size", "hqr_apply_qt", "hqr_apply_q", "hqr_lstsq_workspace_size", "hqr_lstsq",
           "hqr_status", "hqr_status_ex", "hqr_release_plans", "hqr_strerror", "hqr_last_error", "hqr_timeline", "hqr_version",
           "hqr_batch_create", "hqr_batch_workspace_size", "hqr_batch_num_tasks", "hqr_batch_bind", "hqr_batch_run",
           "hqr_batch_status", "hqr_batch_publish_status", "hqr_batch_destroy", "hqr_lstsq_batched",
           "hqr_lstsq_batched_workspace_size", "hqr_solve", "hqr_batch_export_factors", "hqr_batch_export_all",
           "hqr_factors_apply_workspace_size", "hqr_factors_apply_qt", "hqr_factors_apply_q", "hqr_factors_solve",
           "hqr_factors_query", "hqr_factors_destroy", "hqr_lstsq_noalloc")

_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    try:
        # PyTorch ships its own HIP runtime (same soname as ROCm's).  Loading it
        # first makes libhqr.so bind to that copy, so that the process holds a
        # single HIP runtime and device pointers/streams are shared.
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError("libhqr.so is not built (%s); run __graft_entry__.build() first" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    P = ctypes.POINTER
    lib.hqr_elimlist.argtypes = [i32, i32, P(Params), P(Elim), i64, P(i64)]
    lib.hqr_elimlist_validate.argtypes = [i32, i32, P(Elim), i64]
    lib.hqr_dag_stats.argtypes = [i32, i32, P(Params), P(DagInfo)]
    lib.hqr_plan_tasks.argtypes = [i32, i32, P(Params), i32, vp, i64, P(i64)]
    lib.hqr_workspace_size.argtypes = [i64, i64, P(Params), P(ctypes.c_size_t)]
    lib.hqr_factor.argtypes = [vp, i64, i64, i64, P(Params), P(Exec), vp, ctypes.c_size_t, vp, P(vp)]
    lib.hqr_workspace_size_f32.argtypes = [i64, i64, P(Params), P(ctypes.c_size_t)]
    lib.hqr_factor_f32.argtypes = [vp, i64, i64, i64, P(Params), P(Exec), vp, ctypes.c_size_t, vp, P(vp)]
    lib.hqr_apply_workspace_size.argtypes = [i64, i32, P(Params), P(ctypes.c_size_t)]
    lib.hqr_lstsq_ir_workspace_size.argtypes = [i64, i64, P(Params), P(ctypes.c_size_t)]
    lib.hqr_lstsq_ir.argtypes = [vp, i64, i64, i64, vp, vp, vp, P(Params), P(Exec), i32, ctypes.c_double, vp,
                                 ctypes.c_size_t, vp, P(IrInfo)]
    apply_args = [i64, i64, P(Params), P(Exec), vp, ctypes.c_size_t, vp, i64, i32, vp, ctypes.c_size_t, vp]
    lib.hqr_apply_qt.argtypes = apply_args
    lib.hqr_solve.argtypes = apply_args
    lib.hqr_batch_export_factors.argtypes = [vp, i32, vp, vp, ctypes.c_size_t, vp]
    lib.hqr_apply_q.argtypes = apply_args
    lib.hqr_lstsq_workspace_size.argtypes = [i64, i64, i32, P(Params), P(ctypes.c_size_t)]
    lib.hqr_lstsq.argtypes = [vp, i64, i64, i64, vp, i64, i32, P(Params), P(Exec), vp, ctypes.c_size_t, vp, P(vp)]
    lib.hqr_factors_apply_workspace_size.argtypes = [vp, i32, P(ctypes.c_size_t)]
    handle_args = [vp, P(Exec), vp, i64, i32, vp, ctypes.c_size_t, vp]
    lib.hqr_factors_apply_qt.argtypes = handle_args
    lib.hqr_factors_apply_q.argtypes = handle_args
    lib.hqr_factors_solve.argtypes = handle_args
    lib.hqr_factors_query.argtypes = [vp, P(i64), P(i64), P(Params), P(vp), P(ctypes.c_size_t)]
    lib.hqr_lstsq_noalloc.argtypes = [vp, i64, i64, i64, vp, i64, i32, P(Params), P(Exec), vp, vp]
    lib.hqr_lstsq_noalloc.restype = ctypes.c_int
    lib.hqr_factors_destroy.argtypes = [vp]
    lib.hqr_factors_destroy.restype = None
    lib.hqr_batch_create.argtypes = [i32, vp, vp, vp, P(Params), P(Exec), P(vp)]
    lib.hqr_batch_workspace_size.argtypes = [vp, P(ctypes.c_size_t)]
    lib.hqr_batch_num_tasks.argtypes = [vp, vp, vp, i64, P(i64)]
    lib.hqr_batch_bind.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.hqr_batch_run.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.hqr_batch_status.argtypes = [vp, vp, vp, ctypes.c_double, P(i32), vp]
    lib.hqr_batch_publish_status.argtypes = [vp, vp, vp, vp]
    lib.hqr_batch_export_all.argtypes = [vp, vp, vp, vp, vp]
    lib.hqr_batch_destroy.argtypes = [vp]
    lib.hqr_batch_destroy.restype = None
    lib.hqr_lstsq_batched.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, P(Params), P(Exec), vp, ctypes.c_size_t, vp]
    lib.hqr_lstsq_batched_workspace_size.argtypes = [i32, vp, vp, vp, P(Params), P(ctypes.c_size_t)]
    lib.hqr_status.argtypes = [vp, vp, P(i32)]
    lib.hqr_status_ex.argtypes = [vp, vp, ctypes.c_double, P(i32), P(i32)]
    lib.hqr_release_plans.argtypes = []
    lib.hqr_release_plans.restype = None
    lib.hqr_strerror.argtypes = [ctypes.c_int]
    lib.hqr_strerror.restype = ctypes.c_char_p
    lib.hqr_timeline.argtypes = [vp, vp, i64, P(i64)]
    lib.hqr_timeline.restype = ctypes.c_int
    lib.hqr_last_error.argtypes = []
    lib.hqr_last_error.restype = ctypes.c_char_p
    lib.hqr_version.argtypes = []
    lib.hqr_version.restype = ctypes.c_char_p
    for name in ("hqr_elimlist", "hqr_plan_tasks", "hqr_elimlist_validate", "hqr_dag_stats", "hqr_workspace_size",
                 "hqr_factor", "hqr_apply_workspace_size", "hqr_apply_qt", "hqr_apply_q", "hqr_lstsq_workspace_size",
                 "hqr_lstsq", "hqr_status", "hqr_status_ex", "hqr_workspace_size_f32", "hqr_factor_f32",
                 "hqr_lstsq_ir_workspace_size", "hqr_lstsq_ir", "hqr_batch_create", "hqr_batch_workspace_size",
                 "hqr_batch_num_tasks", "hqr_batch_bind", "hqr_batch_run", "hqr_batch_status", "hqr_batch_publish_status",
                 "hqr_lstsq_batched",
                 "hqr_lstsq_batched_workspace_size", "hqr_solve", "hqr_batch_export_factors", "hqr_batch_export_all",
                 "hqr_factors_apply_workspace_size", "hqr_factors_apply_qt", "hqr_factors_apply_q",
                 "hqr_factors_solve", "hqr_factors_query"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class HQRError(RuntimeError):
    def __init__(self, fn, code):
        msg = load().hqr_strerror(code).decode()
        detail = load().hqr_last_error().decode() if code == 1 else ""
        super().__init__("%s failed with code %d (%s)%s" % (fn, code, msg, (": " + detail) if detail else ""))
        self.code = code


def _check(fn, rc):
    if rc != 0:
        raise HQRError(fn, rc)


def make_params(nb=256, p=1, a=1, low="greedy", high="flat", coupling="chain", domino=0, ib=16,
                precision="fp64") -> Params:
    t = lambda x: TREES[x] if isinstance(x, str) else int(x)  # noqa: E731
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return Params(nb, ib, p, a, t(low), t(high), t(coupling), int(domino), prec)


def make_exec(workers=0, order=0, spin_limit=0, ev_begin=None, ev_end=None) -> Exec:
    """Execution controls; ev_begin / ev_end are raw hipEvent_t handles (int) recorded around the
    persistent launch of a factorization."""
    return Exec(workers, order, spin_limit, ev_begin, ev_end)


def elimlist(mt: int, nt: int, params: Params) -> np.ndarray:
    lib = load()
    n = ctypes.c_int64()
    _check("hqr_elimlist", lib.hqr_elimlist(mt, nt, ctypes.byref(params), None, 0, ctypes.byref(n)))
    out = (Elim * max(n.value, 1))()
    _check("hqr_elimlist", lib.hqr_elimlist(mt, nt, ctypes.byref(params), out, n.value, ctypes.byref(n)))
    arr = np.frombuffer(out, dtype=np.int32).reshape(-1, 6)[: n.value].copy()
    return arr


def validate(mt: int, nt: int, records) -> int:
    recs = np.ascontiguousarray(np.asarray(records, dtype=np.int32).reshape(-1, 6))
    ptr = recs.ctypes.data_as(ctypes.POINTER(Elim)) if len(recs) else None
    return load().hqr_elimlist_validate(mt, nt, ptr, len(recs))


def dag_stats(mt: int, nt: int, params: Params) -> dict:
    info = DagInfo()
    _check("hqr_dag_stats", load().hqr_dag_stats(mt, nt, ctypes.byref(params), ctypes.byref(info)))
    return {"eliminations": info.eliminations, "tasks": info.tasks,
            "count": dict(zip(OPS, list(info.count))), "weight": info.weight,
            "critical_path": info.critical_path, "device_tasks": info.device_tasks}


def plan_tasks(mt: int, nt: int, params: Params, order: int = 0) -> np.ndarray:
    """The persistent launch's task table (structured array, TASK_DTYPE)."""
    lib = load()
    n = ctypes.c_int64()
    _check("hqr_plan_tasks", lib.hqr_plan_tasks(mt, nt, ctypes.byref(params), order, None, 0, ctypes.byref(n)))
    out = np.zeros(n.value, dtype=TASK_DTYPE)
    _check("hqr_plan_tasks", lib.hqr_plan_tasks(mt, nt, ctypes.byref(params), order, ctypes.c_void_p(out.ctypes.data),
                                                n.value, ctypes.byref(n)))
    return out


def workspace_size(M: int, N: int, params: Params) -> int:
    n = ctypes.c_size_t()
    _check("hqr_workspace_size", load().hqr_workspace_size(M, N, ctypes.byref(params), ctypes.byref(n)))
    return n.value


def factor_ptr(dA: int, M: int, N: int, lda: int, params: Params, exec_: Exec, dwork: int, work_bytes: int,
               stream: int, handle: bool = False):
    """hqr_factor; with ``handle`` returns a :class:`Factors` of the result."""
    h = ctypes.c_void_p()
    rc = load().hqr_factor(ctypes.c_void_p(dA), M, N, lda, ctypes.byref(params),
                           ctypes.byref(exec_) if exec_ is not None else None,
                           ctypes.c_void_p(dwork), work_bytes, ctypes.c_void_p(stream),
                           ctypes.byref(h) if handle else None)
    _check("hqr_factor", rc)
    return Factors(h) if handle else None


def workspace_size_f32(M: int, N: int, params: Params) -> int:
    n = ctypes.c_size_t()
    _check("hqr_workspace_size_f32", load().hqr_workspace_size_f32(M, N, ctypes.byref(params), ctypes.byref(n)))
    return n.value


def factor_f32_ptr(dA: int, M: int, N: int, lda: int, params: Params, exec_: Exec, dwork: int, work_bytes: int,
                   stream: int, handle: bool = False):
    h = ctypes.c_void_p()
    rc = load().hqr_factor_f32(ctypes.c_void_p(dA), M, N, lda, ctypes.byref(params),
                               ctypes.byref(exec_) if exec_ is not None else None,
                               ctypes.c_void_p(dwork), work_bytes, ctypes.c_void_p(stream),
                               ctypes.byref(h) if handle else None)
    _check("hqr_factor_f32", rc)
    return Factors(h) if handle else None


def lstsq_ir_workspace_size(M: int, N: int, params: Params) -> int:
    n = ctypes.c_size_t()
    _check("hqr_lstsq_ir_workspace_size", load().hqr_lstsq_ir_workspace_size(M, N, ctypes.byref(params),
                                                                           ctypes.byref(n)))
    return n.value


def lstsq_ir_ptr(dA: int, M: int, N: int, lda: int, db: int, dx: int, dr: int, params: Params, exec_: Exec,
                 max_iter: int, tol: float, dwork: int, work_bytes: int, stream: int) -> IrInfo:
    info = IrInfo()
    rc = load().hqr_lstsq_ir(ctypes.c_void_p(dA), M, N, lda, ctypes.c_void_p(db), ctypes.c_void_p(dx),
                             ctypes.c_void_p(dr) if dr else None, ctypes.byref(params),
                             ctypes.byref(exec_) if exec_ is not None else None, max_iter, tol,
                             ctypes.c_void_p(dwork), work_bytes, ctypes.c_void_p(stream), ctypes.byref(info))
    _check("hqr_lstsq_ir", rc)
    return info


def apply_workspace_size(M: int, nrhs: int, params: Params) -> int:
    n = ctypes.c_size_t()
    _check("hqr_apply_workspace_size", load().hqr_apply_workspace_size(M, nrhs, ctypes.byref(params), ctypes.byref(n)))
    return n.value


def apply_ptr(trans: bool, M: int, N: int, params: Params, exec_: Exec, dwork: int, work_bytes: int, dB: int,
              ldb: int, nrhs: int, bwork: int, bwork_bytes: int, stream: int) -> None:
    lib = load()
    fn = lib.hqr_apply_qt if trans else lib.hqr_apply_q
    rc = fn(M, N, ctypes.byref(params), ctypes.byref(exec_) if exec_ is not None else None, ctypes.c_void_p(dwork),
            work_bytes, ctypes.c_void_p(dB), ldb, nrhs, ctypes.c_void_p(bwork), bwork_bytes, ctypes.c_void_p(stream))
    _check("hqr_apply_qt" if trans else "hqr_apply_q", rc)


def solve_ptr(M: int, N: int, params: Params, exec_: Exec, dwork: int, work_bytes: int, dB: int, ldb: int,
              nrhs: int, bwork: int, bwork_bytes: int, stream: int) -> None:
    rc = load().hqr_solve(M, N, ctypes.byref(params), ctypes.byref(exec_) if exec_ is not None else None,
                          ctypes.c_void_p(dwork), work_bytes, ctypes.c_void_p(dB), ldb, nrhs, ctypes.c_void_p(bwork),
                          bwork_bytes, ctypes.c_void_p(stream))
    _check("hqr_solve", rc)


def lstsq_workspace_size(M: int, N: int, nrhs: int, params: Params) -> int:
    n = ctypes.c_size_t()
    _check("hqr_lstsq_workspace_size",
           load().hqr_lstsq_workspace_size(M, N, nrhs, ctypes.byref(params), ctypes.byref(n)))
    return n.value


def lstsq_ptr(dA: int, M: int, N: int, lda: int, dB: int, ldb: int, nrhs: int, params: Params, exec_: Exec,
              dwork: int, work_bytes: int, stream: int, handle: bool = False):
    h = ctypes.c_void_p()
    rc = load().hqr_lstsq(ctypes.c_void_p(dA), M, N, lda, ctypes.c_void_p(dB), ldb, nrhs, ctypes.byref(params),
                          ctypes.byref(exec_) if exec_ is not None else None, ctypes.c_void_p(dwork), work_bytes,
                          ctypes.c_void_p(stream), ctypes.byref(h) if handle else None)
    _check("hqr_lstsq", rc)
    return Factors(h) if handle else None


def lstsq_noalloc_ptr(dA: int, M: int, N: int, lda: int, dB: int, ldb: int, nrhs: int, params: Params,
                      exec_: Exec, dinfo: int, stream: int) -> int:
    """hqr_lstsq_noalloc; returns its code (0, or an error code without raising, so that callers can
    test the size limit)."""
    return load().hqr_lstsq_noalloc(ctypes.c_void_p(dA), M, N, lda, ctypes.c_void_p(dB), ldb, nrhs,
                                    ctypes.byref(params), ctypes.byref(exec_) if exec_ is not None else None,
                                    ctypes.c_void_p(dinfo) if dinfo else None, ctypes.c_void_p(stream))


NOALLOC_SCRATCH_BYTES = 64 << 20


class Factors:
    """An hqr_factors handle (shape, parameters and workspace of a finished
    factorization); freed with the object."""

    def __init__(self, handle: ctypes.c_void_p):
        self.handle = handle

    def query(self):
        """(M, N, params, dwork pointer, workspace bytes)."""
        M, N, w, n = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_void_p(), ctypes.c_size_t()
        prm = Params()
        _check("hqr_factors_query", load().hqr_factors_query(self.handle, ctypes.byref(M), ctypes.byref(N),
                                                             ctypes.byref(prm), ctypes.byref(w), ctypes.byref(n)))
        return M.value, N.value, prm, w.value or 0, n.value

    def apply_workspace_size(self, nrhs: int) -> int:
        n = ctypes.c_size_t()
        _check("hqr_factors_apply_workspace_size",
               load().hqr_factors_apply_workspace_size(self.handle, nrhs, ctypes.byref(n)))
        return n.value

    def _run(self, name, exec_, dB, ldb, nrhs, bwork, bwork_bytes, stream):
        fn = getattr(load(), name)
        _check(name, fn(self.handle, ctypes.byref(exec_) if exec_ is not None else None, ctypes.c_void_p(dB), ldb,
                        nrhs, ctypes.c_void_p(bwork), bwork_bytes, ctypes.c_void_p(stream)))

    def apply_qt(self, dB, ldb, nrhs, bwork, bwork_bytes, stream, exec_=None):
        self._run("hqr_factors_apply_qt", exec_, dB, ldb, nrhs, bwork, bwork_bytes, stream)

    def apply_q(self, dB, ldb, nrhs, bwork, bwork_bytes, stream, exec_=None):
        self._run("hqr_factors_apply_q", exec_, dB, ldb, nrhs, bwork, bwork_bytes, stream)

    def solve(self, dB, ldb, nrhs, bwork, bwork_bytes, stream, exec_=None):
        self._run("hqr_factors_solve", exec_, dB, ldb, nrhs, bwork, bwork_bytes, stream)

    def close(self) -> None:
        if self.handle:
            load().hqr_factors_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def status(dwork: int, stream: int, timeout_s: float = 0.0, detail: bool = False):
    """Status word of the launch that last used ``dwork`` (waits at most
    ``timeout_s`` seconds; 0 = the library default).  With ``detail`` returns
    (status, [task, counter, expected, seen])."""
    s = ctypes.c_int32()
    d = (ctypes.c_int32 * 4)()
    _check("hqr_status_ex", load().hqr_status_ex(ctypes.c_void_p(dwork), ctypes.c_void_p(stream), timeout_s,
                                                 ctypes.byref(s), d))
    return (s.value, list(d)) if detail else s.value


def timeline(stream: int) -> np.ndarray:
    """(ntasks, 4) uint64 timeline of the last launch (HQR_TIMELINE=1)."""
    lib = load()
    n = ctypes.c_int64()
    _check("hqr_timeline", lib.hqr_timeline(ctypes.c_void_p(stream), None, 0, ctypes.byref(n)))
    out = np.zeros((n.value, 4), dtype=np.uint64)
    if n.value:
        _check("hqr_timeline", lib.hqr_timeline(ctypes.c_void_p(stream), ctypes.c_void_p(out.ctypes.data), n.value,
                                                ctypes.byref(n)))
    return out


def _i64(xs):
    return np.ascontiguousarray(np.asarray(xs, dtype=np.int64))


def _i32(xs):
    return np.ascontiguousarray(np.asarray(xs, dtype=np.int32))


def _ptr(arr):
    return ctypes.c_void_p(arr.ctypes.data) if arr is not None else None


class Batch:
    """A planned batch of independent problems (hqr_batch_create); the
    shapes are M[q] x N[q] with nrhs[q] right-hand sides (None: none)."""

    def __init__(self, M, N, nrhs, params: Params, exec_: Exec = None):
        self.M, self.N = _i64(M), _i64(N)
        self.nrhs = _i32(nrhs) if nrhs is not None else None
        self.count = len(self.M)
        h = ctypes.c_void_p()
        rc = load().hqr_batch_create(self.count, _ptr(self.M), _ptr(self.N), _ptr(self.nrhs), ctypes.byref(params),
                                     ctypes.byref(exec_) if exec_ is not None else None, ctypes.byref(h))
        _check("hqr_batch_create", rc)
        self.handle = h

    def workspace_size(self) -> int:
        n = ctypes.c_size_t()
        _check("hqr_batch_workspace_size", load().hqr_batch_workspace_size(self.handle, ctypes.byref(n)))
        return n.value

    def tasks(self):
        """(task table as TASK_DTYPE, problem index of each task)."""
        lib = load()
        n = ctypes.c_int64()
        _check("hqr_batch_num_tasks", lib.hqr_batch_num_tasks(self.handle, None, None, 0, ctypes.byref(n)))
        t = np.zeros(n.value, dtype=TASK_DTYPE)
        q = np.zeros(n.value, dtype=np.int32)
        _check("hqr_batch_num_tasks", lib.hqr_batch_num_tasks(self.handle, _ptr(t), _ptr(q), n.value, ctypes.byref(n)))
        return t, q

    def bind(self, dA, lda, dB, ldb, dwork: int, work_bytes: int, stream: int) -> None:
        self._keep = (_i64(dA).astype(np.uint64), _i64(lda),
                      _i64(dB).astype(np.uint64) if dB is not None else None,
                      _i64(ldb) if ldb is not None else None)
        a, la, b, lb = self._keep
        rc = load().hqr_batch_bind(self.handle, _ptr(a), _ptr(la), _ptr(b), _ptr(lb), ctypes.c_void_p(dwork),
                                   work_bytes, ctypes.c_void_p(stream))
        _check("hqr_batch_bind", rc)

    def run(self, dwork: int, work_bytes: int, stream: int) -> None:
        _check("hqr_batch_run", load().hqr_batch_run(self.handle, ctypes.c_void_p(dwork), work_bytes,
                                                     ctypes.c_void_p(stream)))

    def status(self, dwork: int, stream: int, timeout_s: float = 0.0):
        """(status word, first zero diagonal index per problem or -1)."""
        s = ctypes.c_int32()
        fz = np.zeros(self.count, dtype=np.int32)
        _check("hqr_batch_status", load().hqr_batch_status(self.handle, ctypes.c_void_p(dwork),
                                                           ctypes.c_void_p(stream), timeout_s, ctypes.byref(s),
                                                           _ptr(fz)))
        return s.value, fz

    def publish_status(self, dwork: int, host: int, stream: int) -> None:
        """Enqueues the device-side write of the status into `host` (count + 1
        int32 of pinned host memory): host[0] status, host[1 + q] first zero
        diagonal index of problem q or -1, valid once the stream's work up to
        here has completed."""
        _check("hqr_batch_publish_status", load().hqr_batch_publish_status(
            self.handle, ctypes.c_void_p(dwork), ctypes.c_void_p(host), ctypes.c_void_p(stream)))

    def export_all(self, dwork: int, dsts, dst_bytes, stream: int) -> None:
        """export_factors for every problem q with dsts[q] (a device pointer)
        not 0, in one launch."""
        d = np.array([int(x or 0) for x in dsts], dtype=np.uint64)
        n = np.array([int(x) for x in dst_bytes], dtype=np.uint64)
        if d.size != self.count or n.size != self.count:
            raise ValueError("one destination and size per problem")
        _check("hqr_batch_export_all", load().hqr_batch_export_all(self.handle, ctypes.c_void_p(dwork), _ptr(d),
                                                                   _ptr(n), ctypes.c_void_p(stream)))

    def export_factors(self, q: int, dwork: int, dst: int, dst_bytes: int, stream: int) -> None:
        _check("hqr_batch_export_factors", load().hqr_batch_export_factors(
            self.handle, q, ctypes.c_void_p(dwork), ctypes.c_void_p(dst), dst_bytes, ctypes.c_void_p(stream)))

    def close(self) -> None:
        if self.handle:
            load().hqr_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lstsq_batched_workspace_size(M, N, nrhs, params: Params) -> int:
    m, n_ = _i64(M), _i64(N)
    r = _i32(nrhs) if nrhs is not None else None
    n = ctypes.c_size_t()
    _check("hqr_lstsq_batched_workspace_size",
           load().hqr_lstsq_batched_workspace_size(len(m), _ptr(m), _ptr(n_), _ptr(r), ctypes.byref(params),
                                                   ctypes.byref(n)))
    return n.value


def lstsq_batched_ptr(dA, M, N, lda, dB, ldb, nrhs, params: Params, exec_: Exec, dwork: int, work_bytes: int,
                      stream: int) -> None:
    a = _i64(dA).astype(np.uint64)
    m, n_, la = _i64(M), _i64(N), _i64(lda)
    b = _i64(dB).astype(np.uint64) if dB is not None else None
    lb = _i64(ldb) if ldb is not None else None
    r = _i32(nrhs) if nrhs is not None else None
    rc = load().hqr_lstsq_batched(len(m), _ptr(a), _ptr(m), _ptr(n_), _ptr(la), _ptr(b), _ptr(lb), _ptr(r),
                                  ctypes.byref(params), ctypes.byref(exec_) if exec_ is not None else None,
                                  ctypes.c_void_p(dwork), work_bytes, ctypes.c_void_p(stream))
    _check("hqr_lstsq_batched", rc)


def release_plans() -> None:
    load().hqr_release_plans()


def version() -> str:
    return load().hqr_version().decode()
