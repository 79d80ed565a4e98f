"""Python binding of the MI355X sparse KKT refactorization library (libkkt.so).

Argument marshalling only: every step of the analysis runs in the library's C++ host code
and every step of the refactorization, solves and refinement runs in its HIP kernels.
PyTorch supplies device memory (the workspace and vectors) and the current stream.
"""
from __future__ import annotations

import atexit
import ctypes as C
import dataclasses
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkkt.so")

OK, WARN_PIVOT_PERTURBED, WARN_NOT_CONVERGED = 0, 1, 2
# bytes of the static device array behind KKTSolver.bind_scratch (KKT_SCRATCH_BYTES)
SCRATCH_BYTES = 64 << 20
FP64, FP32 = 0, 1   # factor_precision
ERR_ARG, ERR_PATTERN, ERR_SINGULAR, ERR_NONFINITE, ERR_STATE, ERR_NOMEM, ERR_DEVICE, ERR_SCHEDULE = \
    -1, -2, -3, -4, -5, -6, -7, -8


class KKTError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = _lib().kkt_strerror(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{where}: {msg} ({code})")
        self.code = code


class _Opts(C.Structure):
    _fields_ = [("pivot_tau", C.c_double), ("tiny_pivot", C.c_double), ("equilibrate", C.c_int32),
                ("gmres_restart", C.c_int32), ("max_iters", C.c_int32), ("berr_tol", C.c_double),
                ("sn_max_width", C.c_int32), ("fixed_p", C.c_void_p), ("fixed_q", C.c_void_p),
                ("dense_mfma", C.c_int32), ("persistent_solve", C.c_int32),
                ("graph_refactor", C.c_int32), ("approx_sweeps", C.c_int32),
                ("factor_precision", C.c_int32), ("tiny_pivot_fp32", C.c_double),
                ("approx_kind", C.c_int32)]


class _Tuning(C.Structure):
    _fields_ = [("panel_max", C.c_int32), ("small_rows", C.c_int32), ("group", C.c_int32), ("wide256", C.c_int32),
                ("fuse_chains", C.c_int32), ("tiny_rows", C.c_int32)]


class _ServerOpts(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("max_inflight", C.c_int32), ("max_nrhs", C.c_int32)]


class _ServerStats(C.Structure):
    _fields_ = [("replicas", C.c_int32), ("patterns", C.c_int32), ("bytes_in_use", C.c_size_t),
                ("peak_bytes", C.c_size_t), ("replicas_created", C.c_int64), ("evictions", C.c_int64),
                ("completed", C.c_int64), ("queued", C.c_int64)]


class _Info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("berr", C.c_double),
                ("perturbed_pivots", C.c_int64)]


PROFILE_CLASSES = ["update", "refactor_large", "refactor_small", "to_csr", "lsolve", "usolve",
                   "residual", "krylov", "refactor_medium", "refactor_w256"]


class _Profile(C.Structure):
    _fields_ = [("launches", C.c_int64 * 10), ("ms", C.c_double * 10)]


class _Stats(C.Structure):
    _fields_ = [("n", C.c_int32), ("nsn", C.c_int32), ("nnz_a", C.c_int64), ("nnz_lu", C.c_int64),
                ("levels_f", C.c_int32), ("levels_l", C.c_int32), ("levels_u", C.c_int32),
                ("gpu_levels_f", C.c_int32), ("gpu_levels_l", C.c_int32), ("gpu_levels_u", C.c_int32),
                ("persistent_levels_l", C.c_int32), ("persistent_levels_u", C.c_int32),
                ("flops_refactor", C.c_double), ("nnz_lu_wide", C.c_int64),
                ("nnz_lu_medium", C.c_int64), ("copy_in_levels", C.c_int64), ("nnz_lu_w256", C.c_int64)]


EXPORTS = ["kkt_default_opts", "kkt_analyze", "kkt_get_stats", "kkt_export_symbolic",
           "kkt_workspace_bytes", "kkt_bind", "kkt_bind_scratch", "kkt_refactor", "kkt_refactor_status", "kkt_solve", "kkt_solve_approx",
           "kkt_refine", "kkt_refactor_refine", "kkt_get_tuning", "kkt_set_tuning", "kkt_autotune", "kkt_export_factors", "kkt_profile_enable", "kkt_profile_read",
           "kkt_batch_create", "kkt_batch_refactor", "kkt_batch_refine", "kkt_batch_destroy", "kkt_clone",
           "kkt_server_default_opts", "kkt_server_create", "kkt_server_add_pattern", "kkt_server_submit",
           "kkt_server_wait", "kkt_server_get_stats", "kkt_server_destroy",
           "kkt_destroy", "kkt_strerror"]

_LIB = None
# handles still open; destroyed at interpreter exit before the HIP runtime is torn down
_LIVE = weakref.WeakSet()
_LIVE_BATCHES = weakref.WeakSet()
_LIVE_SERVERS = weakref.WeakSet()


@atexit.register
def _close_all():
    for sv in list(_LIVE_SERVERS):
        sv.close()
    for bt in list(_LIVE_BATCHES):
        bt.close()
    for sk in list(_LIVE):
        sk.close()


def _lib():
    """Loads the HIP library; there is no fallback path."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2302_08656_amd/build.py "
                              "(hipcc --offload-arch=gfx950)")
        L = C.CDLL(LIB_PATH)
        p = C.c_void_p
        L.kkt_default_opts.argtypes = [C.POINTER(_Opts)]
        L.kkt_default_opts.restype = None
        L.kkt_analyze.argtypes = [C.c_int32, p, p, p, C.POINTER(_Opts), C.POINTER(C.c_void_p)]
        L.kkt_get_stats.argtypes = [p, C.POINTER(_Stats)]
        L.kkt_export_symbolic.argtypes = [p] * 11
        L.kkt_workspace_bytes.argtypes = [p, C.c_int32, C.POINTER(C.c_size_t)]
        L.kkt_bind.argtypes = [p, p, C.c_size_t, C.c_int32, p]
        L.kkt_bind_scratch.argtypes = [p, C.c_int32, p]
        L.kkt_refactor.argtypes = [p, p, p]
        L.kkt_refactor_status.argtypes = [p, C.POINTER(C.c_int64), p]
        L.kkt_solve.argtypes = [p, p, p, C.c_int32, C.c_int64, p]
        L.kkt_solve_approx.argtypes = [p, p, p, C.c_int32, C.c_int64, p]
        L.kkt_refine.argtypes = [p, p, p, C.c_int32, C.c_int64, C.POINTER(_Info), p]
        L.kkt_refactor_refine.argtypes = [p, p, p, p, C.POINTER(_Info), p]
        L.kkt_export_factors.argtypes = [p, p, p, p, p]
        L.kkt_get_tuning.argtypes = [p, C.POINTER(_Tuning)]
        L.kkt_set_tuning.argtypes = [p, C.POINTER(_Tuning)]
        L.kkt_autotune.argtypes = [p, p, C.c_int32, C.POINTER(_Tuning), C.POINTER(C.c_double), p]
        L.kkt_profile_enable.argtypes = [p, C.c_int32]
        L.kkt_profile_read.argtypes = [p, C.POINTER(_Profile), p]
        L.kkt_batch_create.argtypes = [p, C.c_int32, C.POINTER(C.c_void_p)]
        L.kkt_batch_refactor.argtypes = [p, p, p]
        L.kkt_batch_refine.argtypes = [p, p, p, C.POINTER(_Info), p]
        L.kkt_batch_destroy.argtypes = [p]
        L.kkt_batch_destroy.restype = None
        L.kkt_clone.argtypes = [p, C.POINTER(C.c_void_p)]
        L.kkt_server_default_opts.argtypes = [C.POINTER(_ServerOpts)]
        L.kkt_server_default_opts.restype = None
        L.kkt_server_create.argtypes = [C.POINTER(_ServerOpts), C.POINTER(C.c_void_p)]
        L.kkt_server_add_pattern.argtypes = [p, C.c_int32, p, p, p, C.POINTER(_Opts), C.POINTER(C.c_int32)]
        L.kkt_server_submit.argtypes = [p, C.c_int32, p, p, p, C.c_int32, C.c_int64, C.POINTER(C.c_int64)]
        L.kkt_server_wait.argtypes = [p, C.c_int64, C.POINTER(_Info), p]
        L.kkt_server_get_stats.argtypes = [p, C.POINTER(_ServerStats)]
        L.kkt_server_destroy.argtypes = [p]
        L.kkt_server_destroy.restype = None
        L.kkt_destroy.argtypes = [p]
        L.kkt_destroy.restype = None
        L.kkt_strerror.argtypes = [C.c_int]
        L.kkt_strerror.restype = C.c_char_p
        _LIB = L
    return _LIB


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def default_opts() -> dict:
    o = _Opts()
    _lib().kkt_default_opts(C.byref(o))
    return {f: getattr(o, f) for f, _ in _Opts._fields_ if f not in ("fixed_p", "fixed_q")}


@dataclasses.dataclass
class Info:
    iters: int
    status: int
    berr: float
    perturbed_pivots: int


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_ptr(t):
    return C.c_void_p(t.data_ptr())


class KKTSolver:
    """One sparsity pattern: analyze once on construction, then bind a device workspace
    and refactor / solve / refine each new system."""

    def __init__(self, n, rowptr, colind, values_k1, *, pivot_tau=None, tiny_pivot=None,
                 equilibrate=None, gmres_restart=None, max_iters=None, berr_tol=None,
                 sn_max_width=None, fixed_p=None, fixed_q=None, dense_mfma=None, persistent_solve=None,
                 graph_refactor=None, approx_sweeps=None, factor_precision=None, tiny_pivot_fp32=None,
                 approx_kind=None):
        L = _lib()
        self.n = int(n)
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        colind = np.ascontiguousarray(colind, dtype=np.int32)
        v = np.ascontiguousarray(values_k1, dtype=np.float64)
        o = _Opts()
        L.kkt_default_opts(C.byref(o))
        for name, val in (("pivot_tau", pivot_tau), ("tiny_pivot", tiny_pivot), ("equilibrate", equilibrate),
                          ("gmres_restart", gmres_restart), ("max_iters", max_iters), ("berr_tol", berr_tol),
                          ("sn_max_width", sn_max_width), ("dense_mfma", dense_mfma),
                          ("persistent_solve", persistent_solve), ("graph_refactor", graph_refactor),
                          ("approx_sweeps", approx_sweeps), ("factor_precision", factor_precision),
                          ("tiny_pivot_fp32", tiny_pivot_fp32), ("approx_kind", approx_kind)):
            if val is not None:
                setattr(o, name, val)
        fp = None if fixed_p is None else np.ascontiguousarray(fixed_p, dtype=np.int32)
        fq = None if fixed_q is None else np.ascontiguousarray(fixed_q, dtype=np.int32)
        o.fixed_p = None if fp is None else fp.ctypes.data
        o.fixed_q = None if fq is None else fq.ctypes.data
        h = C.c_void_p()
        rc = L.kkt_analyze(self.n, _np_ptr(rowptr), _np_ptr(colind), _np_ptr(v), C.byref(o), C.byref(h))
        if rc != OK:
            raise KKTError(rc, "kkt_analyze")
        self._h = h
        _LIVE.add(self)
        self.opts = {f: getattr(o, f) for f, _ in _Opts._fields_ if f not in ("fixed_p", "fixed_q")}
        st = _Stats()
        L.kkt_get_stats(h, C.byref(st))
        self.stats = {f: getattr(st, f) for f, _ in _Stats._fields_}
        self.nnz_a = st.nnz_a
        self.nnz_lu = st.nnz_lu
        self.nsn = st.nsn
        self._ws = None
        self._values = None

    # ---------------------------------------------------------------- host-only queries
    def export_symbolic(self) -> dict:
        n, nlu, na, ns = self.n, self.nnz_lu, self.nnz_a, self.nsn
        out = dict(P=np.empty(n, np.int32), Q=np.empty(n, np.int32), colptr=np.empty(n + 1, np.int64),
                   rowidx=np.empty(nlu, np.int32), parent=np.empty(n, np.int32),
                   lev_f=np.empty(n, np.int32), lev_l=np.empty(n, np.int32), lev_u=np.empty(n, np.int32),
                   sn_start=np.empty(ns + 1, np.int32), map=np.empty(na, np.int64))
        rc = _lib().kkt_export_symbolic(self._h, *[_np_ptr(out[k]) for k in
                                                   ("P", "Q", "colptr", "rowidx", "parent", "lev_f",
                                                    "lev_l", "lev_u", "sn_start", "map")])
        if rc != OK:
            raise KKTError(rc, "kkt_export_symbolic")
        return out

    def workspace_bytes(self, max_nrhs=1) -> int:
        b = C.c_size_t()
        rc = _lib().kkt_workspace_bytes(self._h, int(max_nrhs), C.byref(b))
        if rc != OK:
            raise KKTError(rc, "kkt_workspace_bytes")
        return b.value

    # ---------------------------------------------------------------- device work
    def bind(self, device=None, max_nrhs=1, stream=None):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        nbytes = self.workspace_bytes(max_nrhs)
        with torch.cuda.device(dev):
            ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
            base = ws.data_ptr()
            off = (-base) % 256
            rc = _lib().kkt_bind(self._h, C.c_void_p(base + off), nbytes, int(max_nrhs), _stream_ptr(stream))
        if rc != OK:
            # the handle may still use the previous workspace: keep it alive
            raise KKTError(rc, "kkt_bind")
        self._ws = ws          # the previous workspace is released only now
        self.device = dev
        return self

    def bind_scratch(self, device=None, max_nrhs=1, stream=None):
        """Binds to the library's static device scratch array (kkt_bind_scratch): no
        device memory is allocated, here or by later calls on this handle."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        with torch.cuda.device(dev):
            rc = _lib().kkt_bind_scratch(self._h, int(max_nrhs), _stream_ptr(stream))
        if rc != OK:
            raise KKTError(rc, "kkt_bind_scratch")
        self._ws = None
        self.device = dev
        return self

    def refactor(self, values, stream=None):
        """values: cuda float64 tensor [nnz_a] in the analysed CSR order (kept alive here,
        the library reads it again for residuals)."""
        self._check_vec(values, self.nnz_a)
        rc = _lib().kkt_refactor(self._h, _dev_ptr(values), _stream_ptr(stream))
        if rc != OK:
            raise KKTError(rc, "kkt_refactor")
        self._values = values
        return self

    def refactor_status(self, stream=None):
        pert = C.c_int64()
        rc = _lib().kkt_refactor_status(self._h, C.byref(pert), _stream_ptr(stream))
        if rc < 0:
            raise KKTError(rc, "kkt_refactor_status")
        return rc, pert.value

    def solve(self, b, x=None, stream=None):
        import torch
        nrhs, ld = self._rhs_shape(b)
        if x is None:
            x = torch.empty_like(b)
        rc = _lib().kkt_solve(self._h, _dev_ptr(b), _dev_ptr(x), nrhs, ld, _stream_ptr(stream))
        if rc != OK:
            raise KKTError(rc, "kkt_solve")
        return x

    def solve_approx(self, b, x=None, stream=None):
        """One approximate preconditioner application (kkt_solve_approx)."""
        import torch
        nrhs, ld = self._rhs_shape(b)
        if x is None:
            x = torch.empty_like(b)
        rc = _lib().kkt_solve_approx(self._h, _dev_ptr(b), _dev_ptr(x), nrhs, ld, _stream_ptr(stream))
        if rc != OK:
            raise KKTError(rc, "kkt_solve_approx")
        return x

    def refine(self, b, x=None, stream=None):
        import torch
        nrhs, ld = self._rhs_shape(b)
        if x is None:
            x = torch.empty_like(b)
        info = (_Info * nrhs)()
        rc = _lib().kkt_refine(self._h, _dev_ptr(b), _dev_ptr(x), nrhs, ld, info, _stream_ptr(stream))
        if rc < 0:
            raise KKTError(rc, "kkt_refine")
        return x, [Info(i.iters, i.status, i.berr, i.perturbed_pivots) for i in info]

    def refactor_refine(self, values, b, x=None, stream=None):
        """kkt_refactor(values) then kkt_refine(b) for one right-hand side, with the forward
        substitution running beside the refactorization (kkt_refactor_refine).  b: cuda
        float64 [n]; returns (x, Info)."""
        import torch
        self._check_vec(values, self.nnz_a)
        self._check_vec(b, self.n)
        if x is None:
            x = torch.empty_like(b)
        else:
            self._check_vec(x, self.n)
        info = _Info()
        rc = _lib().kkt_refactor_refine(self._h, _dev_ptr(values), _dev_ptr(b), _dev_ptr(x), C.byref(info),
                                        _stream_ptr(stream))
        self._values = values
        if rc < 0:
            raise KKTError(rc, "kkt_refactor_refine")
        return x, Info(info.iters, info.status, info.berr, info.perturbed_pivots)

    def tuning(self) -> dict:
        t = _Tuning()
        rc = _lib().kkt_get_tuning(self._h, C.byref(t))
        if rc != OK:
            raise KKTError(rc, "kkt_get_tuning")
        return {f: getattr(t, f) for f, _ in _Tuning._fields_}

    def set_tuning(self, panel_max, small_rows, group, wide256=1, fuse_chains=0, tiny_rows=16):
        """Rebuilds the schedule (kkt_set_tuning); the handle must be bound again."""
        t = _Tuning(int(panel_max), int(small_rows), int(group), int(wide256), int(fuse_chains), int(tiny_rows))
        rc = _lib().kkt_set_tuning(self._h, C.byref(t))
        if rc != OK:
            raise KKTError(rc, "kkt_set_tuning")
        self._ws = None
        self._refresh_stats()
        return self

    def autotune(self, values, reps=3, stream=None):
        """Times the candidate schedules on values (kkt_autotune) and keeps the fastest;
        returns (choice, ms per refactorization).  The handle must be bound again."""
        self._check_vec(values, self.nnz_a)
        t = _Tuning()
        ms = C.c_double()
        rc = _lib().kkt_autotune(self._h, _dev_ptr(values), int(reps), C.byref(t), C.byref(ms), _stream_ptr(stream))
        if rc != OK:
            raise KKTError(rc, "kkt_autotune")
        self._ws = None
        self._refresh_stats()
        return {f: getattr(t, f) for f, _ in _Tuning._fields_}, ms.value

    def _refresh_stats(self):
        st = _Stats()
        _lib().kkt_get_stats(self._h, C.byref(st))
        self.stats = {f: getattr(st, f) for f, _ in _Stats._fields_}

    def export_factors(self, stream=None):
        lu = np.empty(self.nnz_lu)
        r = np.empty(self.n)
        c = np.empty(self.n)
        rc = _lib().kkt_export_factors(self._h, _np_ptr(lu), _np_ptr(r), _np_ptr(c), _stream_ptr(stream))
        if rc != OK:
            raise KKTError(rc, "kkt_export_factors")
        return lu, r, c

    def profile(self, on: bool):
        rc = _lib().kkt_profile_enable(self._h, int(bool(on)))
        if rc != OK:
            raise KKTError(rc, "kkt_profile_enable")

    def profile_read(self, stream=None) -> dict:
        """{class: (launches, total ms)} accumulated since profile(True)."""
        pr = _Profile()
        rc = _lib().kkt_profile_read(self._h, C.byref(pr), _stream_ptr(stream))
        if rc != OK:
            raise KKTError(rc, "kkt_profile_read")
        return {name: (pr.launches[i], pr.ms[i]) for i, name in enumerate(PROFILE_CLASSES)}

    def close(self):
        if getattr(self, "_h", None) is not None and _LIB is not None:
            _LIB.kkt_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        self.close()

    # ---------------------------------------------------------------- helpers
    def _check_vec(self, t, size):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and t.numel() == size):
            raise ValueError(f"expected a contiguous cuda float64 tensor with {size} elements")

    def _rhs_shape(self, b):
        import torch
        if not (isinstance(b, torch.Tensor) and b.is_cuda and b.dtype == torch.float64 and b.is_contiguous()):
            raise ValueError("expected a contiguous cuda float64 tensor")
        if b.dim() == 1 and b.numel() == self.n:
            return 1, self.n
        if b.dim() == 2 and b.shape[1] == self.n:
            return b.shape[0], self.n
        raise ValueError(f"right-hand side must have shape [{self.n}] or [nrhs, {self.n}]")


class KKTBatch:
    """Several bound KKTSolver handles refactored together (kkt_batch_*): one launch per
    dependency level across the batch, replayed from one HIP graph.  The solvers must stay
    alive and bound while the batch is used."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        arr = (C.c_void_p * len(self.solvers))(*[sk._h.value for sk in self.solvers])
        h = C.c_void_p()
        rc = _lib().kkt_batch_create(arr, len(self.solvers), C.byref(h))
        if rc != OK:
            raise KKTError(rc, "kkt_batch_create")
        self._h = h
        _LIVE_BATCHES.add(self)

    def refactor(self, values, stream=None):
        if len(values) != len(self.solvers):
            raise ValueError("one value tensor per solver")
        for sk, v in zip(self.solvers, values):
            sk._check_vec(v, sk.nnz_a)
        arr = (C.c_void_p * len(values))(*[v.data_ptr() for v in values])
        rc = _lib().kkt_batch_refactor(self._h, arr, _stream_ptr(stream))
        if rc != OK:
            raise KKTError(rc, "kkt_batch_refactor")
        for sk, v in zip(self.solvers, values):
            sk._values = v
        return self

    def refine(self, bs, xs=None, stream=None):
        import torch
        if xs is None:
            xs = [torch.empty_like(b) for b in bs]
        for sk, b, x in zip(self.solvers, bs, xs):
            if sk._rhs_shape(b) != (1, sk.n) or x.shape != b.shape:
                raise ValueError("one right-hand side of shape [n] per solver")
        ab = (C.c_void_p * len(bs))(*[b.data_ptr() for b in bs])
        ax = (C.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        info = (_Info * len(bs))()
        rc = _lib().kkt_batch_refine(self._h, ab, ax, info, _stream_ptr(stream))
        if rc < 0:
            raise KKTError(rc, "kkt_batch_refine")
        return xs, [Info(i.iters, i.status, i.berr, i.perturbed_pivots) for i in info]

    def close(self):
        if getattr(self, "_h", None) is not None and _LIB is not None:
            _LIB.kkt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


class KKTServer:
    """The serving engine (kkt_server_*): patterns analysed once and kept resident as
    replicas, requests admitted by free replicas and the device-memory budget, run by
    worker threads on their own streams.  Device tensors passed to submit() are kept alive
    here until wait() returns for their ticket."""

    def __init__(self, hbm_budget=None, max_inflight=None, max_nrhs=None):
        L = _lib()
        o = _ServerOpts()
        L.kkt_server_default_opts(C.byref(o))
        if hbm_budget is not None:
            o.hbm_budget = int(hbm_budget)
        if max_inflight is not None:
            o.max_inflight = int(max_inflight)
        if max_nrhs is not None:
            o.max_nrhs = int(max_nrhs)
        h = C.c_void_p()
        rc = L.kkt_server_create(C.byref(o), C.byref(h))
        if rc != OK:
            raise KKTError(rc, "kkt_server_create")
        self._h = h
        self.max_nrhs = o.max_nrhs
        self._n = []
        self._nnz = []
        self._held = {}
        _LIVE_SERVERS.add(self)

    def add_pattern(self, n, rowptr, colind, values_k1, **opts):
        L = _lib()
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        colind = np.ascontiguousarray(colind, dtype=np.int32)
        v = np.ascontiguousarray(values_k1, dtype=np.float64)
        o = _Opts()
        L.kkt_default_opts(C.byref(o))
        for k, val in opts.items():
            setattr(o, k, val)
        pid = C.c_int32()
        rc = L.kkt_server_add_pattern(self._h, int(n), _np_ptr(rowptr), _np_ptr(colind), _np_ptr(v), C.byref(o),
                                      C.byref(pid))
        if rc != OK:
            raise KKTError(rc, "kkt_server_add_pattern")
        self._n.append(int(n))
        self._nnz.append(len(colind))
        return pid.value

    def submit(self, pattern, values, b, x):
        n = self._n[pattern]
        if values.numel() != self._nnz[pattern] or values.dtype != __import__("torch").float64:
            raise ValueError("values must be a float64 cuda tensor of the pattern's nnz")
        nrhs = 1 if b.dim() == 1 else b.shape[0]
        if b.shape != x.shape or b.shape[-1] != n or not (b.is_contiguous() and x.is_contiguous()):
            raise ValueError("b and x: contiguous [n] or [nrhs, n] cuda float64 tensors")
        tk = C.c_int64()
        rc = _lib().kkt_server_submit(self._h, int(pattern), _dev_ptr(values), _dev_ptr(b), _dev_ptr(x), nrhs, n,
                                      C.byref(tk))
        if rc != OK:
            raise KKTError(rc, "kkt_server_submit")
        self._held[tk.value] = (values, b, x, nrhs)
        return tk.value

    def wait(self, ticket):
        """(status, [Info per rhs], {wait_ms, device_ms, latency_ms, new_replica})"""
        _, _, _, nrhs = self._held[ticket]
        info = (_Info * nrhs)()
        t = (C.c_double * 4)()
        rc = _lib().kkt_server_wait(self._h, int(ticket), info, t)
        self._held.pop(ticket, None)
        if rc < 0 and rc != ERR_NONFINITE:
            raise KKTError(rc, "kkt_server_wait")
        return rc, [Info(i.iters, i.status, i.berr, i.perturbed_pivots) for i in info], \
            {"wait_ms": t[0], "device_ms": t[1], "latency_ms": t[2], "new_replica": bool(t[3])}

    def stats(self):
        st = _ServerStats()
        rc = _lib().kkt_server_get_stats(self._h, C.byref(st))
        if rc != OK:
            raise KKTError(rc, "kkt_server_get_stats")
        return {f: getattr(st, f) for f, _ in _ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and _LIB is not None:
            _LIB.kkt_server_destroy(self._h)
            self._h = None
        self._held = {}

    def __del__(self):
        self.close()
