"""ctypes front end of the plain FP64 CPU oracle (kkt_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU-baseline leg
of the benchmark.  The GPU library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kkt_oracle.c")
_LIB = os.path.join(_HERE, "libkkt_oracle.so")

OK, WARN_PERTURBED, WARN_NOT_CONVERGED = 0, 1, 2
ERR_ARG, ERR_PATTERN, ERR_SINGULAR, ERR_NONFINITE, ERR_NOMEM = -1, -2, -3, -4, -6

TAU = 0.0             # threshold-pivoting tolerance (0: keep every nonzero diagonal)
EPS = 2.0 ** -40      # tiny-pivot replacement factor (reading C4)
SN_MAX = 256          # supernode width cap


def build() -> str:
    """Compile the oracle with no operation fused (gcc, -ffp-contract=off)."""
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        p = C.c_void_p
        L.orc_validate.argtypes = [C.c_int32, p, p]
        L.orc_min_degree.argtypes = [C.c_int32, p, p, p]
        L.orc_equilibrate.argtypes = [C.c_int32, p, p, p, C.c_int, p, p]
        L.orc_analyze.argtypes = [C.c_int32, p, p, p, C.c_double, C.c_int32, C.c_int, p, p,
                                  C.POINTER(C.c_void_p), C.POINTER(C.c_int32)]
        L.orc_free.argtypes = [p]
        L.orc_free.restype = None
        L.orc_sizes.argtypes = [p, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
        L.orc_sizes.restype = None
        L.orc_export.argtypes = [p] * 12
        L.orc_export.restype = None
        L.orc_refactor.argtypes = [p, p, C.c_double, C.c_int, p, p, p, C.POINTER(C.c_int64)]
        L.orc_solve.argtypes = [p, p, p, p, p, p, p]
        L.orc_solve.restype = None
        L.orc_residual.argtypes = [C.c_int32, p, p, p, p, p, p]
        L.orc_residual.restype = C.c_double
        L.orc_fgmres.argtypes = [p, p, p, p, p, p, p, C.c_int32, C.c_int32, C.c_double,
                                 C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.orc_approx_solve.argtypes = [p, p, p, p, p, C.c_int32, C.c_int32, C.c_int32, p, p]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code: int, where: str, col: int = -1):
        super().__init__(f"{where}: oracle status {code}" + (f" at step {col}" if col >= 0 else ""))
        self.code = code
        self.col = col


def _csr(rowptr, colind):
    return (np.ascontiguousarray(rowptr, dtype=np.int64),
            np.ascontiguousarray(colind, dtype=np.int32))


def validate(n, rowptr, colind) -> int:
    rowptr, colind = _csr(rowptr, colind)
    return lib().orc_validate(n, _p(rowptr), _p(colind))


def min_degree(n, rowptr, colind) -> np.ndarray:
    rowptr, colind = _csr(rowptr, colind)
    order = np.empty(n, dtype=np.int32)
    rc = lib().orc_min_degree(n, _p(rowptr), _p(colind), _p(order))
    if rc:
        raise OracleError(rc, "min_degree")
    return order


def equilibrate(n, rowptr, colind, values, scale=True):
    rowptr, colind = _csr(rowptr, colind)
    v = np.ascontiguousarray(values, dtype=np.float64)
    r = np.empty(n)
    c = np.empty(n)
    rc = lib().orc_equilibrate(n, _p(rowptr), _p(colind), _p(v), int(scale), _p(r), _p(c))
    if rc:
        raise OracleError(rc, "equilibrate")
    return r, c


class Symbolic:
    """Result of the oracle's analyze step (O0-O4) plus the factors of the analysed system."""

    def __init__(self, n, rowptr, colind, values, *, tau=TAU, sn_max=SN_MAX, scale=True,
                 fixed_p=None, fixed_q=None):
        L = lib()
        self.rowptr, self.colind = _csr(rowptr, colind)
        self.n = int(n)
        self.scale = bool(scale)
        v = np.ascontiguousarray(values, dtype=np.float64)
        fp = None if fixed_p is None else np.ascontiguousarray(fixed_p, dtype=np.int32)
        fq = None if fixed_q is None else np.ascontiguousarray(fixed_q, dtype=np.int32)
        h = C.c_void_p()
        col = C.c_int32(-1)
        rc = L.orc_analyze(self.n, _p(self.rowptr), _p(self.colind), _p(v), float(tau), int(sn_max),
                           int(scale), None if fp is None else _p(fp), None if fq is None else _p(fq),
                           C.byref(h), C.byref(col))
        if rc:
            raise OracleError(rc, "analyze", col.value)
        self._h = h
        n_ = C.c_int32()
        nnz_a, nnz_lu = C.c_int64(), C.c_int64()
        nsn = C.c_int32()
        L.orc_sizes(h, C.byref(n_), C.byref(nnz_a), C.byref(nnz_lu), C.byref(nsn))
        self.nnz_a, self.nnz_lu, self.nsn = nnz_a.value, nnz_lu.value, nsn.value
        n = self.n
        self.P = np.empty(n, np.int32)
        self.Q = np.empty(n, np.int32)
        self.colptr = np.empty(n + 1, np.int64)
        self.rowidx = np.empty(self.nnz_lu, np.int32)
        self.parent = np.empty(n, np.int32)
        self.lev_f = np.empty(n, np.int32)
        self.lev_l = np.empty(n, np.int32)
        self.lev_u = np.empty(n, np.int32)
        self.sn_start = np.empty(self.nsn + 1, np.int32)
        self.map = np.empty(self.nnz_a, np.int64)
        self.lu_k1 = np.empty(self.nnz_lu)
        L.orc_export(h, _p(self.P), _p(self.Q), _p(self.colptr), _p(self.rowidx), _p(self.parent),
                     _p(self.lev_f), _p(self.lev_l), _p(self.lev_u), _p(self.sn_start), _p(self.map),
                     _p(self.lu_k1))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    def refactor(self, values, eps=EPS):
        """Returns (lu canonical values, r, c, n_perturbed, status)."""
        v = np.ascontiguousarray(values, dtype=np.float64)
        lu = np.empty(self.nnz_lu)
        r = np.empty(self.n)
        c = np.empty(self.n)
        npert = C.c_int64(0)
        rc = lib().orc_refactor(self._h, _p(v), float(eps), int(self.scale), _p(lu), _p(r), _p(c),
                                C.byref(npert))
        if rc < 0:
            raise OracleError(rc, "refactor")
        return lu, r, c, npert.value, rc

    def solve(self, lu, r, c, b):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty(self.n)
        w = np.empty(self.n)
        lib().orc_solve(self._h, _p(lu), _p(r), _p(c), _p(b), _p(x), _p(w))
        return x

    def approx_solve(self, lu, r, c, b, sweeps, kind=0, chunk=32):
        """O9: x from `sweeps` Jacobi (kind 0) or block Gauss-Seidel (kind 1, chunks of
        `chunk` permuted rows) sweeps per triangle, each triangle from the zero vector."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty(self.n)
        w = np.empty(3 * self.n)
        rc = lib().orc_approx_solve(self._h, _p(np.ascontiguousarray(lu, dtype=np.float64)), _p(r), _p(c), _p(b),
                                    int(sweeps), int(kind), int(chunk), _p(x), _p(w))
        if rc:
            raise OracleError(rc, "approx_solve")
        return x

    def fgmres(self, values, lu, r, c, b, *, restart=30, max_it=100, tol=1e-10):
        """Returns (x, iterations, berr, status)."""
        v = np.ascontiguousarray(values, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty(self.n)
        it = C.c_int32(0)
        be = C.c_double(0)
        rc = lib().orc_fgmres(self._h, _p(v), _p(lu), _p(r), _p(c), _p(b), _p(x), int(restart),
                              int(max_it), float(tol), C.byref(it), C.byref(be))
        if rc < 0:
            raise OracleError(rc, "fgmres")
        return x, it.value, be.value, rc

    # dense views for small tests --------------------------------------------------
    def dense_factors(self, lu):
        n = self.n
        Lm = np.eye(n)
        Um = np.zeros((n, n))
        for k in range(n):
            for p in range(self.colptr[k], self.colptr[k + 1]):
                i = self.rowidx[p]
                if i > k:
                    Lm[i, k] = lu[p]
                else:
                    Um[i, k] = lu[p]
        return Lm, Um


def residual(n, rowptr, colind, values, x, b):
    """(r = b - A x, normwise backward error)."""
    rowptr, colind = _csr(rowptr, colind)
    v = np.ascontiguousarray(values, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    res = np.empty(n)
    be = lib().orc_residual(n, _p(rowptr), _p(colind), _p(v), _p(x), _p(b), _p(res))
    return res, be
