"""ctypes front end of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product library never imports it.

Every function takes the problem as (dim, n, h, kernel, sigma_t[, sigma_s])
with NumPy float64 arrays laid out x-fastest (cell index j = i0 + n0 (i1 + n1 i2)).
kernel 0 = homogeneous exp(-sigma_t r) (sigma_t[0] is used), 1 = midpoint ray
rule through the d-linear interpolant of sigma_t; adding 2 selects approach
(M-ii) of Sec. 3.2 (Remark 3.1) instead of (M-iii) (Problem(scheme=1) does this).
Operators: 0 -> A x, 1 -> A (sigma_s x), 2 -> x - A (sigma_s x).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_long)


class GmresInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("matvecs", ctypes.c_int),
                ("converged", ctypes.c_int), ("restarts", ctypes.c_int),
                ("rel_resid_est", ctypes.c_double), ("rel_resid_true", ctypes.c_double)]


def build(force=True):
    """Compile liboracle.so with gcc (IEEE double, no fast-math)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        L.oracle_sigma_interp.restype = ctypes.c_double
        L.oracle_sigma_interp.argtypes = [ctypes.c_int, _lp, ctypes.c_double, _dp, _dp]
        L.oracle_tau.restype = ctypes.c_double
        L.oracle_tau.argtypes = [ctypes.c_int, _lp, ctypes.c_double, _dp, _dp, _dp, ctypes.c_long]
        L.oracle_steps_real.restype = ctypes.c_long
        L.oracle_steps_real.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_steps_grid.restype = ctypes.c_long
        L.oracle_steps_grid.argtypes = [ctypes.c_long]
        L.oracle_kernel_points.restype = ctypes.c_double
        L.oracle_kernel_points.argtypes = [ctypes.c_int, _lp, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp]
        L.oracle_kernel_cells.restype = ctypes.c_double
        L.oracle_kernel_cells.argtypes = [ctypes.c_int, _lp, ctypes.c_double, ctypes.c_int, _dp,
                                          ctypes.c_long, ctypes.c_long]
        L.oracle_self_cell.restype = ctypes.c_double
        L.oracle_self_cell.argtypes = [ctypes.c_int, _lp, ctypes.c_double, ctypes.c_int, _dp, ctypes.c_long]
        L.oracle_diag.restype = None
        L.oracle_diag.argtypes = [ctypes.c_int, _lp, ctypes.c_double, ctypes.c_int, _dp, _dp, ctypes.c_int]
        L.oracle_matrix.restype = None
        L.oracle_matrix.argtypes = [ctypes.c_int, _lp, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp,
                                    ctypes.c_int]
        L.oracle_apply.restype = None
        L.oracle_apply.argtypes = [ctypes.c_int, _lp, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp,
                                   ctypes.c_int, _dp, _dp, ctypes.c_int, ctypes.c_int]
        L.oracle_apply_rows.restype = None
        L.oracle_apply_rows.argtypes = [ctypes.c_int, _lp, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp,
                                        ctypes.c_int, _dp, _lp, ctypes.c_long, _dp, ctypes.c_int,
                                        ctypes.c_int]
        L.oracle_cell_integral.restype = ctypes.c_double
        L.oracle_cell_integral.argtypes = [ctypes.c_int, ctypes.c_double, _dp]
        L.oracle_entry.restype = ctypes.c_double
        L.oracle_entry.argtypes = [ctypes.c_int, _lp, ctypes.c_double, ctypes.c_int, _dp, ctypes.c_long,
                                   ctypes.c_long]
        L.oracle_gmres.restype = ctypes.c_int
        L.oracle_gmres.argtypes = [ctypes.c_int, _lp, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp,
                                   _dp, _dp, _dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.POINTER(GmresInfo)]
        _lib = L
    return _lib


def _threads(nthreads):
    if nthreads:
        return int(nthreads)
    return max(1, len(os.sched_getaffinity(0)))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(_dp)


def _n3(n):
    n = list(n) + [1] * (3 - len(n))
    return (ctypes.c_long * 3)(*n)


class Problem:
    """A grid with its media.  sigma_t/sigma_s are flat float64 arrays of length N."""

    def __init__(self, dim, n, h, kernel, sigma_t, sigma_s=None, scheme=0):
        self.dim = int(dim)
        self.n = tuple(int(v) for v in n)[:dim]
        self.N = int(np.prod(self.n))
        self.h = float(h)
        self.scheme = int(scheme)
        self.kernel = int(kernel) + 2 * self.scheme
        self.st = _f64(sigma_t).reshape(-1)
        assert self.st.size == self.N
        self.ss = _f64(sigma_s).reshape(-1) if sigma_s is not None else np.zeros(self.N)
        self._n = _n3(self.n)
        self._diag = None

    # -- building blocks ---------------------------------------------------
    def sigma_interp(self, p):
        p = _f64(p)
        return lib().oracle_sigma_interp(self.dim, self._n, self.h, _p(self.st), _p(p))

    def tau(self, xa, xb, m):
        xa, xb = _f64(xa), _f64(xb)
        return lib().oracle_tau(self.dim, self._n, self.h, _p(self.st), _p(xa), _p(xb), int(m))

    def kernel_points(self, x, y):
        x, y = _f64(x), _f64(y)
        return lib().oracle_kernel_points(self.dim, self._n, self.h, self.kernel, _p(self.st), _p(x), _p(y))

    def kernel_cells(self, j, k):
        return lib().oracle_kernel_cells(self.dim, self._n, self.h, self.kernel, _p(self.st), int(j), int(k))

    def entry(self, j, k):
        """Matrix entry A_jk of the selected approach."""
        return lib().oracle_entry(self.dim, self._n, self.h, self.kernel, _p(self.st), int(j), int(k))

    def self_cell(self, j):
        return lib().oracle_self_cell(self.dim, self._n, self.h, self.kernel, _p(self.st), int(j))

    def diag(self, nthreads=0):
        if self._diag is None:
            d = np.empty(self.N)
            lib().oracle_diag(self.dim, self._n, self.h, self.kernel, _p(self.st), _p(d), _threads(nthreads))
            self._diag = d
        return self._diag

    def matrix(self, nthreads=0):
        d = self.diag(nthreads)
        A = np.empty((self.N, self.N))
        lib().oracle_matrix(self.dim, self._n, self.h, self.kernel, _p(self.st), _p(d), _p(A),
                            _threads(nthreads))
        return A

    # -- the apply ---------------------------------------------------------
    def apply(self, x, op=1, nthreads=0):
        """x: (N,) or (N, nrhs) -> same shape."""
        x = np.asarray(x, dtype=np.float64)
        one = x.ndim == 1
        X = np.asfortranarray(x.reshape(self.N, -1))
        nrhs = X.shape[1]
        Y = np.empty((self.N, nrhs), order="F")
        d = self.diag(nthreads)
        lib().oracle_apply(self.dim, self._n, self.h, self.kernel, _p(self.st), _p(self.ss), _p(d), int(op),
                           _p(X), _p(Y), nrhs, _threads(nthreads))
        return Y[:, 0].copy() if one else Y

    def apply_rows(self, x, rows, op=1, nthreads=0, use_full_diag=False):
        x = np.asarray(x, dtype=np.float64)
        one = x.ndim == 1
        X = np.asfortranarray(x.reshape(self.N, -1))
        nrhs = X.shape[1]
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        Y = np.empty((rows.size, nrhs), order="F")
        d = self.diag(nthreads) if use_full_diag else None
        lib().oracle_apply_rows(self.dim, self._n, self.h, self.kernel, _p(self.st), _p(self.ss),
                                _p(d) if d is not None else None, int(op), _p(X),
                                rows.ctypes.data_as(_lp), rows.size, _p(Y), nrhs, _threads(nthreads))
        return Y[:, 0].copy() if one else Y

    def gmres(self, f, tol=1e-10, maxit=500, restart=0, nthreads=0):
        """Solve (I - A S) U = A f.  Returns (U, phi, info dict)."""
        f = _f64(f).reshape(-1)
        U = np.empty(self.N)
        phi = np.empty(self.N)
        info = GmresInfo()
        d = self.diag(nthreads)
        st = lib().oracle_gmres(self.dim, self._n, self.h, self.kernel, _p(self.st), _p(self.ss), _p(d),
                                _p(f), _p(U), _p(phi), float(tol), int(maxit), int(restart),
                                _threads(nthreads), ctypes.byref(info))
        out = {k: getattr(info, k) for k, _ in GmresInfo._fields_}
        out["status"] = st
        return U, phi, out


def cell_integral(dim, h, t):
    """I(t): integral of |z|^{1-d} over the cell of side h centred at t (Remark 3.1)."""
    tt = np.zeros(3)
    tt[:len(t)] = np.asarray(t, dtype=np.float64)
    return lib().oracle_cell_integral(int(dim), float(h), _p(tt))


def steps_real(r, h):
    return lib().oracle_steps_real(float(r), float(h))


def steps_grid(K):
    return lib().oracle_steps_grid(int(K))
