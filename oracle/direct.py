"""Oracle: exact discrete solution p* = A^{-1} S and an independent iterative check.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The method (ASSOR-PCG) only reaches, to a tolerance, the solution of the linear system
of Eq 2.1, so the oracle for the solve is that solution itself:

* ``solve_band``  : Cholesky elimination of the banded SPD matrix (LAPACK dpbtrf/dpbtrs
                    via SciPy).  In the natural order (theta fastest) every coupling,
                    including the periodic wrap, lies within n_theta of the diagonal.
* ``solve_dense`` : Gaussian elimination on the dense matrix (tiny grids only).
* ``sor_solve``   : lexicographic SOR / Gauss-Seidel sweeps on the CSR matrix, in plain C
                    (``oracle/sor.c``), iterated to a residual tolerance or stagnation.
"""

import ctypes
import os
import subprocess

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SOR_SRC = os.path.join(_HERE, "sor.c")
_SOR_LIB = os.path.join(_HERE, "_sor.so")
_lib = None


def build_native(force=False):
    """Compile the oracle's C helper with gcc (host code only)."""
    if force or not os.path.exists(_SOR_LIB) or os.path.getmtime(_SOR_LIB) < os.path.getmtime(_SOR_SRC):
        tmp = _SOR_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SOR_SRC, "-lm"])
        os.replace(tmp, _SOR_LIB)
    return _SOR_LIB


def _load():
    global _lib
    if _lib is None:
        build_native()
        lib = ctypes.CDLL(_SOR_LIB)
        f = lib.sor_csr
        f.restype = ctypes.c_int64
        f.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int64,
                      ctypes.c_double, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
        _lib = lib
    return _lib


def upper_band(A, u):
    """LAPACK upper band storage ab[u + i - j, j] = A[i, j] for j - u <= i <= j.

    Built in Fortran order, so that LAPACK factors it in place: at 2048 x 1024 the band
    alone is 34 GB, and a second copy would not fit in the memory of a host."""
    A = sp.coo_matrix(A)
    n = A.shape[0]
    keep = (A.col >= A.row)
    if np.any(A.col[keep] - A.row[keep] > u):
        raise ValueError("matrix has entries beyond the declared bandwidth")
    if not np.all(np.isfinite(A.data)):
        raise ValueError("matrix has non-finite entries")
    ab = np.zeros((u + 1, n), dtype=A.dtype, order="F")
    np.add.at(ab, (u + A.row[keep] - A.col[keep], A.col[keep]), A.data[keep])
    return ab


def band_factor(A, bandwidth):
    """Upper Cholesky factor U (A = U^T U) in LAPACK band storage (dpbtrf), in place."""
    ab = upper_band(A, bandwidth)
    return sla.cholesky_banded(ab, overwrite_ab=True, lower=False, check_finite=False)


def band_solve(cb, S):
    """Solve with a factor from ``band_factor``: S may hold one or several right-hand sides
    (n,) or (n, m)."""
    S = np.asarray(S, dtype=float)
    if not np.all(np.isfinite(S)):
        raise ValueError("right-hand side has non-finite entries")
    return sla.cho_solve_banded((cb, False), S, check_finite=False)


def solve_band(A, S, bandwidth):
    """Exact solution of the SPD system by banded Cholesky elimination."""
    return band_solve(band_factor(A, bandwidth), S)


def solve_dense(A, S):
    """Gaussian elimination on the dense matrix (for grids of a few hundred cells)."""
    return np.linalg.solve(np.asarray(A.todense()), np.asarray(S))


def sor_solve(A, S, omega=1.0, tol=1e-14, max_sweeps=200000, x0=None, check_every=10):
    """SOR / Gauss-Seidel (omega=1) sweeps to tolerance.  Returns (x, sweeps, rel_res)."""
    lib = _load()
    A = sp.csr_matrix(A)
    ip = np.ascontiguousarray(A.indptr, dtype=np.int64)
    ix = np.ascontiguousarray(A.indices, dtype=np.int64)
    a = np.ascontiguousarray(A.data, dtype=np.float64)
    b = np.ascontiguousarray(S, dtype=np.float64)
    x = np.zeros(A.shape[0]) if x0 is None else np.array(x0, dtype=np.float64)
    rr = ctypes.c_double(0.0)
    sweeps = lib.sor_csr(A.shape[0], ip.ctypes.data, ix.ctypes.data, a.ctypes.data,
                         b.ctypes.data, x.ctypes.data, float(omega), int(max_sweeps),
                         float(tol), int(check_every), ctypes.byref(rr))
    return x, int(sweeps), rr.value
