"""Host-parallel oracle of the Chebyshev step and the KPM moments (test
infrastructure): ctypes access to oracle/omp/cheb_omp.cpp, the same
definitions as ``spmmv.spmmv`` / ``spmmv.block_dots`` and
``kpm.moments_doubling`` (Sec. 3.2 listing; Sec. 2.2 DOS equation, Sec. 4),
run over the explicit CSR matrix of ``hamiltonian.assemble`` on all host
cores with OpenMP.  Built by ``build()`` with g++ (``oracle/omp/build.py``)."""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "omp", "liboracle_omp.so")
_lib = None
_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python oracle/omp/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        L.oracle_omp_threads.restype = ctypes.c_int
        L.oracle_omp_threads.argtypes = []
        L.oracle_omp_set_threads.restype = None
        L.oracle_omp_set_threads.argtypes = [ctypes.c_int]
        L.oracle_csr_sweep.restype = ctypes.c_int
        L.oracle_csr_sweep.argtypes = [ctypes.c_int64, _i64, _i64, _d, ctypes.c_int, _d, _d, _d,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double, _d]
        L.oracle_kpm_moments.restype = ctypes.c_int
        L.oracle_kpm_moments.argtypes = [ctypes.c_int64, _i64, _i64, _d, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_double, _d, _d]
        _lib = L
    return _lib


class Csr:
    """The explicit matrix in the layout the C++ code reads (int64 indices,
    complex128 values), converted once."""

    def __init__(self, H):
        H = H.tocsr()
        self.n = H.shape[0]
        self.indptr = np.ascontiguousarray(H.indptr, dtype=np.int64)
        self.indices = np.ascontiguousarray(H.indices, dtype=np.int64)
        self.values = np.ascontiguousarray(H.data, dtype=np.complex128)

    def args(self):
        return (self.n, self.indptr.ctypes.data_as(_i64), self.indices.ctypes.data_as(_i64),
                self.values.ctypes.data_as(_d))


def _p(a):
    return None if a is None else a.ctypes.data_as(_d)


def threads() -> int:
    return int(lib().oracle_omp_threads())


def set_threads(n: int) -> None:
    lib().oracle_omp_set_threads(int(n))


def sweep(A: Csr, x, alpha: float, beta: float, gamma: float, z=None, y=None):
    """y = alpha (H x - beta x) + gamma z (uniform scales), dots [nb][4]."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    nb = x.shape[1]
    y = np.empty_like(x) if y is None else y
    z = None if gamma == 0.0 else np.ascontiguousarray(z, dtype=np.complex128)
    dots = np.zeros((nb, 4))
    st = lib().oracle_csr_sweep(*A.args(), nb, _p(x), _p(z), _p(y), alpha, beta, gamma, _p(dots))
    if st:
        raise ValueError("oracle_csr_sweep: bad arguments")
    return y, dots


def kpm_moments(A: Csr, r, M: int, a: float, b: float):
    r = np.ascontiguousarray(r, dtype=np.complex128)
    nb = r.shape[1]
    mu = np.zeros((nb, M))
    st = lib().oracle_kpm_moments(*A.args(), nb, M, a, b, _p(r), _p(mu))
    if st:
        raise ValueError("oracle_kpm_moments: bad arguments")
    return mu
