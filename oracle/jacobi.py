"""ctypes loader for the oracle's C Jacobi eigensolver (oracle/jacobi.c).

TEST INFRASTRUCTURE ONLY.  `build()` compiles jacobi.c with gcc into
oracle/_jacobi.so; `eigh_jacobi` compiles it on first use if it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jacobi.c")
_LIB = os.path.join(_HERE, "_jacobi.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"],
                       check=True)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.jacobi_herm.restype = ctypes.c_int
        lib.jacobi_herm.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int, ctypes.c_double]
        _lib = lib
    return _lib


def eigh_jacobi(H: np.ndarray, max_sweeps: int = 60, tol: float = 1e-15):
    """All eigenpairs of a Hermitian matrix by cyclic Jacobi (ascending).

    Returns (w, V, sweeps) with H V = V diag(w).  Raises if not converged.
    """
    H = np.asarray(H, np.complex128)
    n = H.shape[0]
    a = np.ascontiguousarray(H).copy()
    w = np.zeros(n)
    V = np.zeros((n, n), np.complex128)
    sweeps = _load().jacobi_herm(n, a.ctypes.data, w.ctypes.data, V.ctypes.data,
                                 max_sweeps, tol)
    if sweeps < 0:
        raise RuntimeError("Jacobi did not converge")
    return w, V, sweeps
