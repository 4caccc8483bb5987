"""CPU oracle for the Wilson-Dirac mixed-precision solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this; only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use it.  It shares no code with the GPU path.

* :func:`dslash` -- FP64 Wilson operator from eq. (1) with full 4x4 spin
  matrices (``wilson.c``).
* :mod:`oracle.solvers` -- BiCGStab with the residual / solution rescaling
  (Alg. 4 and Alg. 5) and the iterative refinement (Alg. 2 and Alg. 3), with
  every stored vector rounded to a chosen storage precision.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wilson.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OP_D, OP_H, OP_DDAG, OP_HDAG = 0, 1, 2, 3


def build() -> str:
    """Compile wilson.c (gcc, OpenMP)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.c_void_p
        lib.or_dslash.argtypes = [dp, dp, dp, dp, ctypes.c_double, ctypes.c_int]
        lib.or_dslash.restype = None
        lib.or_dslash_sites.argtypes = [dp, dp, dp, dp, ctypes.c_double, dp, ctypes.c_int64]
        lib.or_dslash_sites.restype = None
        lib.or_gamma.argtypes = [dp]
        lib.or_gamma.restype = None
        _lib = lib
    return _lib


def _dims_arr(dims):
    return np.ascontiguousarray(np.asarray(dims, dtype=np.int32))


def gamma_matrices() -> np.ndarray:
    """The oracle's gamma_mu, shape (4, 4, 4) complex128, mu = 0..3 = x, y, z, t."""
    out = np.empty((4, 4, 4), dtype=np.complex128)
    _load().or_gamma(out.ctypes.data)
    return out


def dslash(U: np.ndarray, phi: np.ndarray, kappa: float, dims, op: int = OP_D) -> np.ndarray:
    """Apply D (op 0), H (1), D^dagger (2) or H^dagger (3) of eq. (1) in FP64.

    U: complex128 (V, 4, 3, 3); phi: complex128 (V, 4, 3) or a flat view of it.
    """
    U = np.ascontiguousarray(U, dtype=np.complex128)
    shape = phi.shape
    phi = np.ascontiguousarray(phi, dtype=np.complex128)
    out = np.empty_like(phi)
    d = _dims_arr(dims)
    assert U.size == 36 * int(np.prod(d)) and phi.size == 12 * int(np.prod(d))
    _load().or_dslash(d.ctypes.data, U.ctypes.data, phi.ctypes.data, out.ctypes.data, float(kappa), int(op))
    return out.reshape(shape)


def dslash_sites(U: np.ndarray, phi: np.ndarray, kappa: float, dims, sites) -> np.ndarray:
    """(D phi)(s) for the listed sites only, shape (len(sites), 4, 3)."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    phi = np.ascontiguousarray(phi, dtype=np.complex128)
    sites = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    out = np.empty((len(sites), 4, 3), dtype=np.complex128)
    d = _dims_arr(dims)
    _load().or_dslash_sites(d.ctypes.data, U.ctypes.data, phi.ctypes.data, out.ctypes.data,
                            float(kappa), sites.ctypes.data, len(sites))
    return out
