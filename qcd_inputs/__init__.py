"""Seeded synthetic inputs for the Wilson-Dirac solver.

Both the CPU oracle and the GPU path take their inputs from here; this module
holds no solver arithmetic.  Arrays are numpy complex128 in the canonical
layouts:

* site index ``s = x + Lx*(y + Ly*(z + Lz*t))``, directions ``mu = 0..3`` = x,y,z,t
* gauge links ``U[s, mu, a, b]`` (the link from ``s`` to ``s + mu``), shape (V, 4, 3, 3)
* spinors ``psi[s, spin, colour]``, shape (V, 4, 3)

The gauge generator follows the workload description of the paper's
benchmarks as restated for this project: ``U = exp(i eps sum_a c_a lambda_a)``
with ``c_a ~ N(0, 1)``, then re-unitarised.  Sources are complex normal with
``E|z|^2 = 1`` or unit point sources.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libqcd_inputs.so")
_lib = None


def build() -> str:
    """Compile gen.c into libqcd_inputs.so (gcc, OpenMP)."""
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
        i64, u64, dp = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
        lib.qi_gauge.argtypes = [dp, i64, ctypes.c_double, u64]
        lib.qi_gauge_transform.argtypes = [dp, i64, ctypes.c_double, u64]
        lib.qi_gaussian.argtypes = [dp, i64, u64]
        lib.qi_uniform.argtypes = [dp, i64, u64]
        lib.qi_splitmix_raw.argtypes = [u64, dp, i64]
        for f in (lib.qi_gauge, lib.qi_gauge_transform, lib.qi_gaussian, lib.qi_uniform,
                  lib.qi_splitmix_raw):
            f.restype = None
        _lib = lib
    return _lib


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def gauge_field(dims, eps: float, seed: int) -> np.ndarray:
    """SU(3) links U[s, mu] = exp(i eps sum_a c_a lambda_a), re-unitarised."""
    v = volume(dims)
    u = np.empty((v, 4, 3, 3), dtype=np.complex128)
    _load().qi_gauge(u.ctypes.data, v, float(eps), int(seed) & (2**64 - 1))
    return u


def unit_gauge(dims) -> np.ndarray:
    """Free field U = 1."""
    v = volume(dims)
    u = np.zeros((v, 4, 3, 3), dtype=np.complex128)
    u[:, :, 0, 0] = u[:, :, 1, 1] = u[:, :, 2, 2] = 1.0
    return u


def gauge_transform(dims, eps: float, seed: int) -> np.ndarray:
    """Random SU(3) matrix per site, shape (V, 3, 3)."""
    v = volume(dims)
    g = np.empty((v, 3, 3), dtype=np.complex128)
    _load().qi_gauge_transform(g.ctypes.data, v, float(eps), int(seed) & (2**64 - 1))
    return g


def gaussian_source(dims, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Complex normal spinor field(s), re and im ~ N(0, 1/2)."""
    v = volume(dims)
    shape = (v, 4, 3) if nrhs is None else (nrhs, v, 4, 3)
    out = np.empty(shape, dtype=np.complex128)
    _load().qi_gaussian(out.ctypes.data, out.size, int(seed) & (2**64 - 1))
    return out


def point_source(dims, spin: int = 0, colour: int = 0, site: int = 0) -> np.ndarray:
    """Unit vector at (site, spin, colour); site 0, spin 0, colour 0 is b = (1, 0, ..., 0)."""
    out = np.zeros((volume(dims), 4, 3), dtype=np.complex128)
    out[site, spin, colour] = 1.0
    return out


def uniform(n: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _load().qi_uniform(out.ctypes.data, int(n), int(seed) & (2**64 - 1))
    return out


def splitmix64_sequence(state: int, n: int) -> np.ndarray:
    """The sequential SplitMix64 outputs from a given state."""
    out = np.empty(n, dtype=np.uint64)
    _load().qi_splitmix_raw(int(state) & (2**64 - 1), out.ctypes.data, int(n))
    return out


def ptc_weights(channels, seed, scale=0.3):
    """Seeded complex weights of the parallel-transport network, one array
    (9, C_out, C_in, 4, 4) per layer channels[0] -> channels[1] -> ...: complex
    Gaussian entries of size scale / sqrt(2 * 9 * 4 * C_in), plus the identity
    on the path p = 0 from input channel j % C_in to output channel j, so that
    an untrained network is close to a multiple of the identity."""
    rng = np.random.default_rng(seed)
    Ws = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        shape = (9, cout, cin, 4, 4)
        W = (rng.normal(size=shape) + 1j * rng.normal(size=shape)) * (scale / np.sqrt(2 * 9 * 4 * cin))
        for j in range(cout):
            W[0, j, j % cin] += np.eye(4)
        Ws.append(W)
    return Ws
