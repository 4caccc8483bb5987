"""Extreme |eigenvalues| of the even-odd matrix of eq. (5), FP64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 6 quotes, for its test configuration, the ratio of the largest to the
smallest modulus of the eigenvalues of the solver's matrix.  Here:

* :func:`eo_dense` -- eq. (5)'s matrix A = 1 - kappa^2 H_eo H_oe written out
  column by column (A applied to every unit vector on the even sites) on a
  lattice small enough for a dense eigen-decomposition;
* :func:`eo_abs_extremes` -- the largest and smallest |eigenvalue| of it;
* :func:`free_eo_eigenvalues` -- the same spectrum for unit links in closed
  form.  For U = 1 the hopping term is diagonal in momentum,
  H(p) = sum_mu [(1 - gamma_mu) e^{i p_mu} + (1 + gamma_mu) e^{-i p_mu}]
       = 2 sum_mu cos p_mu - 2 i sum_mu gamma_mu sin p_mu,
  whose eigenvalues are h = 2 sum cos p -+ 2 i |sin p| (the gamma matrices
  anticommute and square to one, so (sum gamma_mu s_mu)^2 = |s|^2), each
  for two spin directions and three colours.  H maps even sites to odd ones,
  so H v = h v gives H_eo H_oe v_e = h^2 v_e: A has the eigenvalues
  1 - kappa^2 h^2.  The momenta p and p + (pi, pi, pi, pi) give the same
  even-site vector and the same h^2, so every value is listed twice.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import evenodd as EO


def eo_dense(U, kappa, dims):
    """Dense A (n x n, n = 12 V / 2) in the order (even site, spin, colour)."""
    e = EO.even_mask(dims)
    sites = np.flatnonzero(e)
    V = len(e)
    n = len(sites) * 12
    A = np.empty((n, n), dtype=np.complex128)
    for j in range(n):
        v = np.zeros((V, 4, 3), dtype=np.complex128)
        v[sites[j // 12], (j % 12) // 3, j % 3] = 1.0
        A[:, j] = EO.schur(U, v, kappa, dims)[sites].reshape(-1)
    return A


def eo_abs_extremes(U, kappa, dims):
    """(largest, smallest) |eigenvalue| of eq. (5)'s matrix, from numpy's eigvals."""
    lam = np.abs(np.linalg.eigvals(eo_dense(U, kappa, dims)))
    return float(lam.max()), float(lam.min())


def free_eo_eigenvalues(kappa, dims):
    """All 12 V values 1 - kappa^2 h^2 for unit links (each eigenvalue of A twice)."""
    out = []
    for n in itertools.product(*[range(L) for L in dims]):
        p = 2 * np.pi * np.array(n) / np.array(dims)
        c = 2 * np.sum(np.cos(p))
        s = 2 * np.sqrt(np.sum(np.sin(p) ** 2))
        for h in (c - 1j * s, c + 1j * s):
            out += [1 - kappa * kappa * h * h] * 6
    return np.array(out)
