"""Pins of the even-odd spectrum oracle (oracle/spectrum.py).

The dense eigen-decomposition of eq. (5)'s matrix, assembled from the
oracle's operator, is checked against the closed-form plane-wave spectrum of
the free field, and its extremes against that closed form's extremes, which
for kappa < 1/8 and extents divisible by four are 1 + 16 kappa^2 (momenta
pi/2 in every direction, where sum cos p = 0) and 1 - 64 kappa^2 (p = 0).
"""
import numpy as np

import qcd_inputs as qi
from oracle import spectrum as SP


def test_free_field_spectrum_is_the_plane_wave_one():
    dims, kappa = (4, 4, 4, 4), 0.124
    A = SP.eo_dense(qi.unit_gauge(dims), kappa, dims)
    dense = np.sort(np.abs(np.linalg.eigvals(A)))
    closed = np.sort(np.abs(SP.free_eo_eigenvalues(kappa, dims)))[::2]
    assert dense.shape == closed.shape
    assert np.max(np.abs(dense - closed)) < 1e-12
    hi, lo = SP.eo_abs_extremes(qi.unit_gauge(dims), kappa, dims)
    assert abs(hi - (1 + 16 * kappa**2)) < 1e-12
    assert abs(lo - (1 - 64 * kappa**2)) < 1e-12


def test_interacting_spectrum_is_gamma5_symmetric_and_bounded():
    # gamma_5 A gamma_5 = A^dag: the eigenvalues are real or come in complex
    # conjugate pairs; |lambda - 1| <= kappa^2 |H|^2 <= 64 kappa^2 since every
    # link is unitary (|H v| <= 8 |v|)
    dims, kappa = (2, 2, 4, 4), 0.124
    U = qi.gauge_field(dims, 0.3, 91)
    lam = np.linalg.eigvals(SP.eo_dense(U, kappa, dims))
    assert np.max(np.abs(lam - 1)) <= 64 * kappa**2 + 1e-12
    # every conj(lambda) is an eigenvalue too (nearest-neighbour match)
    gap = np.abs(np.conj(lam)[:, None] - lam[None, :]).min(axis=1)
    assert np.max(gap) < 1e-10
    assert np.max(np.abs(lam.imag)) > 1e-3  # the check is not vacuous: complex pairs exist
    hi, lo = SP.eo_abs_extremes(U, kappa, dims)
    assert lo > 0 and hi >= lo
