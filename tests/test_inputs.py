"""The seeded input generator: published RNG values, SU(3) properties, determinism."""
import numpy as np

import qcd_inputs as qi


def test_splitmix64_published_sequence():
    # First five outputs of SplitMix64 from state 1234567, as published with
    # the reference implementation (Steele, Lea & Flood 2014; Vigna's splitmix64.c).
    want = np.array([6457827717110365317, 3203168211198807973, 9817491932198370423,
                     4593380528125082431, 16408922859458223821], dtype=np.uint64)
    assert np.array_equal(qi.splitmix64_sequence(1234567, 5), want)


def test_uniform_range_and_moments():
    u = qi.uniform(200000, 7)
    assert u.min() > 0.0 and u.max() <= 1.0
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / len(u))
    assert abs(u.var() - 1 / 12) < 0.002


def test_gauge_links_are_su3_and_deterministic():
    dims = (2, 4, 6, 8)
    u = qi.gauge_field(dims, 0.3, 101)
    assert u.shape == (384, 4, 3, 3)
    eye = np.eye(3)
    assert np.abs(u @ np.conj(np.swapaxes(u, -1, -2)) - eye).max() < 1e-14
    assert np.abs(np.linalg.det(u) - 1).max() < 1e-14
    assert np.array_equal(u, qi.gauge_field(dims, 0.3, 101))
    assert not np.array_equal(u, qi.gauge_field(dims, 0.3, 102))


def test_gauge_link_generator_small_eps_limit():
    # exp(i eps H) = 1 + i eps H + O(eps^2): the anti-Hermitian part over eps
    # is i H with H traceless Hermitian, whose entries are O(1) normals.
    eps = 1e-6
    u = qi.gauge_field((2, 2, 2, 2), eps, 5)
    h = (u - np.eye(3)) / (1j * eps)
    # the next term, i eps H^2 / 2, is O(1e-5) here
    assert np.abs(h - np.conj(np.swapaxes(h, -1, -2))).max() < 1e-4
    assert np.abs(np.real(np.trace(h, axis1=-2, axis2=-1))).max() < 1e-8   # tr H = 0
    # diagonal of H: (c3 + c8/sqrt3, -c3 + c8/sqrt3, -2 c8/sqrt3), c ~ N(0,1)
    d = np.real(np.diagonal(h, axis1=-2, axis2=-1)).reshape(-1, 3)
    c8 = -d[:, 2] * np.sqrt(3) / 2
    assert 0.4 < np.std(c8) < 1.6


def test_plaquette_like_mean_matches_second_order_estimate():
    # <Re tr U>/3 = 1 - eps^2 <tr H^2>/6 + O(eps^4), and <tr H^2> = 2 * 8 = 16
    # for c_a ~ N(0,1) with tr lambda_a lambda_b = 2 delta_ab.
    eps = 0.05
    u = qi.gauge_field((4, 4, 4, 4), eps, 11)
    m = np.mean(np.real(np.trace(u, axis1=-2, axis2=-1))) / 3
    assert abs(m - (1 - eps**2 * 16 / 6)) < 5e-4


def test_gaussian_source_moments():
    b = qi.gaussian_source((4, 4, 4, 8), 202)
    z = b.reshape(-1)
    assert abs(np.mean(np.abs(z) ** 2) - 1) < 0.03
    assert abs(np.mean(z)) < 0.03
    assert abs(np.mean(z * z)) < 0.03      # circular: E z^2 = 0
    assert np.array_equal(b, qi.gaussian_source((4, 4, 4, 8), 202))


def test_point_source():
    b = qi.point_source((2, 2, 2, 2), 1, 2)
    assert np.count_nonzero(b) == 1 and b[0, 1, 2] == 1
