"""Pins for the oracle of the parallel-transport network.

* one layer whose spin matrices are those of the Wilson hop equals 1 + kappa H
  = 2 - D, computed by the (independently pinned) Wilson oracle: pins the
  transport directions, the link orientation and the spin action;
* the adjoint of each transport, linearity and gauge covariance of the
  network;
* back-propagated gradients against central finite differences.
"""
import numpy as np
import pytest

import oracle
import qcd_inputs as qi
from oracle import ptc


def test_one_layer_with_wilson_spin_matrices_is_one_plus_kappa_h():
    dims = (4, 4, 2, 6)
    U = qi.gauge_field(dims, 0.3, 5)
    psi = qi.gaussian_source(dims, 6)
    k = 0.13
    g = oracle.gamma_matrices()
    W = np.zeros((9, 1, 1, 4, 4), dtype=complex)
    W[0, 0, 0] = np.eye(4)
    for mu in range(4):
        W[1 + 2 * mu, 0, 0] = k * (np.eye(4) - g[mu])   # forward hop
        W[2 + 2 * mu, 0, 0] = k * (np.eye(4) + g[mu])   # backward hop
    nb = ptc.neighbours(dims)
    out = ptc.forward(U, psi, [W], nb)
    want = 2 * psi - oracle.dslash(U, psi, k, dims)
    assert np.abs(out - want).max() < 1e-13


def test_transport_adjoint():
    dims = (4, 2, 4, 4)
    U = qi.gauge_field(dims, 0.5, 7)
    a = qi.gaussian_source(dims, 8)
    b = qi.gaussian_source(dims, 9)
    nb = ptc.neighbours(dims)
    for p in range(9):
        lhs = np.vdot(a, ptc.transport(U, b, nb, p))
        rhs = np.vdot(ptc.transport_adj(U, a, nb, p), b)
        assert abs(lhs - rhs) < 1e-12 * np.sqrt(a.size)


def test_network_is_linear_and_gauge_covariant():
    dims = (4, 4, 4, 2)
    U = qi.gauge_field(dims, 0.3, 11)
    Ws = qi.ptc_weights([1, 2, 2, 1], seed=3, scale=1.0)
    nb = ptc.neighbours(dims)
    a, b = qi.gaussian_source(dims, 12), qi.gaussian_source(dims, 13)
    lhs = ptc.forward(U, 0.7 * a - 1.3j * b, Ws, nb)
    rhs = 0.7 * ptc.forward(U, a, Ws, nb) - 1.3j * ptc.forward(U, b, Ws, nb)
    assert np.abs(lhs - rhs).max() < 1e-12
    g = qi.gauge_transform(dims, 1.0, 14)
    fwd = nb[0]
    Ug = np.einsum("sab,smbc,smdc->smad", g, U, np.conj(g[fwd]))
    ga = np.einsum("sab,sjb->sja", g, a)
    out_g = ptc.forward(Ug, ga, Ws, nb)
    assert np.abs(out_g - np.einsum("sab,sjb->sja", g, ptc.forward(U, a, Ws, nb))).max() < 1e-12


def test_gradients_match_finite_differences():
    dims = (2, 2, 2, 4)
    U = qi.gauge_field(dims, 0.3, 21)
    Ws = qi.ptc_weights([1, 2, 2, 1], seed=4, scale=1.0)
    nb = ptc.neighbours(dims)
    rs = [qi.gaussian_source(dims, 22), qi.gaussian_source(dims, 23)]
    es = [qi.gaussian_source(dims, 24), qi.gaussian_source(dims, 25)]
    L, dWs = ptc.grad(U, rs, es, Ws, nb)
    assert abs(L - ptc.loss(U, rs, es, Ws, nb)) < 1e-12 * L
    rng = np.random.default_rng(0)
    h = 1e-6
    for l in range(3):
        for _ in range(6):
            idx = tuple(rng.integers(0, n) for n in Ws[l].shape)
            for part, unit in ((0, 1.0), (1, 1j)):
                Wp = [W.copy() for W in Ws]
                Wm = [W.copy() for W in Ws]
                Wp[l][idx] += h * unit
                Wm[l][idx] -= h * unit
                fd = (ptc.loss(U, rs, es, Wp, nb) - ptc.loss(U, rs, es, Wm, nb)) / (2 * h)
                an = dWs[l][idx].real if part == 0 else dWs[l][idx].imag
                assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (l, idx, part, fd, an)


def test_forward_at_sampled_sites_equals_the_full_forward():
    # the sampled-site form (three hops of neighbourhood, periodic wrap) gives
    # the full network's output at those sites, on a lattice with four
    # different extents so that every axis and both wrap directions are hit
    dims = (4, 6, 2, 8)
    U = qi.gauge_field(dims, 0.4, 31)
    psi = qi.gaussian_source(dims, 32)
    Ws = qi.ptc_weights([1, 2, 2, 1], seed=5, scale=1.0)
    full = ptc.forward(U, psi, Ws, ptc.neighbours(dims))
    V = int(np.prod(dims))
    sites = np.array([0, 1, 3, 5, V - 1, V // 2, 47, 23, 0])   # repeats allowed
    got = ptc.forward_sites(U, psi, Ws, dims, sites)
    assert np.abs(got - full[sites]).max() < 1e-13


def test_residual_loss_gradients_match_finite_differences():
    # L = mean |D M r - r|^2 / |r|^2 with the Wilson operator of the oracle
    dims = (2, 2, 2, 4)
    k = 0.124
    U = qi.gauge_field(dims, 0.3, 41)
    Ws = qi.ptc_weights([1, 2, 2, 1], seed=6, scale=1.0)
    nb = ptc.neighbours(dims)
    rs = [qi.gaussian_source(dims, 42), qi.gaussian_source(dims, 43)]
    L, dWs = ptc.grad_residual(U, k, rs, Ws, nb, dims)
    assert abs(L - ptc.loss_residual(U, k, rs, Ws, nb, dims)) < 1e-12 * L
    rng = np.random.default_rng(1)
    h = 1e-6
    for l in range(3):
        for _ in range(6):
            idx = tuple(rng.integers(0, n) for n in Ws[l].shape)
            for part, unit in ((0, 1.0), (1, 1j)):
                Wp = [W.copy() for W in Ws]
                Wm = [W.copy() for W in Ws]
                Wp[l][idx] += h * unit
                Wm[l][idx] -= h * unit
                fd = (ptc.loss_residual(U, k, rs, Wp, nb, dims) - ptc.loss_residual(U, k, rs, Wm, nb, dims)) / (2 * h)
                an = dWs[l][idx].real if part == 0 else dWs[l][idx].imag
                assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (l, idx, part, fd, an)


def test_neumann_residual_loss_is_the_fourth_power_of_kappa_h():
    # with M = D^-1 exactly the residual loss vanishes; the third-order Neumann
    # series leaves D M - 1 = -(kappa H)^4, so its loss equals mean |(kappa H)^4 r|^2 / |r|^2
    dims = (2, 2, 4, 4)
    k = 0.124
    U = qi.gauge_field(dims, 0.3, 51)
    nb = ptc.neighbours(dims)
    g = oracle.gamma_matrices()
    Ws = [np.zeros((9, co, ci, 4, 4), complex) for ci, co in ((1, 2), (2, 2), (2, 1))]
    hop = np.zeros((9, 4, 4), complex)
    for mu in range(4):
        hop[1 + 2 * mu] = k * (np.eye(4) - g[mu])
        hop[2 + 2 * mu] = k * (np.eye(4) + g[mu])
    Ws[0][0, 0, 0] = np.eye(4); Ws[0][:, 1, 0] = hop
    Ws[1][0, 0, 0] = np.eye(4); Ws[1][0, 0, 1] = np.eye(4); Ws[1][:, 1, 0] = hop; Ws[1][:, 1, 1] = hop
    Ws[2][0, 0, 0] = np.eye(4); Ws[2][:, 0, 1] = hop
    rs = [qi.gaussian_source(dims, 52)]
    r = rs[0]
    kh = lambda v: v - oracle.dslash(U, v, k, dims)          # kappa H = 1 - D
    want = np.linalg.norm(kh(kh(kh(kh(r))))) ** 2 / np.linalg.norm(r) ** 2
    assert abs(ptc.loss_residual(U, k, rs, Ws, nb, dims) - want) < 1e-12 * want
