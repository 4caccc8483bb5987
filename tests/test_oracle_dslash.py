"""Pins for the oracle's Wilson operator (eq. (1)), independent of its own code.

* the spin matrices: Clifford algebra, Hermiticity, the printed (1 - gamma_1)
  of Sec. 2, and the Dirac representation built here from Pauli matrices;
* the free-field closed form in momentum space and its U(1)-twisted form
  (pins the neighbour sum, the sign of the gamma term and U versus U^dagger);
* gauge covariance (pins neighbour indexing and link orientation);
* the adjoint and gamma_5-hermiticity;
* a dense matrix assembled from Kronecker products with shift matrices,
  compared column by column (brute force on tiny lattices, including 2^4
  where the forward and backward neighbours coincide);
* the norm bound |D psi| <= (1 + 8 kappa) |psi|.
"""
import os

import numpy as np
import pytest

import oracle
import qcd_inputs as qi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dirac_gammas():
    """Dirac representation, built here independently of the oracle."""
    s = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]], complex)]
    z = np.zeros((2, 2), complex)
    g = [np.block([[z, -1j * sk], [1j * sk, z]]) for sk in s]
    g.append(np.diag([1, 1, -1, -1]).astype(complex))
    return np.array(g)


def load_matrix(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append([complex(t) for t in line.split()])
    return np.array(rows)


def test_gamma_matrices():
    g = oracle.gamma_matrices()
    eye = np.eye(4)
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            assert np.allclose(g[mu] @ g[nu] + g[nu] @ g[mu], 2 * eye * (mu == nu))
    # the paper's printed example fixes gamma_1
    assert np.array_equal(eye - g[0], load_matrix("one_minus_gamma1.txt"))
    # the rest is the Dirac representation
    assert np.allclose(g, dirac_gammas())
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    assert np.allclose(g5, g5.conj().T) and np.allclose(g5 @ g5, eye)
    assert np.allclose(g5, np.block([[np.zeros((2, 2)), -np.eye(2)], [-np.eye(2), np.zeros((2, 2))]]))


def plane_wave(dims, n, chi):
    """e^{i p.x} chi with p_mu = 2 pi n_mu / L_mu, canonical layout (V, 4, 3)."""
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    ph = 2 * np.pi * (n[0] * x / lx + n[1] * y / ly + n[2] * z / lz + n[3] * t / lt)
    return np.exp(1j * ph).reshape(-1)[:, None, None] * chi[None]


def free_symbol(p, kappa, g):
    """D(p) = (1 - 2 kappa sum cos p_mu) 1 + 2 i kappa sum gamma_mu sin p_mu (spin part)."""
    return (1 - 2 * kappa * np.sum(np.cos(p))) * np.eye(4) + 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4))


@pytest.mark.parametrize("dims,n", [((4, 4, 4, 4), (1, 0, 2, 3)), ((2, 4, 6, 8), (1, 3, 5, 7)),
                                    ((3, 5, 4, 6), (2, 1, 3, 5))])
def test_free_field_plane_wave(dims, n):
    rng = np.random.default_rng(0)
    kappa = 0.13
    chi = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
    phi = plane_wave(dims, n, chi)
    U = qi.unit_gauge(dims)
    out = oracle.dslash(U, phi, kappa, dims)
    p = 2 * np.pi * np.array(n) / np.array(dims)
    want = plane_wave(dims, n, free_symbol(p, kappa, dirac_gammas()) @ chi)
    assert np.abs(out - want).max() < 1e-13


def test_u1_twisted_field_shifts_momentum():
    # U_mu(x) = e^{i theta_mu} 1 acts as p -> p + theta; the backward hop sees
    # U^dagger = e^{-i theta}.  A U / U^dagger swap would give p - theta.
    dims = (4, 6, 4, 8)
    theta = np.array([0.3, -0.7, 1.1, 0.25])
    kappa = 0.11
    U = qi.unit_gauge(dims) * np.exp(1j * theta)[None, :, None, None]
    rng = np.random.default_rng(1)
    chi = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
    n = (1, 2, 3, 1)
    phi = plane_wave(dims, n, chi)
    out = oracle.dslash(U, phi, kappa, dims)
    p = 2 * np.pi * np.array(n) / np.array(dims) + theta
    want = plane_wave(dims, n, free_symbol(p, kappa, dirac_gammas()) @ chi)
    assert np.abs(out - want).max() < 1e-13


def neighbour(dims, s, mu, d):
    c = np.array(np.unravel_index(s, dims[::-1])[::-1])
    c[mu] = (c[mu] + d) % dims[mu]
    return int(np.ravel_multi_index(tuple(c[::-1]), dims[::-1]))


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 6, 8)])
def test_gauge_covariance(dims):
    # U^g_mu(x) = g(x) U_mu(x) g(x+mu)^dagger  =>  D[U^g] (g psi) = g D[U] psi
    V = int(np.prod(dims))
    U = qi.gauge_field(dims, 0.3, 7)
    g = qi.gauge_transform(dims, 1.0, 8)
    fwd = np.array([[neighbour(dims, s, mu, 1) for mu in range(4)] for s in range(V)])
    Ug = np.einsum("sab,smbc,smdc->smad", g, U, np.conj(g[fwd]))
    psi = qi.gaussian_source(dims, 9)
    gpsi = np.einsum("sab,sjb->sja", g, psi)
    lhs = oracle.dslash(Ug, gpsi, 0.124, dims)
    rhs = np.einsum("sab,sjb->sja", g, oracle.dslash(U, psi, 0.124, dims))
    assert np.abs(lhs - rhs).max() < 1e-13


def test_adjoint_and_gamma5_hermiticity():
    dims = (4, 4, 2, 6)
    U = qi.gauge_field(dims, 0.3, 3)
    a = qi.gaussian_source(dims, 4)
    b = qi.gaussian_source(dims, 5)
    k = 0.124
    Db = oracle.dslash(U, b, k, dims, oracle.OP_D)
    Dda = oracle.dslash(U, a, k, dims, oracle.OP_DDAG)
    # <a, D b> = <D^dag a, b>
    assert abs(np.vdot(a, Db) - np.vdot(Dda, b)) < 1e-12 * np.sqrt(a.size)
    g5 = dirac_gammas()
    g5 = g5[0] @ g5[1] @ g5[2] @ g5[3]
    apply_g5 = lambda v: np.einsum("ij,sjc->sic", g5, v)
    # D^dag = gamma5 D gamma5
    assert np.abs(Dda - apply_g5(oracle.dslash(U, apply_g5(a), k, dims))).max() < 1e-14


def dense_wilson(U, kappa, dims):
    """D as a dense (12V x 12V) matrix: 1 - kappa sum_mu [(1-g_mu) x U_mu T_+mu + (1+g_mu) x T_-mu U_mu^dag]
    built from Kronecker products of spin matrices with colour-site blocks."""
    V = int(np.prod(dims))
    g = dirac_gammas()
    n = 12 * V
    D = np.eye(n, dtype=complex)
    # index = site*12 + spin*3 + colour
    for mu in range(4):
        F = np.zeros((3 * V, 3 * V), complex)   # colour x site block of U_mu(x) delta_{x+mu,y}
        B = np.zeros((3 * V, 3 * V), complex)   # U_mu(x-mu)^dag delta_{x-mu,y}
        for s in range(V):
            f = neighbour(dims, s, mu, 1)
            bk = neighbour(dims, s, mu, -1)
            F[3 * s:3 * s + 3, 3 * f:3 * f + 3] += U[s, mu]
            B[3 * s:3 * s + 3, 3 * bk:3 * bk + 3] += U[bk, mu].conj().T
        # reorder (site, colour) x spin into (site, spin, colour)
        def embed(S, CS):
            M = np.einsum("ij,sctd->sictjd", S, CS.reshape(V, 3, V, 3))
            return M.reshape(n, n)
        D -= kappa * (embed(np.eye(4) - g[mu], F) + embed(np.eye(4) + g[mu], B))
    return D


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 3, 4, 5)])
def test_dense_bruteforce(dims):
    U = qi.gauge_field(dims, 0.3, 21)
    k = 0.124
    D = dense_wilson(U, k, dims)
    V = int(np.prod(dims))
    rng = np.random.default_rng(2)
    cols = rng.choice(12 * V, size=min(12 * V, 48), replace=False)
    for c in cols:
        e = np.zeros(12 * V, complex)
        e[c] = 1
        out = oracle.dslash(U, e.reshape(V, 4, 3), k, dims).reshape(-1)
        assert np.abs(out - D[:, c]).max() < 1e-14
    psi = qi.gaussian_source(dims, 22)
    assert np.abs(oracle.dslash(U, psi, k, dims).reshape(-1) - D @ psi.reshape(-1)).max() < 1e-13


def test_norm_bound_and_hopping_relation():
    dims = (4, 4, 4, 4)
    U = qi.gauge_field(dims, 0.3, 31)
    psi = qi.gaussian_source(dims, 32)
    for k in (0.1, 0.124, 0.13):
        Dp = oracle.dslash(U, psi, k, dims)
        assert np.linalg.norm(Dp) <= (1 + 8 * k) * np.linalg.norm(psi)
        H = oracle.dslash(U, psi, k, dims, oracle.OP_H)
        assert np.abs(Dp - (psi - k * H)).max() < 1e-14


def test_sampled_sites_match_full():
    dims = (4, 6, 4, 6)
    U = qi.gauge_field(dims, 0.3, 41)
    psi = qi.gaussian_source(dims, 42)
    full = oracle.dslash(U, psi, 0.12, dims)
    sites = np.array([0, 5, 77, 300, 575])
    assert np.array_equal(oracle.dslash_sites(U, psi, 0.12, dims, sites), full[sites])
