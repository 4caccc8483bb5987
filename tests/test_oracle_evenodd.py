"""Pins of the even-odd reduction (eq. (4)-(6)) in oracle/evenodd.py."""
import numpy as np

import oracle
import qcd_inputs as qi
from oracle import evenodd as EO


def test_reduction_solves_the_full_system():
    # Schur solve + reconstruction equals a dense LU solve of the full D
    dims = (2, 2, 2, 4)
    kappa = 0.124
    U = qi.gauge_field(dims, 0.4, 601)
    b = qi.gaussian_source(dims, 602)
    V = int(np.prod(dims))
    n = 12 * V
    D = np.empty((n, n), complex)
    eye = np.eye(n)
    for j in range(n):
        D[:, j] = oracle.dslash(U, eye[j].reshape(V, 4, 3).astype(complex), kappa, dims).reshape(-1)
    x_lu = np.linalg.solve(D, b.reshape(-1)).reshape(V, 4, 3)
    x, info = EO.solve_fp64(U, kappa, dims, b, tol=1e-13)
    assert np.linalg.norm(x - x_lu) <= 1e-11 * np.linalg.norm(x_lu)


def test_reconstructed_solution_has_no_odd_residual():
    # for ANY even field x_e, x = reconstruct(x_e) satisfies (b - D x)_o = 0 and
    # (b - D x)_e = b' - A x_e
    dims = (4, 4, 4, 4)
    kappa = 0.12
    U = qi.gauge_field(dims, 0.3, 611)
    b = qi.gaussian_source(dims, 612)
    xe = qi.gaussian_source(dims, 613)
    e = EO.even_mask(dims)
    x = EO.reconstruct(U, xe, b, kappa, dims)
    r = b - oracle.dslash(U, x, kappa, dims)
    assert np.abs(r[~e]).max() <= 1e-13 * np.abs(b).max()
    r_even = EO.rhs(U, b, kappa, dims) - EO.schur(U, xe, kappa, dims)
    assert np.allclose(r[e], r_even[e], rtol=0, atol=1e-12)


def test_schur_spectrum_from_the_hopping_spectrum():
    # H maps even to odd and back, so on the even subspace A = 1 - kappa^2 H^2
    # and tr(A^k) over even fields = (1/2) sum over eigenvalues lam of H of (1 - kappa^2 lam^2)^k
    dims = (2, 2, 2, 2)
    kappa = 0.13
    U = qi.gauge_field(dims, 0.5, 621)
    V = int(np.prod(dims))
    n = 12 * V
    eye = np.eye(n)
    H = np.empty((n, n), complex)
    for j in range(n):
        H[:, j] = oracle.dslash(U, eye[j].reshape(V, 4, 3).astype(complex), 0.0, dims, oracle.OP_H).reshape(-1)
    lam = np.linalg.eigvals(H)
    e = np.repeat(EO.even_mask(dims), 12)
    idx = np.nonzero(e)[0]
    A = np.empty((len(idx), len(idx)), complex)
    for k, j in enumerate(idx):
        col = EO.schur(U, eye[j].reshape(V, 4, 3).astype(complex), kappa, dims).reshape(-1)
        A[:, k] = col[idx]
    mu = 1 - kappa * kappa * lam * lam
    P = np.eye(len(idx), dtype=complex)
    for k in range(1, 5):
        P = P @ A
        assert abs(np.trace(P) - 0.5 * np.sum(mu ** k)) <= 1e-9 * len(idx)


def test_even_odd_needs_fewer_iterations():
    dims = (4, 4, 4, 8)
    kappa = 0.124
    U = qi.gauge_field(dims, 0.3, 631)
    b = qi.gaussian_source(dims, 632)
    x_eo, info_eo = EO.solve_fp64(U, kappa, dims, b, tol=1e-12)
    x_full, info_full = oracle.solvers.solve_fp64(U, kappa, dims, b, tol=1e-12)
    assert np.linalg.norm(x_eo - x_full) <= 1e-9 * np.linalg.norm(x_full)
    assert info_eo.converged and info_full.converged
    assert info_eo.iterations < info_full.iterations


def _dense(apply, n, idx=None):
    eye = np.eye(n)
    cols = [apply(eye[j]) for j in (range(n) if idx is None else idx)]
    return np.array(cols).T


def test_even_block_of_the_inverse_inverts_the_schur_matrix():
    # block elimination of D = [[1, -kappa H_eo], [-kappa H_oe, 1]]: the even-even
    # block of D^-1 is (1 - kappa^2 H_eo H_oe)^-1, so a preconditioner of D acts on
    # eq. (5) through its even-even block
    dims = (2, 2, 2, 4)
    kappa = 0.124
    U = qi.gauge_field(dims, 0.4, 641)
    V = int(np.prod(dims))
    n = 12 * V
    shape = (V, 4, 3)
    D = _dense(lambda c: oracle.dslash(U, c.reshape(shape).astype(complex), kappa, dims).reshape(-1), n)
    idx = np.nonzero(np.repeat(EO.even_mask(dims), 12))[0]
    A = _dense(lambda c: EO.schur(U, c.reshape(shape).astype(complex), kappa, dims).reshape(-1), n, idx)[idx]
    Dinv_ee = np.linalg.inv(D)[np.ix_(idx, idx)]
    assert np.abs(Dinv_ee @ A - np.eye(len(idx))).max() < 1e-12
    # and the even-even block of kappa-expanded D^-1 to third order is 1 + kappa^2 H_eo H_oe
    kh = lambda v: v - oracle.dslash(U, v, kappa, dims)      # kappa H = 1 - D
    v = qi.gaussian_source(dims, 642)
    ve = EO.restrict(v, EO.even_mask(dims))
    series = ve + kh(ve) + kh(kh(ve)) + kh(kh(kh(ve)))
    e = EO.even_mask(dims)
    assert np.allclose(EO.restrict(series, e), 2 * ve - EO.schur(U, ve, kappa, dims), rtol=0, atol=1e-13)


def test_neumann_network_even_block_is_the_first_order_schur_series():
    # the network with the third-order Neumann weights, applied to (v_e, 0), has
    # even rows v_e + kappa^2 H_eo H_oe v_e; times eq. (5)'s matrix that leaves
    # v_e - (kappa^2 H_eo H_oe)^2 v_e
    from oracle import ptc
    dims = (2, 4, 2, 4)
    k = 0.124
    U = qi.gauge_field(dims, 0.3, 651)
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
    e = EO.even_mask(dims)
    ve = EO.restrict(qi.gaussian_source(dims, 652), e)
    out = ptc.forward(U, ve, Ws, nb)
    z = EO.restrict(out, e)
    A = lambda w: EO.schur(U, w, k, dims)
    assert np.allclose(z, 2 * ve - A(ve), rtol=0, atol=1e-13)
    a2 = A(A(ve)) - 2 * A(ve) + ve                          # (1 - A)^2 v_e = (kappa^2 H_eo H_oe)^2 v_e
    assert np.allclose(A(z), ve - a2, rtol=0, atol=1e-13)
