"""Even-odd reduction of the Wilson system (eq. (4)-(6)), FP64 numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

With sites split by parity (even: x + y + z + t even), D = 1 - kappa H has
unit diagonal blocks and off-diagonal blocks D_eo = -kappa H_eo,
D_oe = -kappa H_oe, so eq. (5) reads

    (1 - kappa^2 H_eo H_oe) xi_e = eta_e + kappa H_eo eta_o,

and eq. (6) gives xi_o = eta_o + kappa H_oe xi_e.

Fields here are full-size arrays (V, 4, 3) that are zero on the parity they
do not belong to; H_eo and H_oe are the full hopping term applied to a field
of one parity and restricted to the other.
"""
from __future__ import annotations

import numpy as np

from . import OP_H, dslash
from . import solvers as S


def even_mask(dims):
    """(V,) boolean: True on even sites, lexicographic order x fastest."""
    lx, ly, lz, lt = dims
    s = np.arange(lx * ly * lz * lt)
    c = [s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)]
    return (c[0] + c[1] + c[2] + c[3]) % 2 == 0


def restrict(v, mask):
    out = np.zeros_like(v)
    out[mask] = v[mask]
    return out


def hop_to(U, v, dims, target_even):
    """H applied to v (taken on the other parity), kept on the target parity."""
    e = even_mask(dims)
    src = restrict(v, ~e if target_even else e)
    return restrict(dslash(U, src, 0.0, dims, OP_H), e if target_even else ~e)


def schur(U, xe, kappa, dims):
    """(1 - kappa^2 H_eo H_oe) x_e, eq. (5)'s matrix."""
    e = even_mask(dims)
    xe = restrict(xe, e)
    return xe - kappa * kappa * hop_to(U, hop_to(U, xe, dims, False), dims, True)


def rhs(U, b, kappa, dims):
    """eta_e + kappa H_eo eta_o, eq. (5)'s right-hand side (D_ee^-1 = 1, D_eo = -kappa H_eo)."""
    e = even_mask(dims)
    return restrict(b, e) + kappa * hop_to(U, b, dims, True)


def reconstruct(U, xe, b, kappa, dims):
    """The full solution: xi_e and xi_o = eta_o + kappa H_oe xi_e (eq. (6))."""
    e = even_mask(dims)
    xe = restrict(xe, e)
    return xe + restrict(b, ~e) + kappa * hop_to(U, xe, dims, False)


def solve_fp64(U, kappa, dims, b, tol=1e-12, maxiter=20000):
    """FP64 BiCGStab on eq. (5), then eq. (6); returns (x, info of the even solve)."""
    bp = rhs(U, b, kappa, dims)
    A = lambda v: schur(U, v, kappa, dims)
    xe, info = S.bicgstab(A, bp, S.FP64, tol2=tol * tol, maxiter=maxiter, sigma=None)
    return reconstruct(U, xe, b, kappa, dims), info
