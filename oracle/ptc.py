"""Oracle of the gauge-covariant parallel-transport network (FP64, numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A layer maps C_in spinor fields to C_out fields:

    out_j(x) = sum_i sum_p W[p, j, i] (T_p psi_i)(x)

with nine paths p = 0 (identity), +mu, -mu (mu = x, y, z, t):

    (T_{+mu} psi)(x) = U_mu(x) psi(x + mu),
    (T_{-mu} psi)(x) = U_mu(x - mu)^dagger psi(x - mu),

and W[p, j, i] a complex 4x4 matrix acting on spin (colour is carried by the
transport), so the layer is gauge covariant.  The network is the composition
of its layers (no nonlinearity: it is a fixed linear operator, usable as a
right preconditioner of a Krylov solver).

Gradients use the convention grad = dL/dRe + i dL/dIm for complex values.
"""
from __future__ import annotations

import numpy as np

from . import OP_DDAG, dslash

PATHS = [(None, 0)] + [(mu, d) for mu in range(4) for d in (+1, -1)]   # p = 0, +x, -x, +y, ...


def neighbours(dims):
    """fwd[s, mu], bwd[s, mu]: lexicographic index of s + mu and s - mu (periodic)."""
    lx, ly, lz, lt = dims
    V = lx * ly * lz * lt
    s = np.arange(V)
    c = [s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)]
    fwd = np.empty((V, 4), dtype=np.int64)
    bwd = np.empty((V, 4), dtype=np.int64)
    for mu in range(4):
        for d, out in ((+1, fwd), (-1, bwd)):
            cc = list(c)
            cc[mu] = (c[mu] + d) % dims[mu]
            out[:, mu] = cc[0] + lx * (cc[1] + ly * (cc[2] + lz * cc[3]))
    return fwd, bwd


def transport(U, psi, nb, p):
    """T_p psi for one field psi (V, 4, 3)."""
    mu, d = PATHS[p]
    if mu is None:
        return psi.copy()
    fwd, bwd = nb
    if d > 0:
        return np.einsum("sab,sjb->sja", U[:, mu], psi[fwd[:, mu]])
    return np.einsum("sba,sjb->sja", np.conj(U[bwd[:, mu], mu]), psi[bwd[:, mu]])


def transport_adj(U, phi, nb, p):
    """(T_p)^dagger phi; for unitary links T_{+mu}^dagger = T_{-mu} and vice versa."""
    mu, d = PATHS[p]
    if mu is None:
        return phi.copy()
    return transport(U, phi, nb, p + 1 if d > 0 else p - 1)


def layer(U, fields, W, nb):
    """fields (C_in, V, 4, 3), W (9, C_out, C_in, 4, 4) -> (C_out, V, 4, 3)."""
    cin = fields.shape[0]
    out = np.zeros((W.shape[1],) + fields.shape[1:], dtype=np.complex128)
    for i in range(cin):
        for p in range(9):
            t = transport(U, fields[i], nb, p)
            out += np.einsum("jab,sbc->jsac", W[p, :, i], t)
    return out


def forward(U, psi, Ws, nb, keep=False):
    """Network applied to psi (V, 4, 3); nb = neighbours(dims); with keep, also the layer inputs."""
    x = psi[None]
    inputs = []
    for W in Ws:
        inputs.append(x)
        x = layer(U, x, W, nb)
    return (x[0], inputs) if keep else x[0]


def site_neighbour(dims, sites, mu, d):
    """Lexicographic index of site + d * mu-hat (periodic) for an array of sites."""
    lx, ly, lz, lt = dims
    c = [sites % lx, (sites // lx) % ly, (sites // (lx * ly)) % lz, sites // (lx * ly * lz)]
    c[mu] = (c[mu] + d) % dims[mu]
    return c[0] + lx * (c[1] + ly * (c[2] + lz * c[3]))


def forward_sites(U, psi, Ws, dims, sites):
    """The network's output M(psi) at the listed sites only, shape (len(sites), 4, 3).

    Layer l's output at a site needs layer l's input at that site and its
    eight neighbours, so going backwards from the last layer the sites that
    each layer must be evaluated on grow by one hop per layer; each layer is
    then the same sum over paths and input channels as :func:`layer`,
    evaluated on that set only (for lattices too large to run the full
    network in numpy).
    """
    sites = np.asarray(sites, dtype=np.int64)
    L = len(Ws)
    need = [None] * (L + 1)
    need[L] = np.unique(sites)
    for l in range(L, 0, -1):
        grown = [need[l]] + [site_neighbour(dims, need[l], mu, d) for mu in range(4) for d in (+1, -1)]
        need[l - 1] = np.unique(np.concatenate(grown))
    x = psi[need[0]][None]                       # (C_in = 1, sites of need[0], 4, 3)
    for l, W in enumerate(Ws):
        have, want = need[l], need[l + 1]
        out = np.zeros((W.shape[1], len(want), 4, 3), dtype=np.complex128)
        for p in range(9):
            mu, d = PATHS[p]
            if mu is None:
                src = want
            else:
                src = site_neighbour(dims, want, mu, d)
            pos = np.searchsorted(have, src)
            assert np.all(have[pos] == src)
            for i in range(x.shape[0]):
                f = x[i, pos]
                if mu is None:
                    t = f
                elif d > 0:                      # U_mu(x) psi(x + mu)
                    t = np.einsum("sab,sjb->sja", U[want, mu], f)
                else:                            # U_mu(x - mu)^dagger psi(x - mu)
                    t = np.einsum("sba,sjb->sja", np.conj(U[src, mu]), f)
                out += np.einsum("jab,sbc->jsac", W[p, :, i], t)
        x = out
    pos = np.searchsorted(need[L], sites)
    return x[0, pos]


def loss(U, rs, es, Ws, nb):
    """mean over the batch of |M(r_b) - e_b|^2 / |e_b|^2."""
    tot = 0.0
    for r, e in zip(rs, es):
        m = forward(U, r, Ws, nb)
        tot += np.vdot(m - e, m - e).real / np.vdot(e, e).real
    return tot / len(rs)


def backprop(U, Ws, inputs, dout, nb, dWs):
    """Add the weight gradients of one sample to dWs, given the layer inputs
    of its forward pass and the gradient dout (1, V, 4, 3) of its output."""
    for l in range(len(Ws) - 1, -1, -1):
        W, fields = Ws[l], inputs[l]
        cin = fields.shape[0]
        din = np.zeros_like(fields)
        for i in range(cin):
            for p in range(9):
                t = transport(U, fields[i], nb, p)
                # dW[p, j, i] = sum_x dout_j(x) t(x)^H over spin (colour summed)
                dWs[l][p, :, i] += np.einsum("jsac,sbc->jab", dout, np.conj(t))
                # dX = W^H dout, then the adjoint transport
                dx = np.einsum("jba,jsbc->sac", np.conj(W[p, :, i]), dout)
                din[i] += transport_adj(U, dx, nb, p)
        dout = din


def loss_residual(U, kappa, rs, Ws, nb, dims):
    """mean over the batch of |D M(r_b) - r_b|^2 / |r_b|^2, D the Wilson matrix of eq. (1)."""
    tot = 0.0
    for r in rs:
        y = dslash(U, forward(U, r, Ws, nb), kappa, dims)
        tot += np.vdot(y - r, y - r).real / np.vdot(r, r).real
    return tot / len(rs)


def grad_residual(U, kappa, rs, Ws, nb, dims):
    """(residual loss, [dW per layer]): the output gradient of sample b is
    2 / (B |r_b|^2) D^dagger (D M r_b - r_b), then back-propagation."""
    dWs = [np.zeros_like(W) for W in Ws]
    tot = 0.0
    B = len(rs)
    for r in rs:
        m, inputs = forward(U, r, Ws, nb, keep=True)
        y = dslash(U, m, kappa, dims)
        rn = np.vdot(r, r).real
        tot += np.vdot(y - r, y - r).real / rn
        dout = (2.0 / (B * rn)) * dslash(U, y - r, kappa, dims, OP_DDAG)[None]
        backprop(U, Ws, inputs, dout, nb, dWs)
    return tot / B, dWs


def grad(U, rs, es, Ws, nb):
    """(loss, [dW per layer]) by back-propagation through the layers."""
    dWs = [np.zeros_like(W) for W in Ws]
    tot = 0.0
    B = len(rs)
    for r, e in zip(rs, es):
        m, inputs = forward(U, r, Ws, nb, keep=True)
        en = np.vdot(e, e).real
        tot += np.vdot(m - e, m - e).real / en
        dout = (2.0 / (B * en)) * (m - e)[None]          # dL/dRe + i dL/dIm of the output
        backprop(U, Ws, inputs, dout, nb, dWs)
    return tot / B, dWs

