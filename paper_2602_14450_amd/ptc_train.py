"""Training of the parallel-transport preconditioner on pairs the solver makes.

Each pair is a Gaussian source r (generated on the device) and e = D^-1 r
from the library's own FP32 BiCGStab (relative residual 1e-6).  Pairs live on the device as complex64
(half the bytes of the canonical complex128 that the C ABI takes; a batch is
widened just before each call).  The network starts from the third-order
Neumann series of D^-1 and is trained with Adam through qcd_ptc_train_step,
one gauge field after another with shared weights and optimiser state.

Every arithmetic step runs in libqcd's kernels; this module only moves
tensors and loops.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import torch

import qcd_inputs as qi

from . import FP32, PTC, Gauge, bicgstab, gauge_upload, gaussian_spinors


@dataclass
class PairSet:
    gauge: Gauge
    r: torch.Tensor   # (P, V, 4, 3) complex64, device
    e: torch.Tensor   # (P, V, 4, 3) complex64, device
    solve_iters: list = field(default_factory=list)


def make_pairs(dims, kappa, gauge_seed, npairs, source_seed, eps=0.3, batch=16, tol=1e-6, max_iter=5000):
    """npairs (r, D^-1 r) pairs on the gauge field of seed gauge_seed."""
    U = torch.from_numpy(qi.gauge_field(dims, eps, gauge_seed)).to("cuda")
    g = gauge_upload(U, dims)
    del U
    V = qi.volume(dims)
    R = torch.empty((npairs, V, 4, 3), dtype=torch.complex64, device="cuda")
    E = torch.empty_like(R)
    iters = []
    for b0 in range(0, npairs, batch):
        nb = min(batch, npairs - b0)
        r = gaussian_spinors((nb, V, 4, 3), source_seed + b0)
        x = torch.zeros_like(r)
        infos = bicgstab(g, kappa, x, r, prec=FP32, tol=tol, max_iter=max_iter, history=False)
        infos = infos if isinstance(infos, list) else [infos]
        iters += [i.inner_iters for i in infos]
        R[b0:b0 + nb] = r.to(torch.complex64)
        E[b0:b0 + nb] = x.to(torch.complex64)
    return PairSet(g, R, E, iters)


def train(net: PTC, sets, epochs=1, batch=16, lr=1e-3, log=None):
    """Adam over all pairs of all sets, one set (gauge field) after another per
    epoch; returns the per-step losses."""
    losses = []
    for ep in range(epochs):
        for ps in sets:
            net.set_gauge(ps.gauge)
            P = ps.r.shape[0]
            for b0 in range(0, P - batch + 1, batch):
                r = ps.r[b0:b0 + batch].to(torch.complex128)
                e = ps.e[b0:b0 + batch].to(torch.complex128)
                losses.append(net.train_step(r, e, lr=lr))
        if log:
            log(f"epoch {ep}: mean loss of the last field {sum(losses[-(P // batch):]) / max(1, P // batch):.4f}")
    return losses


def evaluate(net: PTC, ps: PairSet, batch=16):
    """Mean loss |M r - e|^2 / |e|^2 over a pair set (no weight change)."""
    net.set_gauge(ps.gauge)
    tot, cnt = 0.0, 0
    P = ps.r.shape[0]
    for b0 in range(0, P - batch + 1, batch):
        r = ps.r[b0:b0 + batch].to(torch.complex128)
        e = ps.e[b0:b0 + batch].to(torch.complex128)
        tot += net.loss_grad(r, e, want_grad=False) * batch
        cnt += batch
    return tot / max(cnt, 1)


def train_preconditioner(dims=(16, 16, 16, 16), kappa=0.124, nfields=8, pairs_per_field=512, epochs=1,
                         batch=16, lr=1e-3, gauge_seed0=1000, source_seed0=2_000_000, channels=(1, 2, 2, 1),
                         log=None):
    """The learned form: pairs on nfields seeded fields, Neumann start, Adam.
    Returns (net, sets, info); the network is bound to the last field."""
    t0 = time.perf_counter()
    sets = [make_pairs(dims, kappa, gauge_seed0 + f, pairs_per_field, source_seed0 + 100_000 * f, batch=batch)
            for f in range(nfields)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    net = PTC(sets[0].gauge, channels, max_batch=batch)
    net.init_neumann(kappa)
    loss0 = evaluate(net, sets[0], batch)
    losses = train(net, sets, epochs=epochs, batch=batch, lr=lr, log=log)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = {"pairs": nfields * pairs_per_field, "fields": nfields, "epochs": epochs, "batch": batch, "lr": lr,
            "pair_seconds": t1 - t0, "train_seconds": t2 - t1, "loss_neumann_field0": loss0,
            "loss_first": losses[0] if losses else None, "loss_last": losses[-1] if losses else None,
            "fp32_solve_iters_mean": sum(sum(s.solve_iters) for s in sets) / max(1, sum(len(s.solve_iters)
                                                                                        for s in sets))}
    return net, sets, info


def residual_loss(net: PTC, g: Gauge, kappa, seed, nsrc=32, batch=16):
    """Mean residual loss |D M r - r|^2 / |r|^2 over nsrc seeded Gaussian
    sources on gauge field g (no weight change)."""
    net.set_gauge(g)
    V = g.volume
    tot = 0.0
    for b0 in range(0, nsrc, batch):
        nb = min(batch, nsrc - b0)
        r = gaussian_spinors((nb, V, 4, 3), seed + b0)
        tot += net.loss_grad_residual(kappa, r, want_grad=False) * nb
    return tot / nsrc


def train_residual(dims=(16, 16, 16, 16), kappa=0.124, nfields=8, sources_per_field=512, epochs=1, batch=16,
                   lr=1e-3, gauge_seed0=1000, source_seed0=3_000_000, channels=(1, 2, 2, 1), eps=0.3,
                   gauges=None, log=None):
    """The learned form trained on the residual loss |D M r - r|^2 / |r|^2
    (how far D M is from the identity, what a right preconditioner is judged
    by) over Gaussian sources r drawn on the device: no solves are needed.
    Neumann start, Adam, one gauge field after another with shared weights.
    Returns (net, gauges, info); the network is bound to the last field."""
    t0 = time.perf_counter()
    if gauges is None:
        gauges = []
        for f in range(nfields):
            U = torch.from_numpy(qi.gauge_field(dims, eps, gauge_seed0 + f)).to("cuda")
            gauges.append(gauge_upload(U, dims))
            del U
    V = qi.volume(dims)
    net = PTC(gauges[0], channels, max_batch=batch)
    net.init_neumann(kappa)
    loss0 = residual_loss(net, gauges[0], kappa, source_seed0 - 1_000_000)
    t1 = time.perf_counter()
    losses = []
    for ep in range(epochs):
        for f, g in enumerate(gauges):
            net.set_gauge(g)
            for b0 in range(0, sources_per_field - batch + 1, batch):
                r = gaussian_spinors((batch, V, 4, 3), source_seed0 + 100_000 * f + 10_000_000 * ep + b0)
                losses.append(net.train_step_residual(kappa, r, lr=lr))
        if log:
            log(f"epoch {ep}: last loss {losses[-1]:.5f}")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = {"loss": "residual |D M r - r|^2 / |r|^2", "sources": nfields * sources_per_field, "fields": nfields,
            "epochs": epochs, "batch": batch, "lr": lr, "setup_seconds": t1 - t0, "train_seconds": t2 - t1,
            "loss_neumann_field0": loss0, "loss_first": losses[0] if losses else None,
            "loss_last": losses[-1] if losses else None}
    return net, gauges, info
