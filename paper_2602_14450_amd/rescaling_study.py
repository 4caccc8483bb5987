"""The rescaling study of Sec. 6 on synthetic fields.

For a grid of the refinement's normalisation s (Alg. 3) and the inner
residual norm sigma (Alg. 4; Alg. 5 with sigma_lambda = sigma when the
solution is rescaled too), with and without the recalculated gamma, this
counts the FP16 matrix applications the even-odd FP16-inner refinement needs
to reach a true residual of 1e-12 (the quantity of Fig. 8), and records the
fraction of zero-valued reals in the inner right-hand side at every
refinement step (Fig. 9).  The paper's set-up is a point source and binary16
values below 2^-14 flushed to zero (ftz), which is the default here.  A few
points of the grid are repeated with BF16 storage (8 exponent bits, as FP32:
the comparison the paper's conclusion proposes), where neither underflow nor
overflow should call for rescaling.

Every solve runs in libqcd's kernels; this module only loops.

    python -m paper_2602_14450_amd.rescaling_study            # 32^3 x 64, full grid
"""
from __future__ import annotations

import argparse
import json
import time

import torch

import qcd_inputs as qi

from . import BF16, FP16, FP32, QcdError, gauge_upload, solve_mixed_ir

S_GRID = (1.0, 16.0, 128.0, 1024.0, 4096.0)
SIGMA_GRID = (0.0, 1.0, 16.0, 64.0, 256.0, 1024.0)
PANELS = ((False, False), (False, True), (True, False), (True, True))   # (rescale solution, recalculate gamma)
BF16_POINTS = ((1.0, 0.0), (128.0, 64.0), (4096.0, 0.0), (1.0, 64.0))   # (s, sigma), recalculated gamma


def run_one(g, kappa, b, s, sigma, rescale_x, recalc, ftz=True, max_outer=60, inner_max_iter=3000, prec=FP16):
    """One refinement; returns a record (matvecs None if it did not converge)."""
    if rescale_x and sigma == 0:
        return dict(s=s, sigma=sigma, rescale_x=rescale_x, recalc_gamma=recalc, matvecs=None, note="n/a")
    x = torch.zeros_like(b)
    t0 = time.perf_counter()
    try:
        info = solve_mixed_ir(g, kappa, x, b, inner_prec=prec, s=s, recalc_shat=True, sigma=sigma,
                              sigma_lambda=sigma if rescale_x else 0.0, recalc_gamma=recalc, ftz=ftz, tol=1e-12,
                              inner_tol=1e-2, max_outer=max_outer, inner_max_iter=inner_max_iter, even_odd=True,
                              raise_on_error=False)
    except QcdError as e:
        return dict(s=s, sigma=sigma, rescale_x=rescale_x, recalc_gamma=recalc, matvecs=None, note=str(e))
    torch.cuda.synchronize()
    ok = info.status == "ok" and info.true_rel_residual <= 1e-12
    vh = g.volume // 2
    return dict(s=s, sigma=sigma, rescale_x=rescale_x, recalc_gamma=recalc, matvecs=info.matvec_low // 2 if ok else None,
                prec="bf16" if prec == BF16 else ("fp16" if prec == FP16 else "fp32"),
                outer=info.outer_iters, inner=info.inner_iters, true_rel_residual=info.true_rel_residual,
                seconds=time.perf_counter() - t0, status=info.status,
                zero_fraction=[z / (24.0 * vh) for z in info.zeros])


def study(dims=(32, 32, 32, 64), kappa=0.124, eps=0.3, seed=201, s_grid=S_GRID, sigma_grid=SIGMA_GRID,
          panels=PANELS, ftz=True, log=None, bf16_points=BF16_POINTS):
    """The grid on the even-odd system with the point source b = e_0 (spin 0, colour 0, site 0)."""
    U = torch.from_numpy(qi.gauge_field(dims, eps, seed)).cuda()
    g = gauge_upload(U, dims)
    del U
    b = torch.from_numpy(qi.point_source(dims)).cuda()
    out = []
    for rescale_x, recalc in panels:
        for s in s_grid:
            for sigma in sigma_grid:
                rec = run_one(g, kappa, b, s, sigma, rescale_x, recalc, ftz=ftz)
                out.append(rec)
                if log:
                    log(f"rescale_x={int(rescale_x)} recalc_gamma={int(recalc)} s={s:g} sigma={sigma:g}: "
                        f"{rec['matvecs']} FP16 matvecs")
    bf16 = []
    for s, sigma in bf16_points:
        rec = run_one(g, kappa, b, s, sigma, False, True, ftz=ftz, prec=BF16)
        bf16.append(rec)
        if log:
            log(f"bf16 s={s:g} sigma={sigma:g}: {rec['matvecs']} BF16 matvecs")
    # zero-valued inputs: FP32 inner solve for comparison (same tolerance)
    x = torch.zeros_like(b)
    info32 = solve_mixed_ir(g, kappa, x, b, inner_prec=FP32, s=1.0, recalc_shat=False, sigma=0.0, tol=1e-12,
                            inner_tol=1e-2, even_odd=True)
    fp32 = dict(zero_fraction=[z / (24.0 * (g.volume // 2)) for z in info32.zeros], outer=info32.outer_iters,
                inner=info32.inner_iters)
    g.close()
    return dict(records=out, bf16=bf16, fp32_reference=fp32, dims=list(dims), kappa=kappa, eps=eps, ftz=ftz,
                source="point source b = e_0 (site 0, spin 0, colour 0), even-odd system")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", default="32,32,32,64")
    ap.add_argument("--kappa", type=float, default=0.124)
    ap.add_argument("--no-ftz", action="store_true")
    ap.add_argument("--out", default=None, help="write the records as JSON here")
    a = ap.parse_args()
    dims = tuple(int(v) for v in a.dims.split(","))
    res = study(dims, a.kappa, ftz=not a.no_ftz, log=lambda m: print(m, flush=True))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f)


if __name__ == "__main__":
    main()
