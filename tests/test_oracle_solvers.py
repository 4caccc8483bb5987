"""Pins for the oracle's solvers (Alg. 2-5), independent of their own code.

* FP64 BiCGStab against a dense LU solve (2^4, 2x3x4x5) and against the
  free-field momentum-space solution by FFT (U = 1);
* beta = 1 in the first iteration with rho' = |r|^2, and the FP16 overflow of
  beta that the paper's initialisation avoids (Sec. 3);
* rescaling is a no-op in exact arithmetic: in FP64 the rescaled variants of
  Alg. 4/5 give the same iterates as gamma = 1;
* one refinement step with an exact inner solve is exact (pins the
  correction factor of Alg. 2/3);
* s^ differs from s by FP16 rounding only, and the zero count of the first
  inner input for b = e_0 is what the paper prints (Sec. 6, Fig. 9 text);
* storage rounding matches IEEE binary16 values of Table 1, and BF16
  rounding (Table 1's format) matches the conversion of a library (torch's
  bfloat16, float32 inputs) and hand-derived ties;
* the BF16-inner refinement (the comparison the paper's conclusion proposes)
  reaches the FP64 solution.
"""
import math
import os

import numpy as np
import pytest

import oracle
import qcd_inputs as qi
from oracle import solvers as S
from test_oracle_dslash import dense_wilson, dirac_gammas

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def paper_facts():
    out = {}
    with open(os.path.join(GOLDEN, "paper_facts.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split()
                out[k] = float(v)
    return out


def test_binary16_rounding_matches_table1():
    f = paper_facts()
    big = np.array([65504.0, 65519.0, 65520.0, 2.0 ** -14, 2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -26])
    r = S.lowp(big.astype(complex), S.FP16).real
    assert r[0] == f["fp16_max_normal"] and r[1] == 65504.0 and np.isinf(r[2])
    assert r[3] == 2.0 ** f["fp16_emin"] and abs(r[3] - f["fp16_min_normal"]) < 1e-7
    assert r[4] == 2.0 ** -24                 # smallest subnormal
    assert r[5] == 0.0                        # tie to even -> 0
    assert r[6] == 2.0 ** -24                 # 1.5 ulp rounds up to nearest even
    # round to nearest even at 1 + 2^-11 (a tie): goes to 1; 1 + 3*2^-11 -> 1 + 2^-9
    eps = 2.0 ** -f["fp16_fraction_bits"]
    t = S.lowp(np.array([1 + eps / 2, 1 + 3 * eps / 2], complex), S.FP16).real
    assert t[0] == 1.0 and t[1] == 1 + 2 * eps
    # flush to zero removes subnormals only
    z = S.lowp(np.array([2.0 ** -15, 2.0 ** -14], complex), S.FP16, ftz=True).real
    assert z[0] == 0.0 and z[1] == 2.0 ** -14
    # one rounding from FP64: 1 + 2^-11 + 2^-40 is just above the tie and
    # rounds up; two roundings through FP32 would land on the tie and give 1
    d = S.lowp(np.array([1 + 2.0 ** -11 + 2.0 ** -40], complex), S.FP16).real
    assert d[0] == 1 + 2.0 ** -10
    e32 = S.lowp(np.array([1 + 2.0 ** -24, 1 + 3 * 2.0 ** -24], complex), S.FP32).real
    assert e32[0] == 1.0 and e32[1] == 1 + 2.0 ** -22


def test_bf16_rounding_matches_table1_and_a_library():
    f = paper_facts()
    fb = int(f["bf16_fraction_bits"])
    eps = 2.0 ** -fb
    # ties to even at 1 + eps/2 and 1 + 3 eps/2; just above a tie rounds up
    # even when FP32 could not hold the excess (one rounding from FP64)
    t = S.lowp(np.array([1 + eps / 2, 1 + 3 * eps / 2, 1 + eps / 2 + 2.0 ** -40, -(1 + eps / 2 + 2.0 ** -40)],
                        complex), S.BF16).real
    assert t[0] == 1.0 and t[1] == 1 + 2 * eps and t[2] == 1 + eps and t[3] == -(1 + eps)
    emin, emax = int(f["bf16_emin"]), int(f["bf16_emax"])
    top = (2 - eps) * 2.0 ** emax
    r = S.round_bf16(np.array([top, top * (1 + 2.0 ** -10), top + 2.0 ** (emax - fb - 1), 2.0 ** emin,
                               2.0 ** (emin - fb), 2.0 ** (emin - fb - 1), 3 * 2.0 ** (emin - fb - 1)]))
    assert r[0] == top and r[1] == top and np.isinf(r[2])    # the tie above the largest value overflows
    assert r[3] == 2.0 ** emin                                 # smallest normal
    assert r[4] == 2.0 ** (emin - fb)                          # smallest subnormal
    assert r[5] == 0.0 and r[6] == 2.0 ** (emin - fb + 1)      # ties to even among subnormals
    z = S.lowp(np.array([2.0 ** (emin - 1), 2.0 ** emin], complex), S.BF16, ftz=True).real
    assert z[0] == 0.0 and z[1] == 2.0 ** emin
    # a library's float32 -> bfloat16 conversion (round to nearest even) on
    # values exactly representable in float32, ties included
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    v = (rng.standard_normal(20000) * np.exp(rng.uniform(-60, 60, 20000))).astype(np.float32)
    bits = v.view(np.uint32)
    v = np.concatenate([v, ((bits & ~np.uint32(0xFFFF)) | np.uint32(0x8000)).view(np.float32)])   # exact ties
    lib = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    mine = S.round_bf16(v.astype(np.float64))
    assert np.array_equal(lib, mine)


def test_bf16_inner_refinement_matches_fp64():
    dims = (4, 4, 4, 8)
    U = qi.gauge_field(dims, 0.3, 97)
    b = qi.gaussian_source(dims, 98)
    k = 0.12
    x64, _ = S.solve_fp64(U, k, dims, b, tol=1e-14)
    for s, sig in [(1.0, None), (128.0, 64.0)]:
        x, info = S.solve_mixed_ir(U, k, dims, b, inner_prec=S.BF16, s=s, sigma=sig, recalc_shat=(s != 1.0))
        assert info.converged and info.true_rel_residual <= 1e-12
        r = b - oracle.dslash(U, x, k, dims)
        assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-12
        assert np.linalg.norm(x - x64) / np.linalg.norm(x64) < 1e-10
        # the stored inner right-hand side is the BF16 rounding of the rescaled residual
        assert abs(info.shat_over_s[0] - 1) < 2.0 ** -8


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 3, 4, 5)])
def test_fp64_bicgstab_matches_dense_lu(dims):
    U = qi.gauge_field(dims, 0.3, 51)
    b = qi.gaussian_source(dims, 52)
    k = 0.124
    x, info = S.solve_fp64(U, k, dims, b, tol=1e-14)
    assert info.converged
    xs = np.linalg.solve(dense_wilson(U, k, dims), b.reshape(-1)).reshape(b.shape)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-12


def fft_free_solve(b, kappa, dims):
    """x = D^{-1} b for U = 1, mode by mode: x(p) = D(p)^{-1} b(p)."""
    lx, ly, lz, lt = dims
    g = dirac_gammas()
    bt = np.fft.fftn(b.reshape(lt, lz, ly, lx, 4, 3), axes=(0, 1, 2, 3))
    xt = np.empty_like(bt)
    for it in range(lt):
        for iz in range(lz):
            for iy in range(ly):
                for ix in range(lx):
                    p = 2 * np.pi * np.array([ix / lx, iy / ly, iz / lz, it / lt])
                    Dp = (1 - 2 * kappa * np.cos(p).sum()) * np.eye(4) + 2j * kappa * sum(
                        g[m] * np.sin(p[m]) for m in range(4))
                    xt[it, iz, iy, ix] = np.linalg.solve(Dp, bt[it, iz, iy, ix])
    return np.fft.ifftn(xt, axes=(0, 1, 2, 3)).reshape(b.shape)


def test_fp64_bicgstab_free_field_fft():
    dims = (4, 4, 4, 6)
    b = qi.gaussian_source(dims, 61)
    k = 0.11
    x, info = S.solve_fp64(qi.unit_gauge(dims), k, dims, b, tol=1e-14)
    assert info.converged
    xs = fft_free_solve(b, k, dims)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-12


def test_first_beta_is_one_and_unit_rho_overflows_fp16():
    dims = (4, 4, 4, 4)
    U = qi.gauge_field(dims, 0.3, 71)
    b = 40.0 * qi.gaussian_source(dims, 72)           # |b|^2 ~ 1.2e6 > 65504
    A = S.LowPrecWilson(U, 0.12, dims, S.FP16)
    _, info = S.bicgstab(A, b, S.FP16, tol2=1e-4, maxiter=3, sigma=64.0)
    assert info.betas[0] == 1.0
    # with rho' = 1 (an FP64/FP32 habit) the first beta equals |b|^2, beyond
    # the largest binary16 value, so beta itself is not representable in FP16
    _, info1 = S.bicgstab(A, b, S.FP16, tol2=1e-4, maxiter=1, sigma=64.0, rho_init=1.0)
    assert abs(info1.betas[0]) > paper_facts()["fp16_max_normal"]
    assert np.isinf(np.float16(abs(info1.betas[0])))


@pytest.mark.parametrize("variant", [dict(sigma=64.0, recalc_gamma=False), dict(sigma=64.0, recalc_gamma=True),
                                     dict(sigma=256.0, recalc_gamma=True, sigma_lambda=256.0),
                                     dict(sigma=1e-3, recalc_gamma=True, sigma_lambda=1e3)])
def test_rescaling_is_a_noop_in_fp64(variant):
    dims = (4, 4, 4, 4)
    U = qi.gauge_field(dims, 0.3, 81)
    b = qi.gaussian_source(dims, 82)
    A = lambda v: oracle.dslash(U, v, 0.124, dims)
    x0, i0 = S.bicgstab(A, b, S.FP64, tol2=0.0, maxiter=12)
    x1, i1 = S.bicgstab(A, b, S.FP64, tol2=0.0, maxiter=12, **variant)
    assert i0.iterations == i1.iterations == 12
    assert np.linalg.norm(x1 - x0) / np.linalg.norm(x0) < 1e-12
    # the unscaled residual history agrees too
    assert np.allclose(i0.history, i1.history, rtol=1e-9, atol=0)


@pytest.mark.parametrize("s,recalc", [(1.0, False), (128.0, True), (4096.0, True)])
def test_one_exact_inner_solve_gives_exact_refinement_step(s, recalc):
    dims = (2, 3, 4, 5)
    U = qi.gauge_field(dims, 0.3, 91)
    b = qi.gaussian_source(dims, 92)
    k = 0.124
    Dd = dense_wilson(U, k, dims)
    exact = lambda y: (np.linalg.solve(Dd, y.reshape(-1)).reshape(y.shape), S.BicgstabInfo(iterations=1))
    x, info = S.solve_mixed_ir(U, k, dims, b, inner_prec=S.FP64, s=s, recalc_shat=recalc, tol=1e-12,
                               max_outer=1, inner_solver=exact)
    assert info.outer == 1 and info.true_rel_residual < 1e-13


def test_shat_and_zero_count_for_unit_source():
    f = paper_facts()
    dims = (4, 4, 4, 4)
    U = qi.gauge_field(dims, 0.3, 93)
    b = qi.point_source(dims)                          # the paper's b = (1, 0, ..., 0)
    _, info = S.solve_mixed_ir(U, 0.12, dims, b, inner_prec=S.FP16, s=128.0, sigma=64.0, max_outer=1,
                               inner_maxiter=3)
    nreal = 2 * 12 * int(np.prod(dims))
    assert info.zeros[0] == nreal - int(f["nonzero_first_input"])
    # s^ = |single(y~)| differs from s by binary16 rounding only
    assert abs(info.shat_over_s[0] - 1) < 2.0 ** -11


def test_mixed_ir_reaches_target_and_matches_fp64():
    dims = (4, 4, 4, 8)
    U = qi.gauge_field(dims, 0.3, 95)
    b = qi.gaussian_source(dims, 96)
    k = 0.12
    x64, _ = S.solve_fp64(U, k, dims, b, tol=1e-14)
    for prec, s, sig in [(S.FP32, 1.0, None), (S.FP16, 128.0, 64.0), (S.FP16, 4096.0, None)]:
        x, info = S.solve_mixed_ir(U, k, dims, b, inner_prec=prec, s=s, sigma=sig, recalc_shat=(s != 1.0))
        assert info.converged and info.true_rel_residual <= 1e-12
        r = b - oracle.dslash(U, x, k, dims)
        assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-12
        assert np.linalg.norm(x - x64) / np.linalg.norm(x64) < 1e-10


def test_point_source_breaks_down_on_full_operator():
    # With r* = r = e_0 and D = 1 - kappa H, s = kappa H e_0 lives on the
    # other checkerboard and (H^2 e_0)(0) = 0 because (1 - g)(1 + g) = 0, so
    # rho = (r*, r) vanishes in the second iteration.
    dims = (4, 4, 4, 4)
    U = qi.gauge_field(dims, 0.3, 97)
    _, info = S.solve_fp64(U, 0.12, dims, qi.point_source(dims), tol=1e-12)
    assert info.breakdown and info.iterations == 1


def test_omega_prescription_first_iteration_by_hand():
    # Alg. 4's omega clause: a 2 x 2 complex system whose first omega^ is
    # 1/sqrt(5) < 0.7, so the prescription acts with omega0 = 0.7 and not with
    # omega0 = 0.4 or 0; the first iterate and residual norm against the values
    # derived by hand in golden/omega0_first_iteration.txt
    A = np.array([[1, 2], [1, 1j]])
    b = np.array([1, 0], dtype=complex)
    rows = []
    with open(os.path.join(GOLDEN, "omega0_first_iteration.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                w0, *vals = line.split()
                rows.append((float(w0), [complex(v) for v in vals]))
    assert [w0 for w0, _ in rows] == [0.7, 0.4, 0.0]
    for w0, (x0, x1, r0, r1) in rows:
        x, info = S.bicgstab(lambda v: A @ v, b, S.FP64, tol2=0.0, maxiter=1, omega0=w0)
        assert info.iterations == 1
        assert abs(x[0] - x0) < 1e-15 and abs(x[1] - x1) < 1e-15, (w0, x)
        assert abs(info.history[1] - (abs(r0) ** 2 + abs(r1) ** 2)) < 1e-15, (w0, info.history)
    # the two forms differ, so a rule that never fires (or always fires) fails one row
    assert abs(rows[0][1][1] - rows[1][1][1]) > 0.1
