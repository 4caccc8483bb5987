"""Parity of the HIP solvers with the CPU oracle (through the C ABI).

* FP64 BiCGStab: solution within 1e-10 of the oracle's x* and a true FP64
  residual <= 1e-12; the rescaled variants of Alg. 4/5 follow the oracle's
  iterates step by step in FP64 (pins the device-side bookkeeping).
* Mixed-precision refinement (FP32, FP16 and BF16 inner, each rescaling
  variant of Table 2): true residual <= 1e-12 and x within 1e-10 of the oracle's.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import qcd_inputs as qi  # noqa: E402
from oracle import solvers as S  # noqa: E402
from gpu_common import compare, fields, to_dev, to_host  # noqa: E402


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2602_14450_amd as q
    return q


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def true_res(U, k, dims, x, b):
    return np.linalg.norm(b - oracle.dslash(U, x, k, dims)) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def c1(q):
    dims = (8, 8, 8, 8)
    k = 0.12
    U, b = fields(dims, gseed=101, sseed=102)
    xs, info = S.solve_fp64(U, k, dims, b, tol=1e-14)
    assert info.converged
    g = q.gauge_upload(to_dev(U), dims)
    yield dict(dims=dims, k=k, U=U, b=b, xs=xs, g=g)
    g.close()


def test_fp64_bicgstab_solution(q, c1):
    x = torch.zeros(c1["b"].shape, dtype=torch.complex128, device="cuda")
    info = q.bicgstab(c1["g"], c1["k"], x, to_dev(c1["b"]), prec=q.FP64, tol=1e-12)
    xh = to_host(x)
    assert info.status == "ok"
    assert info.true_rel_residual <= 1e-12
    assert true_res(c1["U"], c1["k"], c1["dims"], xh, c1["b"]) <= 1e-12
    assert rel(xh, c1["xs"]) < 1e-10


@pytest.mark.parametrize("variant", [dict(), dict(sigma=64.0, recalc_gamma=True),
                                     dict(sigma=64.0, recalc_gamma=False),
                                     dict(sigma=256.0, recalc_gamma=True, sigma_lambda=256.0)])
def test_fp64_trajectory_matches_oracle(q, c1, variant):
    k_it = 7
    A = lambda v: oracle.dslash(c1["U"], v, c1["k"], c1["dims"])
    xo, io = S.bicgstab(A, c1["b"], S.FP64, tol2=0.0, maxiter=k_it, **variant)
    x = torch.zeros(c1["b"].shape, dtype=torch.complex128, device="cuda")
    info = q.bicgstab(c1["g"], c1["k"], x, to_dev(c1["b"]), prec=q.FP64, tol=0.0, max_iter=k_it,
                      check_every=1, **variant)
    assert info.status == "not_converged" and info.inner_iters == k_it
    assert rel(to_host(x), xo) < 1e-11
    # unscaled residual history, relative to |b|^2
    bn2 = S.norm2(c1["b"])
    np.testing.assert_allclose(np.array(info.history), np.array(io.history[1:]) / bn2, rtol=1e-8)


@pytest.mark.parametrize("cfg", [
    dict(inner_prec=1, s=1.0, recalc_shat=False, sigma=0.0),                 # Alg. 2 + Alg. 4, gamma = 1
    dict(inner_prec=2, s=128.0, recalc_shat=True, sigma=64.0),               # Alg. 3 + Alg. 4
    dict(inner_prec=2, s=4096.0, recalc_shat=True, sigma=0.0),               # outer rescaling only
    dict(inner_prec=2, s=128.0, recalc_shat=True, sigma=256.0, sigma_lambda=256.0),  # Alg. 3 + Alg. 5
    dict(inner_prec=2, s=128.0, recalc_shat=True, sigma=64.0, recalc_gamma=False),
    dict(inner_prec=2, s=1.0, recalc_shat=False, sigma=0.0),                 # no rescaling at all
    dict(inner_prec=3, s=1.0, recalc_shat=False, sigma=0.0),                 # BF16 inner, no rescaling
    dict(inner_prec=3, s=128.0, recalc_shat=True, sigma=64.0),               # BF16 inner, Alg. 3 + Alg. 4
])
def test_mixed_ir(q, c1, cfg):
    x = torch.zeros(c1["b"].shape, dtype=torch.complex128, device="cuda")
    info = q.solve_mixed_ir(c1["g"], c1["k"], x, to_dev(c1["b"]), tol=1e-12, inner_tol=1e-2, **cfg)
    _check_mixed(c1, cfg, x, info)


@pytest.mark.parametrize("inner_tol", [1e-4, 1e-3])
def test_mixed_ir_other_inner_tolerances(q, c1, inner_tol):
    # the FP32-inner form with |r| <= 1e-4 |b| per inner solve (the small
    # configuration's inner tolerance read literally rather than as eps_tol^2),
    # and the FP16 form at the benchmark's 1e-3
    for cfg in (dict(inner_prec=1, s=1.0, recalc_shat=False, sigma=0.0),
                dict(inner_prec=2, s=128.0, recalc_shat=True, sigma=64.0)):
        x = torch.zeros(c1["b"].shape, dtype=torch.complex128, device="cuda")
        info = q.solve_mixed_ir(c1["g"], c1["k"], x, to_dev(c1["b"]), tol=1e-12, inner_tol=inner_tol, **cfg)
        _check_mixed(c1, cfg, x, info)


def _check_mixed(c1, cfg, x, info):
    xh = to_host(x)
    assert info.status == "ok", info
    assert info.true_rel_residual <= 1e-12
    assert true_res(c1["U"], c1["k"], c1["dims"], xh, c1["b"]) <= 1e-12
    assert rel(xh, c1["xs"]) < 1e-10
    if cfg.get("recalc_shat"):   # s^ is the norm of the stored (rounded) vector
        assert abs(info.first_shat_over_s - 1) < (2.0 ** -10 if cfg["inner_prec"] == 2 else 2.0 ** -8)


def test_zero_rhs(q, c1):
    b = torch.zeros(c1["b"].shape, dtype=torch.complex128, device="cuda")
    x = torch.ones_like(b)
    info = q.solve_mixed_ir(c1["g"], c1["k"], x, b)
    assert info.status == "ok" and info.outer_iters == 0
    assert torch.count_nonzero(x) == 0


def test_max_outer_gives_not_converged_with_valid_x(q, c1):
    x = torch.zeros(c1["b"].shape, dtype=torch.complex128, device="cuda")
    info = q.solve_mixed_ir(c1["g"], c1["k"], x, to_dev(c1["b"]), max_outer=1)
    assert info.status == "not_converged" and info.outer_iters == 1
    r = true_res(c1["U"], c1["k"], c1["dims"], to_host(x), c1["b"])
    assert abs(r - info.true_rel_residual) < 1e-6 * r and r < 0.05


def test_point_source_breakdown_reported(q):
    # r* = r = e_0 on the full operator breaks down in iteration 2
    dims = (4, 4, 4, 4)
    U = qi.gauge_field(dims, 0.3, 97)
    g = q.gauge_upload(to_dev(U), dims)
    b = to_dev(qi.point_source(dims))
    x = torch.zeros_like(b)
    info = q.bicgstab(g, 0.12, x, b, prec=q.FP64, tol=1e-12, raise_on_error=False, check_every=1)
    assert info.status == "err_breakdown" and info.inner_iters == 1
    g.close()


def test_full_size_fp16_refinement(q):
    # The benchmark workload: 32^3 x 64, eps = 0.3, kappa = 0.124, one
    # Gaussian source, FP16 inner with s = 128, sigma = 64.  The true
    # residual is re-checked with the oracle's operator on the host.
    dims = (32, 32, 32, 64)
    k = 0.124
    U, b = fields(dims, gseed=201, sseed=202)
    g = q.gauge_upload(to_dev(U), dims)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    info = q.solve_mixed_ir(g, k, x, to_dev(b), inner_prec=q.FP16, s=128.0, sigma=64.0, tol=1e-12)
    assert info.status == "ok" and info.true_rel_residual <= 1e-12
    xh = to_host(x)
    assert true_res(U, k, dims, xh, b) <= 1.05e-12
    x64 = torch.zeros_like(x)
    i64 = q.bicgstab(g, k, x64, to_dev(b), prec=q.FP64, tol=1e-12)
    assert i64.true_rel_residual <= 1.05e-12
    assert rel(xh, to_host(x64)) < 1e-10
    g.close()
