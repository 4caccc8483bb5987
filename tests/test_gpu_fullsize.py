"""The benchmark's workloads at their full sizes, in the configurations the
benchmark times, checked against the oracle.

* the headline: 32^3 x 64, eps = 0.3, kappa = 0.124, the Gaussian source of
  seed 202, FP16-inner refinement (s = 128, sigma = 64) on the even-odd system;
  the oracle's |b - D x| / |b| of the returned x, and x against the oracle's
  own solution x* (its FP64 BiCGStab on eq. (5) to 1e-14, then eq. (6)),
  as are the FP32-inner refinement and the FP64 BiCGStab of the library;
* the 12 spin-colour point sources at the origin in one batched even-odd call
  with graph replay;
* the mixed batch 16^4 + 24^3 x 48 + 32^3 x 64 with 4 Gaussian sources each.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import qcd_inputs as qi  # noqa: E402
from oracle import evenodd as EO  # noqa: E402
from gpu_common import to_dev, to_host  # noqa: E402

DIMS = (32, 32, 32, 64)
KAPPA = 0.124


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2602_14450_amd as q
    return q


@pytest.fixture(scope="module")
def field(q):
    U = qi.gauge_field(DIMS, 0.3, 201)
    g = q.gauge_upload(to_dev(U), DIMS)
    yield U, g
    g.close()
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def xstar(field):
    """The oracle's x* for the headline source: FP64 BiCGStab on the even-odd
    system to a relative residual of 1e-14, then the odd half (about 40 s on
    16 host cores)."""
    U, _ = field
    b = qi.gaussian_source(DIMS, 202)
    print("[fullsize] oracle x* at 32^3 x 64 ...", flush=True)
    xs, info = EO.solve_fp64(U, KAPPA, DIMS, b, tol=1e-14)
    assert info.converged
    res = oracle_rel_res(U, xs, b, DIMS, KAPPA)
    assert res <= 2e-14, res
    return b, xs


def oracle_rel_res(U, x, b, dims, kappa):
    return np.linalg.norm(b - oracle.dslash(U, x, kappa, dims)) / np.linalg.norm(b)


@pytest.mark.parametrize("inner_tol", [1e-2, 1e-3])  # the paper's eps_tol^2 = 1e-4, and the benchmark's
def test_headline_even_odd(q, field, xstar, inner_tol):
    U, g = field
    b, xs = xstar
    bd = to_dev(b)
    x = torch.zeros_like(bd)
    info = q.solve_mixed_ir(g, KAPPA, x, bd, inner_prec=q.FP16, s=128.0, sigma=64.0, tol=1e-12, inner_tol=inner_tol,
                            even_odd=True)
    assert info.status == "ok" and info.true_rel_residual <= 1e-12
    xh = to_host(x)
    res = oracle_rel_res(U, xh, b, DIMS, KAPPA)
    assert res <= 1.01e-12 and abs(res - info.true_rel_residual) <= 1e-3 * res
    # x within 1e-10 of the oracle's solution
    err = np.linalg.norm(xh - xs) / np.linalg.norm(xs)
    assert err <= 1e-10, err
    x64 = torch.zeros_like(bd)
    i64 = q.bicgstab(g, KAPPA, x64, bd, prec=q.FP64, tol=1e-12, even_odd=True)
    assert i64.true_rel_residual <= 1e-12
    assert np.linalg.norm(to_host(x64) - xs) <= 1e-10 * np.linalg.norm(xs)
    # the iteration count stays within 20% of the FP64 solver's (the paper's claim)
    assert 2 * info.inner_iters <= 1.2 * 2 * i64.inner_iters + 4


def test_fp32_inner_and_full_matrix_against_oracle_solution(q, field, xstar):
    # the FP32-inner refinement (Alg. 2, s = 1) on the even-odd system and the
    # FP16-inner refinement on the full matrix reach the oracle's x* as well
    U, g = field
    b, xs = xstar
    bd = to_dev(b)
    for kw in (dict(inner_prec=q.FP32, s=1.0, recalc_shat=False, sigma=0.0, even_odd=True),
               dict(inner_prec=q.FP16, s=128.0, sigma=64.0, even_odd=False)):
        x = torch.zeros_like(bd)
        info = q.solve_mixed_ir(g, KAPPA, x, bd, tol=1e-12, inner_tol=1e-2, **kw)
        assert info.status == "ok" and info.true_rel_residual <= 1e-12, kw
        xh = to_host(x)
        assert np.linalg.norm(xh - xs) <= 1e-10 * np.linalg.norm(xs), kw
        assert oracle_rel_res(U, xh, b, DIMS, KAPPA) <= 1.01e-12, kw


def test_twelve_point_sources_even_odd(q, field):
    U, g = field
    bs = np.stack([qi.point_source(DIMS, sp, c) for sp in range(4) for c in range(3)])
    b = to_dev(bs)
    x = torch.zeros_like(b)
    infos = q.solve_mixed_ir(g, KAPPA, x, b, inner_prec=q.FP16, s=128.0, sigma=64.0, tol=1e-12, even_odd=True,
                             use_graph=True, inner_tol=1e-3)
    for i in infos:
        assert i.status == "ok" and i.true_rel_residual <= 1e-12
    for r in (0, 5, 11):
        assert oracle_rel_res(U, to_host(x[r]), bs[r], DIMS, KAPPA) <= 1.01e-12
    del b, x
    torch.cuda.empty_cache()


def test_mixed_batch(q):
    specs = [((16, 16, 16, 16), 301), ((24, 24, 24, 48), 302), ((32, 32, 32, 64), 303)]
    Us, gauges, bs, xs = [], [], [], []
    for dims, seed in specs:
        U = qi.gauge_field(dims, 0.3, seed)
        Us.append(U)
        gauges.append(q.gauge_upload(to_dev(U), dims))
        bs.append(qi.gaussian_source(dims, seed + 1000, nrhs=4))
        xs.append(torch.zeros(bs[-1].shape, dtype=torch.complex128, device="cuda"))
    infos = q.solve_mixed_ir_batched(gauges, [KAPPA] * 3, xs, [to_dev(b) for b in bs], inner_prec=q.FP16,
                                     s=128.0, sigma=64.0, tol=1e-12, even_odd=True, use_graph=True,
                                     inner_tol=1e-3)
    for (dims, _), U, b, x, lat in zip(specs, Us, bs, xs, infos):
        for i in lat:
            assert i.status == "ok" and i.true_rel_residual <= 1e-12
        xh = to_host(x)
        for r in (0, 3):
            assert oracle_rel_res(U, xh[r], b[r], dims, KAPPA) <= 1.01e-12, dims
    for g in gauges:
        g.close()
    torch.cuda.empty_cache()
