"""Even-odd form (eq. (4)-(6)) on the GPU against oracle/evenodd.py, through the C ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import qcd_inputs as qi  # noqa: E402
from oracle import evenodd as EO  # noqa: E402
from gpu_common import TOL, compare, to_dev, to_host  # noqa: E402


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2602_14450_amd as q
    return q


# (4,6,8,10): 960 half sites, a ragged last 256-site block; (8,8,8,8): whole blocks
SHAPES = [(4, 6, 8, 10), (8, 8, 8, 8), (2, 4, 6, 8)]


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_schur_operator_matches_oracle(q, dims, prec):
    kappa = 0.124
    U = qi.gauge_field(dims, 0.3, 700 + sum(dims))
    psi = qi.gaussian_source(dims, 701, nrhs=2)
    e = EO.even_mask(dims)
    g = q.gauge_upload(to_dev(U), dims)
    out = torch.empty(psi.shape, dtype=torch.complex128, device="cuda")
    q.dslash(g, kappa, out, to_dev(psi), op=q.OP_SCHUR, prec=prec)
    torch.cuda.synchronize()
    got = to_host(out)
    for r in range(2):
        want = EO.schur(U, psi[r], kappa, dims)
        assert not np.any(got[r][~e])
        compare(got[r][e], want[e], TOL[prec], f"schur dims={dims} prec={prec} rhs={r}")
    g.close()


def test_bicgstab_even_odd_fp64(q):
    dims = (8, 8, 8, 8)
    kappa = 0.12
    U = qi.gauge_field(dims, 0.3, 710)
    b = qi.gaussian_source(dims, 711)
    x_ref, info_ref = EO.solve_fp64(U, kappa, dims, b, tol=1e-13)
    g = q.gauge_upload(to_dev(U), dims)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    info = q.bicgstab(g, kappa, x, to_dev(b), prec=q.FP64, tol=1e-12, even_odd=True)
    assert info.status == "ok" and info.true_rel_residual <= 1.5e-12
    assert np.linalg.norm(to_host(x) - x_ref) <= 1e-10 * np.linalg.norm(x_ref)
    full = q.bicgstab(g, kappa, torch.zeros_like(x), to_dev(b), prec=q.FP64, tol=1e-12)
    assert info.inner_iters < full.inner_iters
    assert abs(info.inner_iters - info_ref.iterations) <= 1
    g.close()


@pytest.mark.parametrize("inner_prec", [1, 2, 3])
def test_refinement_even_odd(q, inner_prec):
    dims = (8, 8, 8, 8)
    kappa = 0.12
    U = qi.gauge_field(dims, 0.3, 720)
    bs = qi.gaussian_source(dims, 721, nrhs=3)
    bs[1] = 0.0
    g = q.gauge_upload(to_dev(U), dims)
    b = to_dev(bs)
    x = torch.zeros_like(b)
    infos = q.solve_mixed_ir(g, kappa, x, b, inner_prec=inner_prec, tol=1e-12, even_odd=True)
    xh = to_host(x)
    full = q.solve_mixed_ir(g, kappa, torch.zeros_like(b), b, inner_prec=inner_prec, tol=1e-12)
    for r in (0, 2):
        assert infos[r].true_rel_residual <= 1e-12
        res = bs[r] - oracle.dslash(U, xh[r], kappa, dims)
        assert np.linalg.norm(res) <= 1.01e-12 * np.linalg.norm(bs[r])
        x_ref, _ = EO.solve_fp64(U, kappa, dims, bs[r], tol=1e-13)
        assert np.linalg.norm(xh[r] - x_ref) <= 1e-10 * np.linalg.norm(x_ref)
        assert infos[r].inner_iters < full[r].inner_iters
    assert not np.any(xh[1]) and infos[1].true_rel_residual == 0.0
    g.close()


def test_even_odd_graph_replay_and_batched_lattices(q):
    specs = [((8, 8, 8, 8), 0.12, 730), ((4, 6, 8, 10), 0.124, 731)]
    gauges, bs = [], []
    for dims, k, seed in specs:
        gauges.append(q.gauge_upload(to_dev(qi.gauge_field(dims, 0.3, seed)), dims))
        bs.append(to_dev(qi.gaussian_source(dims, seed + 1, nrhs=2)))
    single = []
    for g, (dims, k, _), b in zip(gauges, specs, bs):
        xs = []
        for use_graph in (False, True):
            x = torch.zeros_like(b)
            q.solve_mixed_ir(g, k, x, b, inner_prec=q.FP16, tol=1e-12, even_odd=True, use_graph=use_graph)
            xs.append(x)
        assert torch.equal(xs[0], xs[1])
        single.append(xs[0])
    xb = [torch.zeros_like(b) for b in bs]
    q.solve_mixed_ir_batched(gauges, [s[1] for s in specs], xb, bs, inner_prec=q.FP16, tol=1e-12, even_odd=True,
                             use_graph=True)
    for a, b in zip(xb, single):
        assert torch.equal(a, b)
    for g in gauges:
        g.close()


# The network preconditions eq. (5) through its even-even block (the even rows
# of M (v, 0)); with the third-order Neumann weights that block is
# 1 + kappa^2 H_eo H_oe, so the inner solve needs fewer iterations, and every
# solve must still reach the oracle's x*.
@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (4, 6, 8, 10)])
def test_even_odd_refinement_with_network(q, dims):
    kappa = 0.124
    U = qi.gauge_field(dims, 0.3, 740)
    bs = qi.gaussian_source(dims, 741, nrhs=3)
    bs[1] *= 1e-3          # different norms in one batch
    g = q.gauge_upload(to_dev(U), dims)
    net = q.PTC(g, (1, 2, 2, 1), max_batch=3)
    net.init_neumann(kappa)
    b = to_dev(bs)
    runs = []
    for use_graph in (False, True):
        x = torch.zeros_like(b)
        infos = q.solve_mixed_ir(g, kappa, x, b, inner_prec=q.FP16, tol=1e-12, precond=net, even_odd=True,
                                 use_graph=use_graph)
        runs.append((x, infos))
    plain = q.solve_mixed_ir(g, kappa, torch.zeros_like(b), b, inner_prec=q.FP16, tol=1e-12, even_odd=True)
    assert torch.equal(runs[0][0], runs[1][0])
    xh = to_host(runs[0][0])
    steps = max(info.outer_iters for info in runs[0][1])   # the network's step count is the call's
    for r in range(3):
        info = runs[0][1][r]
        assert info.status == "ok" and info.true_rel_residual <= 1e-12
        assert runs[1][1][r].inner_iters == info.inner_iters
        assert info.precond_fallback == -1 and info.precond_steps == steps and info.precond_scale > 0
        res = bs[r] - oracle.dslash(U, xh[r], kappa, dims)
        assert np.linalg.norm(res) <= 1.01e-12 * np.linalg.norm(bs[r])
        x_ref, _ = EO.solve_fp64(U, kappa, dims, bs[r], tol=1e-13)
        assert np.linalg.norm(xh[r] - x_ref) <= 1e-10 * np.linalg.norm(x_ref)
        assert info.inner_iters < plain[r].inner_iters, (r, info.inner_iters, plain[r].inner_iters)
    net.close()
    g.close()


def test_even_odd_zero_network_falls_back(q):
    # M = 0 breaks the first inner solve down; the step is undone (x_e restored,
    # the even residual recomputed) and the call finishes with the plain solver
    dims = (4, 6, 8, 10)
    kappa = 0.124
    U = qi.gauge_field(dims, 0.3, 742)
    b = qi.gaussian_source(dims, 743)
    g = q.gauge_upload(to_dev(U), dims)
    net = q.PTC(g, (1, 2, 2, 1), max_batch=1)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    info = q.solve_mixed_ir(g, kappa, x, to_dev(b), inner_prec=q.FP16, tol=1e-12, precond=net, even_odd=True)
    assert info.status == "ok" and info.true_rel_residual <= 1e-12
    assert info.precond_fallback == 0 and info.precond_steps == 0
    x_ref, _ = EO.solve_fp64(U, kappa, dims, b, tol=1e-13)
    assert np.linalg.norm(to_host(x) - x_ref) <= 1e-10 * np.linalg.norm(x_ref)
    res = b - oracle.dslash(U, to_host(x), kappa, dims)
    assert np.linalg.norm(res) <= 1.01e-12 * np.linalg.norm(b)
    # a caller workspace of the size the library reports for it (what = 3 + 8)
    # gives the same solve; one byte less is refused before any launch
    need = g.workspace_bytes(3 | 8, q.FP16, 1000, 1)
    assert need > g.workspace_bytes(8, q.FP16, 1000, 1)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    x2 = torch.zeros_like(x)
    info2 = q.solve_mixed_ir(g, kappa, x2, to_dev(b), inner_prec=q.FP16, tol=1e-12, precond=net, even_odd=True,
                             inner_max_iter=1000, workspace=ws)
    assert torch.equal(x, x2) and info2.inner_iters == info.inner_iters
    with pytest.raises(q.QcdError):
        q.solve_mixed_ir(g, kappa, torch.zeros_like(x), to_dev(b), inner_prec=q.FP16, tol=1e-12, precond=net,
                         even_odd=True, inner_max_iter=1000, workspace=ws[:need - 1])
    net.close()
    g.close()


@pytest.mark.parametrize("fp64_tile", [2, -2])
def test_even_odd_refinement_with_fp64_tiles(q, fp64_tile):
    # the final residual of the even-odd solve sums two launches with different
    # partial-sum layouts when the FP64 operator runs with a lane or register
    # tile; the reported residual must still be the oracle's |b - D x| / |b|
    dims = (4, 6, 8, 10)
    kappa = 0.124
    U = qi.gauge_field(dims, 0.3, 750)
    bs = qi.gaussian_source(dims, 751, nrhs=4)
    bs[2] = 0.0
    g = q.gauge_upload(to_dev(U), dims)
    g.set_tuning(q.FP64, 1, 0, fp64_tile)
    b = to_dev(bs)
    x = torch.zeros_like(b)
    infos = q.solve_mixed_ir(g, kappa, x, b, inner_prec=q.FP16, tol=1e-12, even_odd=True)
    xh = to_host(x)
    for r in (0, 1, 3):
        res = np.linalg.norm(bs[r] - oracle.dslash(U, xh[r], kappa, dims)) / np.linalg.norm(bs[r])
        assert infos[r].true_rel_residual <= 1e-12 and res <= 1.01e-12
        assert abs(infos[r].true_rel_residual - res) <= 1e-3 * res + 1e-16
    assert not np.any(xh[2]) and infos[2].true_rel_residual == 0.0
    g.close()


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_even_odd_bicgstab_low_precision_several_sources(q, prec):
    # qcd_bicgstab on the even-odd system in a storage precision, several
    # right-hand sides (one zero) on a lattice with a ragged last block: the
    # reported full residual is the oracle's, and it meets the requested
    # tolerance relative to |b'| up to the precision's floor
    dims = (4, 6, 8, 10)
    kappa = 0.124
    U = qi.gauge_field(dims, 0.3, 760)
    bs = qi.gaussian_source(dims, 761, nrhs=3)
    bs[1] = 0.0
    g = q.gauge_upload(to_dev(U), dims)
    b = to_dev(bs)
    x = torch.zeros_like(b)
    tol = {1: 1e-5, 2: 1e-2, 3: 5e-2}[prec]
    infos = q.bicgstab(g, kappa, x, b, prec=prec, tol=tol, even_odd=True, raise_on_error=False)
    xh = to_host(x)
    for r in (0, 2):
        res = np.linalg.norm(bs[r] - oracle.dslash(U, xh[r], kappa, dims)) / np.linalg.norm(bs[r])
        assert abs(infos[r].true_rel_residual - res) <= 1e-6 * res + 1e-15
        assert res <= 20 * tol
    assert not np.any(xh[1])
    g.close()


# Lattices where blocks of 256 half sites of one parity cover whole x rows, so
# that the one-parity launches take the LDS-staged form (launch variants 6
# and 7): the y halo rows wrap onto the block's own rows when R = Ly and come
# from the neighbouring block's rows otherwise; the XCD-slab schedules apply
# on the second and third; (128, 4, 2, 2) has the longest rows the 16-bit and
# FP32 forms take (FP64 falls back there), (4, 6, 8, 10) takes the plain form.
LDS_EO_SHAPES = [(16, 64, 2, 4), (32, 32, 8, 2), (64, 16, 2, 8), (128, 4, 2, 2), (4, 6, 8, 10)]
# (plain variant, LDS variant) per precision: the LDS variant falls back to the plain one
LDS_PAIRS = {0: (0, 7), 1: (1, 6), 2: (1, 6), 3: (1, 6)}
UNIT = {0: 2.0 ** -52, 1: 2.0 ** -23, 2: 2.0 ** -10, 3: 2.0 ** -7}


@pytest.mark.parametrize("dims", LDS_EO_SHAPES)
@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_lds_staged_schur_operator(q, dims, prec):
    # the Schur operator (two one-parity launches, the intermediate rounded to
    # storage) with the LDS variant against the plain one, element by element,
    # and against the oracle: the hops are the same products in the same
    # order, so the two differ only where the compiler fuses a sum
    # differently: in 16-bit storage a unit of the format in rare elements
    # (which the second hop can carry into a second unit), in FP32 and FP64 a
    # few units of the sums' terms
    kappa = 0.124
    U = qi.gauge_field(dims, 0.3, 760 + sum(dims))
    psi = qi.gaussian_source(dims, 761)
    e = EO.even_mask(dims)
    want = EO.schur(U, psi, kappa, dims)
    g = q.gauge_upload(to_dev(U), dims, precs=(q.FP64, prec) if prec else (q.FP64,))
    unit = UNIT[prec]
    plain, lds = LDS_PAIRS[prec]
    ref = torch.empty(psi.shape, dtype=torch.complex128, device="cuda")
    got = torch.empty_like(ref)
    for sched in (0, 1, 4):
        g.set_tuning(prec, sched, plain, 1)
        q.dslash(g, kappa, ref, to_dev(psi), op=q.OP_SCHUR, prec=prec)
        g.set_tuning(prec, sched, lds, 1)
        q.dslash(g, kappa, got, to_dev(psi), op=q.OP_SCHUR, prec=prec)
        torch.cuda.synchronize()
        r, v = to_host(ref).reshape(-1), to_host(got).reshape(-1)
        rms = np.sqrt(np.mean(np.abs(r) ** 2))
        for part in (np.real, np.imag):
            d = np.abs(part(v) - part(r))
            if prec >= 2:
                assert np.all(d <= 2 * unit * np.abs(part(r)) + 1e-30), (dims, prec, sched, d.max())
            else:
                assert np.all(d <= 16 * unit * rms), (dims, prec, sched, d.max() / rms)
        if prec >= 2:
            assert np.mean(r != v) <= 1e-2, (dims, prec, sched, np.mean(r != v))
        gv = to_host(got)
        assert not np.any(gv[~e])
        compare(gv[e], want[e], TOL[prec], f"lds schur dims={dims} prec={prec} sched={sched}")
    g.close()


@pytest.mark.parametrize("inner_prec", [1, 2])
def test_lds_staged_even_odd_refinement(q, inner_prec):
    # the even-odd refinement on a lattice where its one-parity launches (the
    # inner ones and the FP64 residual's) take the LDS form, against the
    # oracle's x* and against the plain launches (iteration counts within one
    # of each other); FP16 inner with and without graph replay
    dims = (32, 32, 8, 2)
    kappa = 0.124
    U = qi.gauge_field(dims, 0.3, 770)
    bs = qi.gaussian_source(dims, 771)
    x_ref, _ = EO.solve_fp64(U, kappa, dims, bs, tol=1e-13)
    g = q.gauge_upload(to_dev(U), dims)
    b = to_dev(bs)
    iters = {}
    for form in (0, 1):
        g.set_tuning(inner_prec, 1, LDS_PAIRS[inner_prec][form], 1)
        g.set_tuning(q.FP64, 1, LDS_PAIRS[0][form], 1)
        for graph in ((False, True) if inner_prec == 2 else (False,)):
            x = torch.zeros_like(b)
            info = q.solve_mixed_ir(g, kappa, x, b, inner_prec=inner_prec, tol=1e-12, inner_tol=1e-3,
                                    even_odd=True, use_graph=graph,
                                    s=128.0 if inner_prec == 2 else 1.0, sigma=64.0 if inner_prec == 2 else 0.0)
            assert info.status == "ok" and info.true_rel_residual <= 1e-12, (form, graph, info)
            xh = to_host(x)
            assert np.linalg.norm(xh - x_ref) <= 1e-10 * np.linalg.norm(x_ref), (form, graph)
            iters[(form, graph)] = info.inner_iters
    assert abs(iters[(1, False)] - iters[(0, False)]) <= 1, iters
    if inner_prec == 2:
        assert iters[(1, True)] == iters[(1, False)], iters
    g.close()
