"""Several right-hand sides at once: the multi-RHS Wilson operator (links read
once per site for all right-hand sides) and the batched solvers with
per-right-hand-side scalars and masks, against the CPU oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import qcd_inputs as qi  # noqa: E402
from oracle import evenodd as EO  # noqa: E402
from oracle import solvers as S  # noqa: E402
from gpu_common import TOL, compare, to_dev, to_host  # noqa: E402


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2602_14450_amd as q
    return q


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (2, 4, 6, 10), (4, 6, 8, 10)])
@pytest.mark.parametrize("nrhs", [2, 3, 4, 12])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_multi_rhs_dslash(q, dims, nrhs, prec):
    U = qi.gauge_field(dims, 0.3, 31 + nrhs)
    psi = qi.gaussian_source(dims, 32, nrhs=nrhs)
    g = q.gauge_upload(to_dev(U), dims)
    x = to_dev(psi)
    out = torch.empty_like(x)
    for op in (0, 2):
        q.dslash(g, 0.124, out, x, op=op, prec=prec, layout=q.CANONICAL)
        torch.cuda.synchronize()
        got = to_host(out)
        for r in range(nrhs):
            compare(got[r], oracle.dslash(U, psi[r], 0.124, dims, op), TOL[prec], f"{dims} n={nrhs} rhs={r} op={op}")
    g.close()


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (2, 4, 6, 10), (4, 6, 8, 10), (2, 2, 2, 2)])
@pytest.mark.parametrize("nrhs", [4, 6, 8, 12, 16])
def test_matrix_core_multi_rhs_dslash(q, dims, nrhs):
    # the matrix-core form of the FP16 operator (rhs_tile 8: tiles of 4, 6, 8,
    # 12 or 16 right-hand sides, one or two instructions per hop) against the
    # oracle, all four operators; ragged volumes (an odd number of site pairs
    # per block of four) and the 2^4 lattice where x + mu and x - mu coincide
    U = qi.gauge_field(dims, 0.3, 131 + nrhs)
    psi = qi.gaussian_source(dims, 132, nrhs=nrhs)
    g = q.gauge_upload(to_dev(U), dims)
    g.set_tuning(q.FP16, 0, 0, 8)
    x = to_dev(psi)
    out = torch.empty_like(x)
    for op in (0, 1, 2, 3):
        q.dslash(g, 0.124, out, x, op=op, prec=q.FP16, layout=q.CANONICAL)
        torch.cuda.synchronize()
        got = to_host(out)
        for r in range(nrhs):
            compare(got[r], oracle.dslash(U, psi[r], 0.124, dims, op), TOL[2], f"mfma {dims} n={nrhs} rhs={r} op={op}")
    g.close()


def test_matrix_core_form_at_full_size_on_sampled_sites(q):
    # 12 right-hand sides at 32^3 x 64, the benchmark's batched operator, with
    # the matrix-core form: sampled output sites against the oracle's operator
    dims = (32, 32, 32, 64)
    V = qi.volume(dims)
    U = qi.gauge_field(dims, 0.3, 201)
    psi = qi.gaussian_source(dims, 141, nrhs=12)
    g = q.gauge_upload(to_dev(U), dims, precs=(q.FP64, q.FP16))
    g.set_tuning(q.FP16, 0, 0, 8)
    x = to_dev(psi)
    out = torch.empty_like(x)
    q.dslash(g, 0.124, out, x, op=0, prec=q.FP16, layout=q.CANONICAL)
    torch.cuda.synchronize()
    rng = np.random.default_rng(142)
    sites = np.concatenate([[0, 1, V - 1], rng.integers(0, V, 200)])
    got = to_host(out)
    for r in (0, 5, 11):
        want = oracle.dslash_sites(U, psi[r], 0.124, dims, sites)
        compare(got[r][sites], want, TOL[2], f"mfma 32^3x64 rhs={r}")
    del x, out
    g.close()
    torch.cuda.empty_cache()


def test_matrix_core_form_in_the_even_odd_batched_solve(q):
    # with rhs_tile 8 the hop-only one-parity launches of a batched even-odd
    # solve take the matrix-core form: every true residual still meets 1e-12
    dims, k = (8, 8, 8, 8), 0.12
    U = qi.gauge_field(dims, 0.3, 151)
    b = qi.gaussian_source(dims, 152, nrhs=8)
    g = q.gauge_upload(to_dev(U), dims)
    g.set_tuning(q.FP16, 0, 0, 8)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    infos = q.solve_mixed_ir(g, k, x, to_dev(b), inner_prec=q.FP16, s=128.0, sigma=64.0, tol=1e-12, even_odd=True,
                             use_graph=True)
    xh = to_host(x)
    for r in range(8):
        assert infos[r].status == "ok" and infos[r].true_rel_residual <= 1e-12
        res = np.linalg.norm(b[r] - oracle.dslash(U, xh[r], k, dims)) / np.linalg.norm(b[r])
        assert res <= 1.01e-12, (r, res)
    g.close()


@pytest.mark.parametrize("dims", [(8, 16, 32, 4), (8, 32, 8, 16)])
@pytest.mark.parametrize("rhs_tile", [1, 2, 4, -2, -4])
def test_rhs_tile_choices_agree_bitwise(q, rhs_tile, dims):
    # every launch shape (schedule incl. the sub-slab and t-slab orders,
    # right-hand-side tile) gives bit-identical output
    U = qi.gauge_field(dims, 0.3, 41)
    psi = qi.gaussian_source(dims, 42, nrhs=4)
    g = q.gauge_upload(to_dev(U), dims)
    x = to_dev(psi)
    ref = torch.empty_like(x)
    g.set_tuning(q.FP16, 0, 0, 1)
    q.dslash(g, 0.124, ref, x, prec=q.FP16)
    out = torch.empty_like(x)
    for sched in (0, 1, 2, 3, 4):
        g.set_tuning(q.FP16, sched, 0, rhs_tile)
        q.dslash(g, 0.124, out, x, prec=q.FP16)
        torch.cuda.synchronize()
        if rhs_tile > 0:
            assert torch.equal(out, ref), (sched, rhs_tile)
        else:
            same_to_one_fp16_ulp(out, ref)
    g.close()


def same_to_one_fp16_ulp(out, ref):
    # A thread holding several right-hand sides evaluates the same expressions,
    # but the compiler may fuse a multiply-add differently: the FP32 sum can then
    # round to the neighbouring binary16 value (seen at 2 of 1.6e6 outputs).
    d = (out - ref).abs()
    ulp = ref.abs() * 2.0 ** -10 + 2.0 ** -24
    assert bool((d <= ulp).all())
    assert int((d > 0).sum()) <= max(4, out.numel() // 10000)


@pytest.fixture(scope="module")
def c1b(q):
    dims = (8, 8, 8, 8)
    k = 0.12
    U = qi.gauge_field(dims, 0.3, 101)
    b = qi.gaussian_source(dims, 102, nrhs=4)
    b[2] *= 1e-3                    # a small source
    b[3] = 0.0                      # a zero source: masked from the start
    xs = [S.solve_fp64(U, k, dims, b[r], tol=1e-14)[0] for r in range(3)]
    g = q.gauge_upload(to_dev(U), dims)
    yield dict(dims=dims, k=k, U=U, b=b, xs=xs, g=g)
    g.close()


def test_batched_fp64_bicgstab(q, c1b):
    x = torch.zeros(c1b["b"].shape, dtype=torch.complex128, device="cuda")
    infos = q.bicgstab(c1b["g"], c1b["k"], x, to_dev(c1b["b"]), prec=q.FP64, tol=1e-12)
    xh = to_host(x)
    for r in range(3):
        assert infos[r].inner_status == 1 and infos[r].true_rel_residual <= 1e-12
        assert rel(xh[r], c1b["xs"][r]) < 1e-10
    assert infos[3].inner_iters == 0 and np.count_nonzero(xh[3]) == 0


@pytest.mark.parametrize("inner_prec,s,sigma", [(2, 128.0, 64.0), (1, 1.0, 0.0), (2, 4096.0, 0.0)])
def test_batched_mixed_ir(q, c1b, inner_prec, s, sigma):
    x = torch.zeros(c1b["b"].shape, dtype=torch.complex128, device="cuda")
    infos = q.solve_mixed_ir(c1b["g"], c1b["k"], x, to_dev(c1b["b"]), inner_prec=inner_prec, s=s, sigma=sigma,
                             recalc_shat=(s != 1.0), tol=1e-12)
    xh = to_host(x)
    for r in range(3):
        assert infos[r].true_rel_residual <= 1e-12
        res = np.linalg.norm(c1b["b"][r] - oracle.dslash(c1b["U"], xh[r], c1b["k"], c1b["dims"])) / np.linalg.norm(
            c1b["b"][r])
        assert res <= 1e-12
        assert rel(xh[r], c1b["xs"][r]) < 1e-10
    assert infos[3].outer_iters == 0 and np.count_nonzero(xh[3]) == 0


def test_batched_matches_single(q, c1b):
    # a right-hand side solved in a batch and alone reaches the same solution
    # (partial sums are grouped differently, so agreement is to the tolerance)
    x = torch.zeros(c1b["b"].shape, dtype=torch.complex128, device="cuda")
    i4 = q.solve_mixed_ir(c1b["g"], c1b["k"], x, to_dev(c1b["b"]))
    x1 = torch.zeros(c1b["b"][1:2].shape, dtype=torch.complex128, device="cuda")
    i1 = q.solve_mixed_ir(c1b["g"], c1b["k"], x1, to_dev(c1b["b"][1:2]))
    assert abs(i4[1].inner_iters - i1.inner_iters) <= 4
    assert rel(to_host(x[1]), to_host(x1[0])) < 1e-10


def test_twelve_point_sources_full_operator(q):
    # the 12 spin-colour point sources of a propagator at the origin; the
    # first inner solve of each breaks down (r* = e_0 on the full operator)
    # and the refinement restarts from the new residual
    dims = (8, 8, 8, 8)
    k = 0.12
    U = qi.gauge_field(dims, 0.3, 101)
    b = np.stack([qi.point_source(dims, sp, c) for sp in range(4) for c in range(3)])
    g = q.gauge_upload(to_dev(U), dims)
    x = torch.zeros(b.shape, dtype=torch.complex128, device="cuda")
    infos = q.solve_mixed_ir(g, k, x, to_dev(b), inner_prec=q.FP16, s=128.0, sigma=64.0, tol=1e-12)
    xh = to_host(x)
    for r in (0, 5, 11):
        res = np.linalg.norm(b[r] - oracle.dslash(U, xh[r], k, dims)) / np.linalg.norm(b[r])
        assert infos[r].true_rel_residual <= 1e-12 and res <= 1e-12
    g.close()


def test_graph_replays_match_eager(q, c1b):
    # one BiCGStab iteration captured in a hip graph and replayed: several
    # solves in a row, with eager work and synchronisation between them, each
    # bit-identical to the eager solve
    b = to_dev(c1b["b"])
    xe = torch.zeros_like(b)
    ie = q.solve_mixed_ir(c1b["g"], c1b["k"], xe, b, use_graph=False)
    for rep in range(3):
        xg = torch.zeros_like(b)
        ig = q.solve_mixed_ir(c1b["g"], c1b["k"], xg, b, use_graph=True)
        torch.cuda.synchronize()
        assert torch.equal(xg, xe), rep
        assert [i.inner_iters for i in ig] == [i.inner_iters for i in ie]
        # unrelated eager work between replays
        y = torch.empty_like(b)
        q.dslash(c1b["g"], c1b["k"], y, b, prec=q.FP32)
        torch.cuda.synchronize()
    xb = torch.zeros_like(b[:3])
    q.bicgstab(c1b["g"], c1b["k"], xb, b[:3], prec=q.FP16, tol=1e-2, use_graph=True)
    xb2 = torch.zeros_like(b[:3])
    q.bicgstab(c1b["g"], c1b["k"], xb2, b[:3], prec=q.FP16, tol=1e-2, use_graph=False)
    torch.cuda.synchronize()
    assert torch.equal(xb, xb2)


@pytest.mark.parametrize("eo", [False, True])
def test_device_driven_steps_match_host_driven(q, c1b, eo):
    # by default the refinement steps run from the device (blocks of inner
    # iterations, each followed by one step's kernels, polled as the
    # convergence predicts; with graph replay or plain launches); with
    # check_every the host drives every step.  Solutions, counts, the
    # per-step residual and zero-count logs and s^/s are the same bit for bit
    # (sources: normal, small, zero), also on a repeated call, whose first
    # poll comes after the blocks the previous call saw
    g, k = c1b["g"], c1b["k"]
    b = to_dev(c1b["b"])
    xh = torch.zeros_like(b)
    ih = q.solve_mixed_ir(g, k, xh, b, use_graph=False, even_odd=eo, check_every=4)
    for graph in (True, False, False):
        xd = torch.zeros_like(b)
        idv = q.solve_mixed_ir(g, k, xd, b, use_graph=graph, even_odd=eo)
        torch.cuda.synchronize()
        assert torch.equal(xh, xd), graph
        for a, d in zip(ih, idv):
            assert (a.status, a.outer_iters, a.inner_iters, a.matvec_low, a.matvec_fp64) == \
                   (d.status, d.outer_iters, d.inner_iters, d.matvec_low, d.matvec_fp64)
            assert a.outer_history == d.outer_history and a.zeros == d.zeros
            assert a.first_shat_over_s == d.first_shat_over_s and a.true_rel_residual == d.true_rel_residual
    # a step cap ends both forms at the same x, reported as not converged
    xh, xd = torch.zeros_like(b), torch.zeros_like(b)
    ih = q.solve_mixed_ir(g, k, xh, b, use_graph=False, even_odd=eo, max_outer=2, raise_on_error=False,
                          check_every=4)
    idv = q.solve_mixed_ir(g, k, xd, b, use_graph=True, even_odd=eo, max_outer=2, raise_on_error=False)
    torch.cuda.synchronize()
    assert torch.equal(xh, xd)
    assert [i.status for i in idv] == [i.status for i in ih]
    assert idv[0].status == "not_converged" and idv[0].outer_iters == 2


def test_device_driven_steps_after_a_harder_call(q, c1b):
    # the first poll of a device-driven refinement takes its block sizes from
    # the handle's previous call: after a normal source, a zero source returns
    # x = 0 with no step, and a small source solves as with host-driven steps
    g, k = c1b["g"], c1b["k"]
    b = to_dev(c1b["b"][:1])
    x = torch.zeros_like(b)
    info = q.solve_mixed_ir(g, k, x, b, even_odd=True)
    assert info.status == "ok" and info.outer_iters > 1
    z = torch.zeros_like(b)
    xz = torch.ones_like(b)
    iz = q.solve_mixed_ir(g, k, xz, z, even_odd=True)
    torch.cuda.synchronize()
    assert iz.status == "ok" and iz.outer_iters == 0 and iz.inner_iters == 0
    assert not bool(xz.abs().max() > 0)
    small = to_dev(c1b["b"][2:3])
    xd, xh = torch.zeros_like(small), torch.zeros_like(small)
    idv = q.solve_mixed_ir(g, k, xd, small, even_odd=True)
    ih = q.solve_mixed_ir(g, k, xh, small, even_odd=True, check_every=4)
    torch.cuda.synchronize()
    assert torch.equal(xd, xh) and idv.inner_iters == ih.inner_iters and idv.status == "ok"


def test_graph_cache_follows_the_workspace_carve(q, c1b):
    # one handle, one caller workspace: inner_max_iter 500 and then 2000 move
    # the partial sums and scalars inside the same buffer (the history before
    # them grows), so the captured iteration must be rebuilt; each graph solve
    # is bit-identical to the eager solve with the same parameters
    g, k = c1b["g"], c1b["k"]
    b = to_dev(c1b["b"][:2])
    ws = torch.empty(g.workspace_bytes(0, q.FP16, 2000, 2), dtype=torch.uint8, device="cuda")
    for mi in (500, 2000, 500):
        xe = torch.zeros_like(b)
        ie = q.solve_mixed_ir(g, k, xe, b, inner_max_iter=mi, workspace=ws, use_graph=False)
        xg = torch.zeros_like(b)
        ig = q.solve_mixed_ir(g, k, xg, b, inner_max_iter=mi, workspace=ws, use_graph=True)
        torch.cuda.synchronize()
        assert all(i.status == "ok" for i in ig), mi
        assert torch.equal(xg, xe), mi
        assert [i.inner_iters for i in ig] == [i.inner_iters for i in ie]


def test_solves_with_caller_workspaces_allocate_nothing(q):
    # with caller-owned workspaces, a single solve, a batched solve over two
    # lattices and an FP64 BiCGStab leave the free device memory unchanged
    # (after one warm-up call of each, which may instantiate graphs)
    specs = [((8, 8, 8, 8), 0.12, 2, 611), ((4, 4, 8, 8), 0.124, 1, 612)]
    gauges, bs, xs = [], [], []
    for dims, k, n, seed in specs:
        gauges.append(q.gauge_upload(to_dev(qi.gauge_field(dims, 0.3, seed)), dims))
        bs.append(to_dev(qi.gaussian_source(dims, seed + 1000, nrhs=n)))
        xs.append(torch.zeros_like(bs[-1]))
    kappas = [s[1] for s in specs]
    for eo in (False, True):
        for use_graph in (False, True):
            what = 8 if eo else 0
            ws = [torch.empty(g.workspace_bytes(what, q.FP16, 1000, s[2]), dtype=torch.uint8, device="cuda")
                  for g, s in zip(gauges, specs)]
            ws1 = torch.empty(gauges[0].workspace_bytes(what, q.FP16, 1000, specs[0][2]), dtype=torch.uint8,
                              device="cuda")
            ws64 = torch.empty(gauges[0].workspace_bytes(1 | what, q.FP64, 1000, specs[0][2]), dtype=torch.uint8,
                               device="cuda")
            kw = dict(inner_prec=q.FP16, tol=1e-12, inner_max_iter=1000, even_odd=eo, use_graph=use_graph)

            def run():
                for x in xs:
                    x.zero_()
                q.solve_mixed_ir(gauges[0], kappas[0], xs[0], bs[0], workspace=ws1, **kw)
                q.solve_mixed_ir_batched(gauges, kappas, xs, bs, workspaces=ws, **kw)
                q.bicgstab(gauges[0], kappas[0], xs[0], bs[0], prec=q.FP64, tol=1e-12, max_iter=1000,
                           workspace=ws64, history=False, even_odd=eo, use_graph=use_graph)

            run()
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            for _ in range(2):
                run()
            torch.cuda.synchronize()
            assert torch.cuda.mem_get_info()[0] == free0, (eo, use_graph)
            del ws, ws1, ws64
    with pytest.raises(q.QcdError):   # a workspace that is too small is refused
        small = [torch.empty(256, dtype=torch.uint8, device="cuda") for _ in gauges]
        q.solve_mixed_ir_batched(gauges, kappas, xs, bs, workspaces=small, inner_prec=q.FP16, tol=1e-12)
    for g in gauges:
        g.close()


def test_autotune_and_cache(q, tmp_path):
    dims = (8, 8, 8, 8)
    U = qi.gauge_field(dims, 0.3, 61)
    g = q.gauge_upload(to_dev(U), dims)
    cache = str(tmp_path / "tune.jsonl")
    r1 = g.autotune(q.FP16, nrhs=4, reps=5, cache_path=cache)
    assert r1[2] in (1, 2, 4, -2, -4) and r1[3] > 0
    g.set_tuning(q.FP16, 0, 0, 1)
    r2 = g.autotune(q.FP16, nrhs=4, reps=5, cache_path=cache)   # read from the cache
    assert r2[:3] == r1[:3] and abs(r2[3] - r1[3]) < 1e-3
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and '"arch": "gfx' in lines[0]
    # results are unchanged by the tuner's choice
    psi = qi.gaussian_source(dims, 62, nrhs=4)
    out = torch.empty(psi.shape, dtype=torch.complex128, device="cuda")
    q.dslash(g, 0.12, out, to_dev(psi), prec=q.FP16)
    torch.cuda.synchronize()
    for r in range(4):
        compare(to_host(out)[r], oracle.dslash(U, psi[r], 0.12, dims), TOL[2], "tuned")
    g.close()


@pytest.mark.parametrize("use_graph", [False, True])
def test_lattices_of_different_volumes_in_one_call(q, use_graph):
    # three lattices (different extents and kappas, 2 / 3 / 1 right-hand sides,
    # one of them zero) solved together: each is bit-identical to solving that
    # lattice alone, and every true residual meets 1e-12 (re-checked by the oracle)
    specs = [((8, 8, 8, 8), 0.12, 2, 501), ((4, 4, 8, 8), 0.124, 3, 502), ((6, 6, 6, 8), 0.12, 1, 503)]
    gauges, Us, bs, kappas = [], [], [], []
    for dims, k, n, seed in specs:
        U = qi.gauge_field(dims, 0.3, seed)
        b = qi.gaussian_source(dims, seed + 1000, nrhs=n)
        if n == 3:
            b[1] = 0.0
        Us.append(U)
        bs.append(b)
        kappas.append(k)
        gauges.append(q.gauge_upload(to_dev(U), dims))
    xs = [torch.zeros(b.shape, dtype=torch.complex128, device="cuda") for b in bs]
    infos = q.solve_mixed_ir_batched(gauges, kappas, xs, [to_dev(b) for b in bs], inner_prec=q.FP16, tol=1e-12,
                                     use_graph=use_graph)
    for (dims, k, n, _), g, U, b, x, inf in zip(specs, gauges, Us, bs, xs, infos):
        x1 = torch.zeros_like(x)
        single = q.solve_mixed_ir(g, k, x1, to_dev(b), inner_prec=q.FP16, tol=1e-12, use_graph=use_graph)
        assert torch.equal(x, x1), dims
        inf = inf if isinstance(inf, list) else [inf]
        single = single if isinstance(single, list) else [single]
        xh = to_host(x)
        for r in range(n):
            assert inf[r].inner_iters == single[r].inner_iters
            if not np.any(b[r]):
                assert not np.any(xh[r]) and inf[r].true_rel_residual == 0.0
                continue
            res = b[r] - oracle.dslash(U, xh[r], k, dims)
            assert np.linalg.norm(res) <= 1.01e-12 * np.linalg.norm(b[r]), (dims, r)
    for g in gauges:
        g.close()


def test_batched_lattices_reject_repeated_handle(q):
    dims = (4, 4, 4, 4)
    U = qi.gauge_field(dims, 0.3, 510)
    g = q.gauge_upload(to_dev(U), dims)
    b = to_dev(qi.gaussian_source(dims, 511))
    with pytest.raises(q.QcdError):
        q.solve_mixed_ir_batched([g, g], [0.12, 0.12], [torch.zeros_like(b), torch.zeros_like(b)], [b, b])
    g.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("op", [0, 1, 2, 3])
def test_register_tile_of_three_matches_single(q, prec, op):
    # 6 right-hand sides as two tiles of 3 per thread: bit-identical to one per thread
    dims = (4, 6, 8, 10)
    U = qi.gauge_field(dims, 0.3, 81)
    psi = qi.gaussian_source(dims, 82, nrhs=6)
    g = q.gauge_upload(to_dev(U), dims)
    x = to_dev(psi)
    ref, out = torch.empty_like(x), torch.empty_like(x)
    g.set_tuning(prec, 1, 0, 1)
    q.dslash(g, 0.124, ref, x, op=op, prec=prec)
    g.set_tuning(prec, 1, 0, -3)
    q.dslash(g, 0.124, out, x, op=op, prec=prec)
    torch.cuda.synchronize()
    if prec == 2:
        same_to_one_fp16_ulp(out, ref)
    else:
        assert torch.equal(out, ref)
    compare(to_host(out)[5], oracle.dslash(U, psi[5], 0.124, dims, op), TOL[prec], "tile 3")
    g.close()


def test_register_tiles_in_the_batched_solver(q):
    # the epilogues (reductions per right-hand side) and the stopped-RHS masks
    # of the register-tiled operator inside a batched FP16 refinement
    dims = (8, 8, 8, 8)
    U = qi.gauge_field(dims, 0.3, 91)
    bs = qi.gaussian_source(dims, 92, nrhs=6)
    bs[2] *= 1e-4
    g = q.gauge_upload(to_dev(U), dims)
    b = to_dev(bs)
    xs = []
    for tile in (1, -2, -3):
        g.set_tuning(q.FP16, 1, 0, tile)
        x = torch.zeros_like(b)
        infos = q.solve_mixed_ir(g, 0.12, x, b, inner_prec=q.FP16, tol=1e-12)
        assert all(i.true_rel_residual <= 1e-12 for i in infos)
        xs.append(x)
    for x in xs[1:]:
        assert float((x - xs[0]).norm() / xs[0].norm()) < 1e-10
    g.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_register_tiles_on_one_parity(q, prec):
    # the Schur operator of the even-odd form (one-parity fields) with 6
    # right-hand sides as tiles of 3 and of 2 per thread, against one per thread
    # and the oracle
    dims = (4, 6, 8, 10)
    U = qi.gauge_field(dims, 0.3, 85)
    psi = qi.gaussian_source(dims, 86, nrhs=6)
    e = EO.even_mask(dims)
    g = q.gauge_upload(to_dev(U), dims)
    x = to_dev(psi)
    ref = torch.empty_like(x)
    g.set_tuning(prec, 1, 0, 1)
    q.dslash(g, 0.124, ref, x, op=q.OP_SCHUR, prec=prec)
    for tile in (-3, -2):
        out = torch.empty_like(x)
        g.set_tuning(prec, 1, 0, tile)
        q.dslash(g, 0.124, out, x, op=q.OP_SCHUR, prec=prec)
        torch.cuda.synchronize()
        if prec == 2:
            same_to_one_fp16_ulp(out, ref)
        else:
            assert torch.equal(out, ref), tile
        got = to_host(out)
        for r in (0, 5):
            compare(got[r][e], EO.schur(U, psi[r], 0.124, dims)[e], TOL[prec], f"schur tile {tile} rhs {r}")
    g.close()


def test_automatic_tile_is_a_register_tile_for_fp16(q):
    # rhs_tile 0 (automatic) takes 3 per thread for FP16 when the count allows,
    # else 2, else 1; FP32 keeps one per thread
    dims = (8, 8, 8, 8)
    U = qi.gauge_field(dims, 0.3, 87)
    g = q.gauge_upload(to_dev(U), dims)
    for n, tile in ((6, -3), (4, -2), (5, 1)):
        x = to_dev(qi.gaussian_source(dims, 88 + n, nrhs=n))
        auto, fixed = torch.empty_like(x), torch.empty_like(x)
        g.set_tuning(q.FP16, 1, 0, 0)
        q.dslash(g, 0.124, auto, x, prec=q.FP16)
        g.set_tuning(q.FP16, 1, 0, tile)
        q.dslash(g, 0.124, fixed, x, prec=q.FP16)
        torch.cuda.synchronize()
        assert torch.equal(auto, fixed), n
    g.close()


def test_register_tiles_in_the_even_odd_solver(q):
    dims = (8, 8, 8, 8)
    U = qi.gauge_field(dims, 0.3, 93)
    bs = qi.gaussian_source(dims, 94, nrhs=6)
    bs[4] *= 1e-4
    g = q.gauge_upload(to_dev(U), dims)
    b = to_dev(bs)
    xs = []
    for tile in (1, -2, -3):
        g.set_tuning(q.FP16, 1, 0, tile)
        x = torch.zeros_like(b)
        infos = q.solve_mixed_ir(g, 0.12, x, b, inner_prec=q.FP16, tol=1e-12, even_odd=True)
        assert all(i.true_rel_residual <= 1e-12 for i in infos)
        xs.append(x)
    for x in xs[1:]:
        assert float((x - xs[0]).norm() / xs[0].norm()) < 1e-10
    xh = to_host(xs[2])
    for r in (0, 4):
        res = bs[r] - oracle.dslash(U, xh[r], 0.12, dims)
        assert np.linalg.norm(res) <= 1.01e-12 * np.linalg.norm(bs[r])
    g.close()


def test_largest_right_hand_side_count(q):
    # 64 right-hand sides (the most one call takes) through the operator and
    # the even-odd FP16-inner refinement; 65 is refused
    dims, k, n = (4, 4, 4, 4), 0.12, 64
    U = qi.gauge_field(dims, 0.3, 610)
    psi = qi.gaussian_source(dims, 611, nrhs=n)
    g = q.gauge_upload(to_dev(U), dims)
    x = to_dev(psi)
    out = torch.empty_like(x)
    q.dslash(g, k, out, x, prec=q.FP16)
    got = to_host(out)
    for r in (0, 31, 63):
        compare(got[r], oracle.dslash(U, psi[r], k, dims, 0), TOL[2], f"64 rhs, rhs={r}")
    sol = torch.zeros_like(x)
    infos = q.solve_mixed_ir(g, k, sol, x, inner_prec=q.FP16, s=128.0, sigma=64.0, tol=1e-12, even_odd=True,
                             use_graph=True)
    assert len(infos) == n and all(i.status == "ok" and i.true_rel_residual <= 1e-12 for i in infos)
    xh = to_host(sol)
    for r in (0, 63):
        res = np.linalg.norm(psi[r] - oracle.dslash(U, xh[r], k, dims)) / np.linalg.norm(psi[r])
        assert res <= 1.01e-12
    big = to_dev(qi.gaussian_source(dims, 612, nrhs=n + 1))
    with pytest.raises(q.QcdError):
        q.dslash(g, k, torch.empty_like(big), big, prec=q.FP16)
    g.close()
