"""Parity of the HIP Wilson operator and conversions with the CPU oracle (through the C ABI)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import qcd_inputs as qi  # noqa: E402
from oracle import solvers as S  # noqa: E402
from gpu_common import TOL, compare, fields, to_dev, to_host  # noqa: E402


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2602_14450_amd as q
    return q


SHAPES = [(2, 2, 2, 2), (2, 4, 6, 8), (4, 6, 8, 10), (2, 4, 6, 10), (8, 8, 8, 8), (6, 4, 2, 12)]
OPS = [0, 1, 2, 3]


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_dslash_all_ops(q, dims, prec):
    U, psi = fields(dims, gseed=11 + sum(dims), sseed=12)
    g = q.gauge_upload(to_dev(U), dims)
    k = 0.124
    x = to_dev(psi)
    out = torch.empty_like(x)
    for op in OPS:
        q.dslash(g, k, out, x, op=op, prec=prec, layout=q.CANONICAL)
        torch.cuda.synchronize()
        want = oracle.dslash(U, psi, k, dims, op)
        compare(to_host(out), want, TOL[prec], f"dims={dims} prec={prec} op={op}")
    g.close()


def test_dslash_native_layout_and_bitwise_rerun(q):
    dims = (4, 6, 8, 10)
    U, psi = fields(dims)
    g = q.gauge_upload(to_dev(U), dims)
    for prec in (0, 1, 2, 3):
        a = g.native_spinor(prec)
        b1 = g.native_spinor(prec)
        b2 = g.native_spinor(prec)
        q.convert(g, prec, a, to_dev(psi))
        q.dslash(g, 0.13, b1, a, prec=prec, layout=q.NATIVE)
        q.dslash(g, 0.13, b2, a, prec=prec, layout=q.NATIVE)
        torch.cuda.synchronize()
        assert torch.equal(b1, b2)
        out = torch.empty(psi.shape, dtype=torch.complex128, device="cuda")
        q.unconvert(g, prec, out, b1)
        compare(to_host(out), oracle.dslash(U, psi, 0.13, dims), TOL[prec], f"native prec={prec}")
    g.close()


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_convert_is_bit_exact(q, prec):
    dims = (2, 4, 6, 10)
    U, psi = fields(dims)
    psi = psi * np.geomspace(1e-9, 50.0, psi.size).reshape(psi.shape)   # FP16 subnormals up to ~3e4 after scaling
    g = q.gauge_upload(to_dev(U), dims)
    for scale, ftz in [(1.0, False), (128.0, False), (3.7e-3, True), (40.0, True)]:
        nat = g.native_spinor(prec)
        n2 = q.convert(g, prec, nat, to_dev(psi), scale=scale, ftz=ftz)
        back = torch.empty(psi.shape, dtype=torch.complex128, device="cuda")
        q.unconvert(g, prec, back, nat)
        torch.cuda.synchronize()
        want = S.lowp(scale * psi, {1: S.FP32, 2: S.FP16, 3: S.BF16}[prec], ftz=ftz)
        got = to_host(back)
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), f"scale={scale} ftz={ftz}"
        assert abs(n2 - S.norm2(want)) <= 1e-6 * S.norm2(want)
    g.close()


def test_residual_fp64(q):
    dims = (4, 4, 6, 8)
    U, b = fields(dims)
    x = qi.gaussian_source(dims, 77)
    g = q.gauge_upload(to_dev(U), dims)
    r = torch.empty_like(to_dev(b))
    n2 = q.residual(g, 0.12, r, to_dev(x), to_dev(b))
    want = b - oracle.dslash(U, x, 0.12, dims)
    compare(to_host(r), want, 1e-14, "residual")
    assert abs(n2 - S.norm2(want)) < 1e-12 * S.norm2(want)
    g.close()


def test_invalid_arguments(q):
    dims = (3, 4, 4, 4)
    U = to_dev(qi.unit_gauge(dims))
    with pytest.raises(q.QcdError):
        q.gauge_upload(U, dims)
    dims = (4, 4, 4, 4)
    g = q.gauge_upload(to_dev(qi.unit_gauge(dims)), dims)
    x = to_dev(qi.gaussian_source(dims, 1))
    with pytest.raises(q.QcdError):
        q.dslash(g, 0.1, x, x)          # aliasing
    with pytest.raises(q.QcdError):
        q.dslash(g, -0.1, torch.empty_like(x), x)
    g.close()


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_dslash_full_size_sampled(q, prec):
    # The benchmark lattice 32^3 x 64 in the launch configuration the
    # benchmark times (native layout); outputs compared at sampled sites.
    dims = (32, 32, 32, 64)
    U, psi = fields(dims, gseed=201, sseed=202)
    g = q.gauge_upload(to_dev(U), dims, precs=(0, prec))
    a = g.native_spinor(prec)
    b = g.native_spinor(prec)
    q.convert(g, prec, a, to_dev(psi), want_norm=False)
    q.dslash(g, 0.124, b, a, prec=prec, layout=q.NATIVE)
    out = torch.empty(psi.shape, dtype=torch.complex128, device="cuda")
    q.unconvert(g, prec, out, b)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    V = int(np.prod(dims))
    sites = np.concatenate([[0, 1, 31, 32, V - 1, V - 32 * 32 * 32], rng.choice(V, 4000, replace=False)])
    got = to_host(out)[sites]
    want = oracle.dslash_sites(U, psi, 0.124, dims, sites)
    compare(got, want, TOL[prec], f"32^3x64 prec={prec}")
    g.close()


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_su3_links_stored_as_two_rows(q, prec):
    # generated links are SU(3): 12 reals per link, same operator as the
    # full 18-real storage within the precision's tolerance, both against the oracle
    dims = (4, 6, 8, 10)
    U, psi = fields(dims, gseed=71, sseed=72)
    g12 = q.gauge_upload(to_dev(U), dims)
    g18 = q.gauge_upload(to_dev(U), dims, full_links=True)
    assert g12.link_reals(prec) == 12 and g18.link_reals(prec) == 18
    x = to_dev(psi)
    for op in OPS:
        want = oracle.dslash(U, psi, 0.124, dims, op)
        for g in (g12, g18):
            out = torch.empty_like(x)
            q.dslash(g, 0.124, out, x, op=op, prec=prec)
            torch.cuda.synchronize()
            compare(to_host(out), want, TOL[prec], f"links={g.link_reals(prec)} prec={prec} op={op}")
    g12.close()
    g18.close()


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_u3_links_keep_all_entries(q, prec):
    # a U(3) field (SU(3) times a site-dependent phase) fails the SU(3) check:
    # all 18 reals are kept and the operator still matches the oracle
    dims = (4, 4, 6, 8)
    U, psi = fields(dims, gseed=73, sseed=74)
    phase = np.exp(1j * 2 * np.pi * qi.uniform(U.shape[0] * 4, 75)).reshape(-1, 4, 1, 1)
    U = U * phase
    g = q.gauge_upload(to_dev(U), dims)
    assert g.link_reals(prec) == 18
    x = to_dev(psi)
    out = torch.empty_like(x)
    for op in OPS:
        q.dslash(g, 0.124, out, x, op=op, prec=prec)
        torch.cuda.synchronize()
        compare(to_host(out), oracle.dslash(U, psi, 0.124, dims, op), TOL[prec], f"U(3) prec={prec} op={op}")
    g.close()


def test_bf16_operator_is_the_rounded_exact_operator(q):
    # With all 18 reals stored, the BF16 operator computes in FP32 on the
    # BF16-rounded links and input and rounds the result once: every element
    # is the oracle's FP64 operator on the same rounded inputs, rounded to BF16,
    # or (where FP32 summation decides a near-tie) its neighbour.
    dims = (4, 6, 8, 10)
    U, psi = fields(dims, gseed=77, sseed=78)
    Ub, pb = S.lowp(U, S.BF16), S.lowp(psi, S.BF16)
    g = q.gauge_upload(to_dev(U), dims, full_links=True)
    x = to_dev(psi)
    out = torch.empty_like(x)
    for op in OPS:
        q.dslash(g, 0.124, out, x, op=op, prec=q.BF16)
        torch.cuda.synchronize()
        got = to_host(out).reshape(-1)
        want = S.lowp(oracle.dslash(Ub, pb, 0.124, dims, op), S.BF16).reshape(-1)
        rms = np.sqrt(np.mean(np.abs(want) ** 2))
        for a, b in ((got.real, want.real), (got.imag, want.imag)):
            ulp = np.ldexp(1.0, np.frexp(np.abs(b))[1] - 8)
            d = np.abs(a - b)
            # FP32 sums of terms of size ~rms: 1e-6 rms absolute on top of one BF16 unit
            assert np.all(d <= ulp + 1e-6 * rms), f"op={op}: {np.max(d / ulp):.2f} ulp"
            assert np.count_nonzero(d) <= max(4, a.size // 200), f"op={op}: {np.count_nonzero(d)} of {a.size} differ"
    g.close()


@pytest.mark.parametrize("dims", [(16, 16, 4, 4), (32, 8, 4, 6), (64, 4, 2, 2), (2, 4, 6, 10), (32, 32, 32, 64)])
@pytest.mark.parametrize("prec", [2, 3])
def test_lds_staged_variant_matches_oracle(q, dims, prec):
    # launch variant 6 (x and y neighbours staged in LDS; blocks of whole x
    # rows, so the halo rows wrap in y on the small lattices) against the
    # oracle for every operator and schedule, and against variant 0 element
    # by element: the same products in the same order, so the two differ at
    # most where the compiler fuses the final FP32 sums differently (one unit
    # of the storage format in rare elements); on (2, 4, 6, 10) a block does
    # not cover whole rows and variant 6 is variant 0 itself
    U, psi = fields(dims, gseed=21 + sum(dims), sseed=22)
    g = q.gauge_upload(to_dev(U), dims, precs=(q.FP64, prec))
    a = g.native_spinor(prec)
    q.convert(g, prec, a, to_dev(psi), want_norm=False)
    ref, got = g.native_spinor(prec), g.native_spinor(prec)
    big = dims == (32, 32, 32, 64)
    unit = 2.0 ** -10 if prec == 2 else 2.0 ** -7     # one unit in the last place, relative, of FP16 / BF16
    o_ref = torch.empty(psi.shape, dtype=torch.complex128, device="cuda")
    o_got = torch.empty_like(o_ref)
    for op in ([0] if big else OPS):
        for sched in ([1] if big else [0, 1, 4]):
            g.set_tuning(prec, sched, 0, 1)
            q.dslash(g, 0.124, ref, a, op=op, prec=prec, layout=q.NATIVE)
            g.set_tuning(prec, sched, 6, 1)
            q.dslash(g, 0.124, got, a, op=op, prec=prec, layout=q.NATIVE)
            q.unconvert(g, prec, o_ref, ref)
            q.unconvert(g, prec, o_got, got)
            torch.cuda.synchronize()
            r, v = to_host(o_ref).reshape(-1), to_host(o_got).reshape(-1)
            for part in (np.real, np.imag):
                d = np.abs(part(v) - part(r))
                assert np.all(d <= unit * np.abs(part(r)) + 1e-30), (dims, prec, op, sched, d.max())
            frac = np.mean(r != v)
            assert frac <= 1e-3, (dims, prec, op, sched, frac)
            if not big:
                compare(to_host(o_got), oracle.dslash(U, psi, 0.124, dims, op), TOL[prec], f"lds {dims} op={op}")
            else:
                V = qi.volume(dims)
                sites = np.random.default_rng(23).integers(0, V, 300)
                compare(to_host(o_got)[sites], oracle.dslash_sites(U, psi, 0.124, dims, sites), TOL[prec], "lds 32^3x64")
    g.close()
