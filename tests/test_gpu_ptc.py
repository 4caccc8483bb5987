"""Parity of the HIP parallel-transport network (forward, gradients, Adam) with
the FP64 oracle in oracle/ptc.py, through the C ABI.

Tolerance.  Channel mixing multiplies BF16-rounded inputs by BF16-rounded
weights (unit roundoff u = 2^-9) with FP32 accumulation.  One layer therefore
carries a relative error of about sqrt(2) u per product, averaged over the
K = 36 C_in terms; three layers compound to under 1e-2 in norm.  Element-wise
we allow 5e-2 of the rms element (tails of the rounding distribution).
Gradients are sums over all sites of such products, back-propagated through
the same layers: 3e-2 in norm per layer.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import qcd_inputs as qi  # noqa: E402
from oracle import ptc as P  # noqa: E402
from gpu_common import to_dev, to_host  # noqa: E402

CH = (1, 2, 2, 1)
U_BF16 = 2.0 ** -9


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2602_14450_amd as q
    return q


def rel(got, want):
    return np.linalg.norm(got - want) / np.linalg.norm(want)


def check(got, want, norm_tol, elem_tol, what):
    got = got.reshape(-1)
    want = want.reshape(-1)
    r = rel(got, want)
    assert r <= norm_tol, f"{what}: norm-relative error {r:.3e} > {norm_tol}"
    rms = np.sqrt(np.mean(np.abs(want) ** 2))
    worst = np.max(np.abs(got - want))
    assert worst <= elem_tol * rms, f"{what}: worst element error {worst:.3e} > {elem_tol} * rms {rms:.3e}"
    return r


# (4,4,4,8): whole 64-site blocks; (6,4,4,6): 288 half-sites, a ragged last block
DIMS = [(4, 4, 4, 8), (6, 4, 4, 6)]


@pytest.mark.parametrize("dims", DIMS)
def test_identity_weights_round_to_bf16(q, dims):
    # W = identity on the p = 0 path of every layer: M(psi) = psi up to BF16 input rounding
    U = qi.gauge_field(dims, 0.3, 5)
    psi = qi.gaussian_source(dims, 6)
    Ws = [np.zeros((9, co, ci, 4, 4), complex) for ci, co in zip(CH[:-1], CH[1:])]
    for W in Ws:
        for j in range(W.shape[1]):
            W[0, j, j % W.shape[2]] = np.eye(4)
    g = q.gauge_upload(to_dev(U), dims)
    net = q.PTC(g, CH, max_batch=1)
    net.set_weights(Ws)
    out = torch.empty_like(to_dev(psi))
    net.apply(out, to_dev(psi))
    got = to_host(out)
    # each layer rounds its input to BF16; 1.0 and 0.0 are exact, so the error is one rounding
    # of re and im per layer boundary (three in a row, each within u |value|)
    err = np.abs(got - psi)
    assert np.all(err <= 3.01 * U_BF16 * np.sqrt(2) * np.abs(psi) + 1e-30)
    net.close()
    g.close()


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("seed", [1, 2])
def test_forward_matches_oracle(q, dims, seed):
    U = qi.gauge_field(dims, 0.3, 10 + seed)
    psi = qi.gaussian_source(dims, 20 + seed)
    Ws = qi.ptc_weights(CH, seed=30 + seed, scale=0.5)
    nb = P.neighbours(dims)
    want = P.forward(U, psi, Ws, nb)
    g = q.gauge_upload(to_dev(U), dims)
    net = q.PTC(g, CH, max_batch=1)
    net.set_weights(Ws)
    out = torch.empty_like(to_dev(psi))
    net.apply(out, to_dev(psi))
    check(to_host(out), want, 1e-2, 5e-2, f"forward dims={dims} seed={seed}")
    # the weights round-trip through FP32
    back = net.get_weights()
    for a, b in zip(back, Ws):
        assert np.max(np.abs(a - b)) <= 2 ** -23 * np.max(np.abs(b)) * 2
    net.close()
    g.close()


@pytest.mark.parametrize("dims", DIMS + [(8, 8, 8, 8)])
@pytest.mark.parametrize("full_links", [False, True])
def test_fp16_forward_matches_oracle(q, dims, full_links):
    # The form the FP16 inner solve applies: binary16 input, links and hidden
    # activations (u = 2^-11 each, well below the BF16 rounding of the channel
    # mixing), so the FP32 form's tolerances hold.  Both link storages: two
    # rows with the third rebuilt, and all three rows.
    U = qi.gauge_field(dims, 0.3, 60)
    psi = qi.gaussian_source(dims, 61, nrhs=2)
    Ws = qi.ptc_weights(CH, seed=62, scale=0.5)
    nb = P.neighbours(dims)
    g = q.gauge_upload(to_dev(U), dims, full_links=full_links)
    net = q.PTC(g, CH, max_batch=2)
    net.set_weights(Ws)
    out = torch.empty_like(to_dev(psi))
    net.apply_prec(out, to_dev(psi), q.FP16)
    got = to_host(out)
    for b in range(2):
        want = P.forward(U, psi[b], Ws, nb)
        check(got[b], want, 1e-2, 5e-2, f"fp16 forward dims={dims} full={full_links} b={b}")
    # one field alone gives the same bits as its slot in the batch
    one = torch.empty_like(to_dev(psi[1]))
    net.apply_prec(one, to_dev(psi[1]), q.FP16)
    assert torch.equal(one, out[1])
    # FP32 through the same entry point is qcd_ptc_apply
    a = torch.empty_like(out)
    b32 = torch.empty_like(out)
    net.apply_prec(a, to_dev(psi), q.FP32)
    net.apply(b32, to_dev(psi))
    assert torch.equal(a, b32)
    net.close()
    g.close()


def test_fp16_apply_needs_fp16_links(q):
    dims = (4, 4, 4, 8)
    g = q.gauge_upload(to_dev(qi.gauge_field(dims, 0.3, 63)), dims, precs=(q.FP64, q.FP32))
    net = q.PTC(g, CH, max_batch=1)
    psi = to_dev(qi.gaussian_source(dims, 64))
    out = torch.empty_like(psi)
    with pytest.raises(q.QcdError):
        net.apply_prec(out, psi, q.FP16)
    with pytest.raises(q.QcdError):
        net.apply_prec(out, psi, q.BF16)
    net.close()
    g.close()


def test_single_layer_weights_layout(q):
    # one layer, one channel, only the +t path with a spin matrix S: out = S (U_t(x) psi(x+t))
    dims = (4, 4, 4, 8)
    U = qi.gauge_field(dims, 0.3, 40)
    psi = qi.gaussian_source(dims, 41)
    rng = np.random.default_rng(42)
    W = np.zeros((9, 1, 1, 4, 4), complex)
    W[7, 0, 0] = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    nb = P.neighbours(dims)
    want = P.forward(U, psi, [W], nb)
    g = q.gauge_upload(to_dev(U), dims)
    net = q.PTC(g, (1, 1), max_batch=1)
    net.set_weights([W])
    out = torch.empty_like(to_dev(psi))
    net.apply(out, to_dev(psi))
    check(to_host(out), want, 1e-2, 5e-2, "single +t path")
    net.close()
    g.close()


def test_batch_equals_single(q):
    dims = (6, 4, 4, 6)
    U = qi.gauge_field(dims, 0.3, 50)
    psis = qi.gaussian_source(dims, 51, nrhs=3)
    Ws = qi.ptc_weights(CH, seed=52, scale=0.5)
    g = q.gauge_upload(to_dev(U), dims)
    net = q.PTC(g, CH, max_batch=3)
    net.set_weights(Ws)
    outb = torch.empty_like(to_dev(psis))
    net.apply(outb, to_dev(psis))
    for b in range(3):
        o = torch.empty_like(to_dev(psis[b]))
        net.apply(o, to_dev(psis[b]))
        # the same BF16 GEMM per column: bitwise equal
        assert torch.equal(o, outb[b])
    net.close()
    g.close()


def test_gauge_covariance(q):
    # M[U^G](G psi) = G M[U](psi), with U^G_mu(x) = G(x) U_mu(x) G(x+mu)^dag
    dims = (4, 4, 4, 8)
    U = qi.gauge_field(dims, 0.3, 60)
    psi = qi.gaussian_source(dims, 61)
    G = qi.gauge_transform(dims, 1.0, 62)
    fwd, _ = P.neighbours(dims)
    UG = np.empty_like(U)
    for mu in range(4):
        UG[:, mu] = G @ U[:, mu] @ np.conj(np.transpose(G[fwd[:, mu]], (0, 2, 1)))
    psiG = np.einsum("sab,sjb->sja", G, psi)
    Ws = qi.ptc_weights(CH, seed=63, scale=0.5)
    outs = []
    for UU, ps in ((U, psi), (UG, psiG)):
        g = q.gauge_upload(to_dev(UU), dims)
        net = q.PTC(g, CH, max_batch=1)
        net.set_weights(Ws)
        o = torch.empty_like(to_dev(ps))
        net.apply(o, to_dev(ps))
        outs.append(to_host(o))
        net.close()
        g.close()
    check(outs[1], np.einsum("sab,sjb->sja", G, outs[0]), 2e-2, 1e-1, "gauge covariance")


@pytest.mark.parametrize("dims", DIMS)
def test_loss_and_gradient_match_oracle(q, dims):
    U = qi.gauge_field(dims, 0.3, 70)
    B = 2
    rs = qi.gaussian_source(dims, 71, nrhs=B)
    es = qi.gaussian_source(dims, 72, nrhs=B)
    Ws = qi.ptc_weights(CH, seed=73, scale=0.5)
    nb = P.neighbours(dims)
    want_loss, want_grad = P.grad(U, list(rs), list(es), Ws, nb)
    g = q.gauge_upload(to_dev(U), dims)
    net = q.PTC(g, CH, max_batch=B)
    net.set_weights(Ws)
    loss, grad = net.loss_grad(to_dev(rs), to_dev(es))
    assert abs(loss - want_loss) <= 1e-2 * want_loss
    for l, (a, b) in enumerate(zip(grad, want_grad)):
        r = rel(a, b)
        assert r <= 3e-2, f"layer {l}: gradient norm-relative error {r:.3e}"
    net.close()
    g.close()


def test_adam_step_matches_formula_and_training_lowers_loss(q):
    dims = (4, 4, 4, 8)
    U = qi.gauge_field(dims, 0.3, 80)
    B = 2
    rs = qi.gaussian_source(dims, 81, nrhs=B)
    Ws = qi.ptc_weights(CH, seed=82, scale=0.5)
    nb = P.neighbours(dims)
    # a target the network can represent: the output of other weights
    Wt = qi.ptc_weights(CH, seed=83, scale=0.5)
    es = np.stack([P.forward(U, r, Wt, nb) for r in rs])
    g = q.gauge_upload(to_dev(U), dims)
    net = q.PTC(g, CH, max_batch=B)
    net.set_weights(Ws)
    r_d, e_d = to_dev(rs), to_dev(es)
    _, grad = net.loss_grad(r_d, e_d)
    lr = 1e-3
    l0 = net.train_step(r_d, e_d, lr=lr)
    w1 = net.get_weights()
    # first Adam step: w -= lr * g / (|g| + eps) component-wise (bias corrections cancel)
    for a, w, gr in zip(w1, Ws, grad):
        for part in (np.real, np.imag):
            gg = part(gr)
            step = lr * gg / (np.abs(gg) + 1e-8)
            want = part(w).astype(np.float32) - step
            assert np.max(np.abs(part(a) - want)) <= 1e-6 + 1e-3 * lr
    losses = [l0]
    for _ in range(40):
        losses.append(net.train_step(r_d, e_d, lr=1e-2))
    assert losses[-1] < 0.5 * losses[0], losses
    net.close()
    g.close()


def test_rejects_bad_configuration(q):
    dims = (4, 4, 4, 8)
    U = qi.gauge_field(dims, 0.3, 90)
    g = q.gauge_upload(to_dev(U), dims)
    with pytest.raises(q.QcdError):
        q.PTC(g, (1, 3, 1))
    with pytest.raises(q.QcdError):
        q.PTC(g, (2, 2, 1))
    with pytest.raises(q.QcdError):
        q.PTC(g, (1, 2, 1), max_batch=0)
    net = q.PTC(g, CH, max_batch=1)
    psis = to_dev(qi.gaussian_source(dims, 91, nrhs=2))
    with pytest.raises(q.QcdError):
        net.apply(torch.empty_like(psis), psis)   # batch above max_batch
    net.close()
    g.close()
    g64 = q.gauge_upload(to_dev(U), dims, precs=(q.FP64,))
    with pytest.raises(q.QcdError):
        q.PTC(g64, CH)
    g64.close()


def test_device_sources_match_the_input_generator(q):
    # the training pairs' sources are drawn on the device from the same
    # counter-based recipe as the seeded input generator (SplitMix64 draws
    # 2j, 2j + 1 and Box-Muller): equal up to the last bits of log / sin / cos
    dims = (4, 4, 6, 8)
    for seed, n in ((2_000_000, 3), (7, 1), (2**63 + 5, 2)):
        got = to_host(q.gaussian_spinors((n, qi.volume(dims), 4, 3), seed))
        want = qi.gaussian_source(dims, seed, nrhs=n)
        assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(want)), seed
    big = to_host(q.gaussian_spinors((1 << 20,), 11))
    assert abs(np.mean(np.abs(big) ** 2) - 1.0) < 1e-2 and abs(np.mean(big)) < 5e-3


@pytest.mark.parametrize("dims", [(32, 32, 32, 64)])
def test_apply_at_full_size_matches_oracle_on_sampled_sites(q, dims):
    # 32^3 x 64, the headline lattice: the oracle's network evaluated on 66
    # sampled sites (its three-hop neighbourhoods only) against the FP32 apply
    # (fused BF16 mixing) and the FP16 form the inner solver applies, whose
    # launches here have the full lattice's block count and schedule
    V = qi.volume(dims)
    U = qi.gauge_field(dims, 0.3, 70)
    psi = qi.gaussian_source(dims, 72)
    Ws = qi.ptc_weights(CH, seed=71, scale=0.5)
    rng = np.random.default_rng(73)
    sites = np.concatenate([[0, V - 1], rng.integers(0, V, 64)])
    want = P.forward_sites(U, psi, Ws, dims, sites)
    g = q.gauge_upload(to_dev(U), dims, precs=(q.FP32, q.FP16))
    net = q.PTC(g, CH, max_batch=1)
    net.set_weights(Ws)
    x = to_dev(psi)
    o16, o32 = torch.empty_like(x), torch.empty_like(x)
    net.apply_prec(o16, x, q.FP16)
    net.apply_prec(o32, x, q.FP32)
    check(to_host(o32)[sites], want, 1e-2, 5e-2, "fp32 apply at 32^3 x 64, sampled sites")
    check(to_host(o16)[sites], want, 1e-2, 5e-2, "fp16 apply at 32^3 x 64, sampled sites")
    net.close()
    g.close()
    del x, o16, o32
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dims", DIMS)
def test_fp32_mixing_matches_oracle_tightly(q, dims):
    # With FP32 mixing (FP32 transported inputs, weights and output gradients on
    # the FP32 matrix cores) every rounding is FP32 (u = 2^-24) over sums of a
    # few hundred terms: forward, loss and gradients agree with the FP64 oracle
    # to 1e-5, for the regression loss and for the residual loss.
    U = qi.gauge_field(dims, 0.3, 75)
    B = 2
    k = 0.124
    rs = qi.gaussian_source(dims, 76, nrhs=B)
    es = qi.gaussian_source(dims, 77, nrhs=B)
    Ws = qi.ptc_weights(CH, seed=78, scale=0.5)
    nb = P.neighbours(dims)
    g = q.gauge_upload(to_dev(U), dims)
    net = q.PTC(g, CH, max_batch=B)
    net.set_weights(Ws)
    net.set_mixing(q.FP32)
    out = torch.empty_like(to_dev(rs))
    net.apply(out, to_dev(rs))
    got = to_host(out)
    for b in range(B):
        check(got[b], P.forward(U, rs[b], Ws, nb), 1e-5, 1e-4, f"fp32-mixing forward dims={dims} b={b}")
    want_loss, want_grad = P.grad(U, list(rs), list(es), Ws, nb)
    loss, grad = net.loss_grad(to_dev(rs), to_dev(es))
    assert abs(loss - want_loss) <= 1e-5 * want_loss, (loss, want_loss)
    for l, (a, b_) in enumerate(zip(grad, want_grad)):
        r = rel(a, b_)
        assert r <= 1e-5, f"layer {l}: gradient norm-relative error {r:.3e}"
    want_loss, want_grad = P.grad_residual(U, k, list(rs), Ws, nb, dims)
    loss, grad = net.loss_grad_residual(k, to_dev(rs))
    assert abs(loss - want_loss) <= 1e-5 * want_loss, (loss, want_loss)
    for l, (a, b_) in enumerate(zip(grad, want_grad)):
        r = rel(a, b_)
        assert r <= 1e-5, f"layer {l}: residual-loss gradient norm-relative error {r:.3e}"
    # back to BF16 mixing: the BF16 results of a fresh network, bit for bit
    net.set_mixing(q.BF16)
    fresh = q.PTC(g, CH, max_batch=B)
    fresh.set_weights(Ws)
    o1, o2 = torch.empty_like(out), torch.empty_like(out)
    net.apply(o1, to_dev(rs))
    fresh.apply(o2, to_dev(rs))
    assert torch.equal(o1, o2)
    fresh.close()
    net.close()
    g.close()


@pytest.mark.parametrize("dims", DIMS)
def test_residual_loss_and_gradient_bf16_match_oracle(q, dims):
    # the residual loss with BF16 mixing: the tolerances of the regression loss
    U = qi.gauge_field(dims, 0.3, 85)
    B = 2
    k = 0.124
    rs = qi.gaussian_source(dims, 86, nrhs=B)
    Ws = qi.ptc_weights(CH, seed=87, scale=0.5)
    nb = P.neighbours(dims)
    want_loss, want_grad = P.grad_residual(U, k, list(rs), Ws, nb, dims)
    g = q.gauge_upload(to_dev(U), dims)
    net = q.PTC(g, CH, max_batch=B)
    net.set_weights(Ws)
    loss, grad = net.loss_grad_residual(k, to_dev(rs))
    assert abs(loss - want_loss) <= 1e-2 * want_loss
    for l, (a, b_) in enumerate(zip(grad, want_grad)):
        r = rel(a, b_)
        assert r <= 3e-2, f"layer {l}: gradient norm-relative error {r:.3e}"
    # a training step on the residual loss lowers it
    l0 = net.train_step_residual(k, to_dev(rs), lr=1e-3)
    for _ in range(20):
        l1 = net.train_step_residual(k, to_dev(rs), lr=1e-3)
    assert l1 < l0, (l0, l1)
    net.close()
    g.close()
