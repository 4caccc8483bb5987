"""What the trained network gains over the method without it, and over its
own starting point (16^4, kappa = 0.124, the learned form of the benchmark
cut to 4 training fields).

* Training on the residual loss |D M r - r|^2 / |r|^2 (the distance of the
  preconditioned operator D M from the identity, over Gaussian sources; no
  solves) lowers that loss on a held-out field by more than a fifth below
  its start, the third-order Neumann series sum_{k<=3} (kappa H)^k that the
  1-2-2-1 network represents exactly (D M = 1 - (kappa H)^4).
* Used as right preconditioner of the flexible FP16-inner refinement on a
  held-out field, the trained network reaches the true FP64 residual 1e-12
  in fewer inner iterations than its Neumann start at the inner tolerance
  1e-3 (the tighter inner solves are where the preconditioner's quality
  shows: at 1e-2 both need two iterations per refinement step), and in at
  most half the iterations of the plain refinement; the plain solver stays
  the fallback, and the FP64 residual decides every step.
"""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import qcd_inputs as qi  # noqa: E402


@pytest.fixture(scope="module")
def q():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2602_14450_amd as q
    return q


def test_trained_network_gains_over_plain_and_over_its_start(q):
    from paper_2602_14450_amd import ptc_train as T
    dims, kappa = (16, 16, 16, 16), 0.124
    net, gauges, info = T.train_residual(dims, kappa, nfields=4, sources_per_field=512, epochs=2, batch=16, lr=1e-3)
    for g in gauges:
        g.close()
    g = q.gauge_upload(torch.from_numpy(qi.gauge_field(dims, 0.3, 999)).cuda(), dims)
    neu = q.PTC(g, (1, 2, 2, 1), max_batch=16)
    neu.init_neumann(kappa)
    loss_start = T.residual_loss(neu, g, kappa, 5_000_000)
    loss_trained = T.residual_loss(net, g, kappa, 5_000_000)
    assert loss_trained < 0.8 * loss_start, (loss_trained, loss_start)
    b = torch.from_numpy(qi.gaussian_source(dims, 4242)).cuda()
    iters = {}
    for itol in (1e-2, 1e-3):
        for name, pc in (("plain", None), ("neumann", neu), ("trained", net)):
            x = torch.zeros_like(b)
            inf = q.solve_mixed_ir(g, kappa, x, b, inner_prec=q.FP16, s=128.0, sigma=64.0, tol=1e-12,
                                   inner_tol=itol, use_graph=True, precond=pc)
            assert inf.status == "ok" and inf.true_rel_residual <= 1e-12, (name, itol, inf)
            iters[(name, itol)] = inf.inner_iters
            if pc is not None:
                assert inf.precond_fallback == -1 and inf.precond_steps == inf.outer_iters
    print(f"held-out residual loss {loss_trained:.5f} (Neumann start {loss_start:.5f}); inner iterations {iters}")
    assert iters[("trained", 1e-2)] * 2 <= iters[("plain", 1e-2)], iters
    assert iters[("trained", 1e-3)] < iters[("neumann", 1e-3)], iters
    assert iters[("trained", 1e-2)] <= iters[("neumann", 1e-2)], iters
    net.close()
    neu.close()
    g.close()
