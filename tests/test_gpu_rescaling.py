"""The (s, sigma) study of Sec. 6 (``rescaling_study``) on a small lattice.

Pins: the first inner right-hand side of the even-odd solve with the point
source b = e_0 has exactly one non-zero element (eta_o = 0, so b' = e_0: the
count the paper prints with Fig. 9); every solve of the grid reaches the true
residual it reports; BF16 storage needs no rescaling for this source.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from test_oracle_solvers import paper_facts  # noqa: E402


@pytest.fixture(scope="module")
def rs():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2602_14450_amd import rescaling_study
    return rescaling_study


def test_small_grid(rs):
    dims = (8, 8, 8, 8)
    res = rs.study(dims, kappa=0.12, eps=0.3, seed=5, s_grid=(1.0, 128.0), sigma_grid=(0.0, 64.0),
                   panels=((False, True),), bf16_points=((1.0, 0.0), (128.0, 64.0)))
    vh = int(np.prod(dims)) // 2
    nonzero = paper_facts()["nonzero_first_input"]
    for rec in res["records"] + res["bf16"]:
        assert rec["matvecs"] is not None, rec
        assert rec["true_rel_residual"] <= 1e-12
        zf = rec["zero_fraction"]
        assert round((1 - zf[0]) * 24 * vh) == nonzero, rec
        assert all(0.0 <= z <= 1.0 for z in zf)
    assert len(res["records"]) == 4 and len(res["bf16"]) == 2
    assert res["fp32_reference"]["zero_fraction"][0] == res["records"][0]["zero_fraction"][0]
    # the rescaled FP16 run is no slower than the unscaled one, and BF16 without
    # rescaling is within a few applications of the rescaled FP16 run
    by = {(r["s"], r["sigma"]): r["matvecs"] for r in res["records"]}
    assert by[(128.0, 64.0)] <= by[(1.0, 0.0)]
    assert res["bf16"][0]["matvecs"] <= by[(128.0, 64.0)] + 4
