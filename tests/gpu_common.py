"""Helpers shared by the GPU parity tests (imported only by tests marked gpu)."""
import numpy as np
import torch

import qcd_inputs as qi

# Tolerances: relative to the oracle's rms element (element-wise) and in
# norm.  FP64: reordering of the sums only.  FP32: link and input rounding
# (2^-24) and FP32 accumulation over ~100 terms.  FP16: storage rounding
# (2^-11) of links, input and output.  BF16: the same with 2^-8.
TOL = {0: 1e-14, 1: 1e-6, 2: 5e-3, 3: 4e-2}


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy()


def compare(got: np.ndarray, want: np.ndarray, tol: float, what: str = ""):
    """Element-wise |got - want| <= tol * rms(want), and norm-relative error <= tol."""
    got = got.reshape(-1)
    want = want.reshape(-1)
    rms = np.sqrt(np.mean(np.abs(want) ** 2))
    err = np.abs(got - want)
    worst = int(np.argmax(err))
    assert err[worst] <= tol * rms, f"{what}: element {worst} differs by {err[worst]:.3e} (rms {rms:.3e}, tol {tol})"
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert rel <= tol, f"{what}: norm-relative error {rel:.3e} > {tol}"
    return rel


def fields(dims, eps=0.3, gseed=101, sseed=102):
    return qi.gauge_field(dims, eps, gseed), qi.gaussian_source(dims, sseed)
