"""Oracle solvers: rescaled BiCGStab and rescaled iterative refinement.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Every vector the low-precision solver stores is rounded to the storage
precision right after it is written (:func:`lowp`); scalars are FP64
throughout, as the paper treats them (Sec. 3, the remark that beta is an FP64
variable).  Arithmetic on stored values is done in FP64, which differs from a
GPU that computes in FP32 only below FP32 rounding.

Readings of the paper that these functions take (each is listed with its
reason in the design notes):

* Alg. 2 / Alg. 3 correction step.  The residual is rescaled to y = r * s/|r|
  and the low-precision solve gives A t ~ y~ with |y~| = s^ (or s).  The
  update that makes A dx = r is therefore x += (|r| / s^) * t, which is what
  :func:`solve_mixed_ir` does; the printed factor 1/s (Alg. 2) and 1/s^
  (Alg. 3) would not reduce the residual.
* Alg. 4 / Alg. 5 recalculated gamma.  The text describes it as the ratio of
  residual norms after and before rescaling; since its later uses (p, v
  rescaling, rho' = gamma rho, gamma' *= gamma) need gamma ~ sigma/g, the
  recalculated value is |r_stored| / g.
* Inner stopping test: (|r| / gamma')^2 <= eps_tol^2 * |b|^2, relative to the
  inner right-hand side.
* Alg. 5 returns the solution divided by the accumulated factor lambda'.
* FP64 -> FP16 conversion is one round-to-nearest-even step (IEEE 754
  format conversion), not two roundings through FP32.  The same holds for
  BF16 (Table 1: 8 exponent bits, 7 fraction bits, e_min = -126), which has
  no IEEE conversion of its own: the value is rounded once, to nearest even,
  to 8 significant bits (subnormal below 2^-126), exactly as the other
  formats are.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import OP_D, dslash

FP64, FP32, FP16, BF16 = "fp64", "fp32", "fp16", "bf16"
FP16_MIN_NORMAL = 2.0 ** -14  # smallest normal binary16 magnitude (Table 1: e_min = -14)
BF16_MIN_NORMAL = 2.0 ** -126  # Table 1: e_min = -126
BF16_SIGNIFICAND = 8           # Table 1: 7 fraction bits plus the implicit one
BF16_EMAX = 127                # Table 1


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Nearest BF16 value of each FP64 number, ties to even mantissa.

    A value in [2^E, 2^(E+1)) is a multiple of 2^(E - 7) in BF16; below
    2^-126 the spacing stays 2^-133 (subnormals).  Results beyond the largest
    finite value become infinities, as in IEEE rounding.
    """
    x = np.asarray(x, dtype=np.float64)
    out = x.copy()
    fin = np.isfinite(x) & (x != 0)
    v = x[fin]
    _, e = np.frexp(v)                      # v = m 2^e with 1/2 <= |m| < 1, i.e. E = e - 1
    q = np.maximum(e - BF16_SIGNIFICAND, -126 - (BF16_SIGNIFICAND - 1))
    r = np.ldexp(np.rint(np.ldexp(v, -q)), q)   # np.rint rounds halves to even
    big = np.abs(r) >= 2.0 ** (BF16_EMAX + 1)
    r[big] = np.copysign(np.inf, r[big])
    out[fin] = r
    return out


def lowp(v: np.ndarray, prec: str, ftz: bool = False) -> np.ndarray:
    """Round real and imaginary parts to the storage precision (RNE).

    Returns complex128 whose parts are exactly representable in ``prec``.
    With ``ftz`` a binary16 (BF16) result below the smallest normal becomes
    zero, as with the flush-to-zero compilation of the paper's runs (Sec. 6).
    """
    v = np.asarray(v, dtype=np.complex128)
    if prec == FP64:
        return v.copy()
    if prec == FP32:
        return v.astype(np.complex64).astype(np.complex128)
    if prec == FP16:
        re = v.real.astype(np.float16)
        im = v.imag.astype(np.float16)
        if ftz:
            re = np.where(np.abs(re) < FP16_MIN_NORMAL, np.float16(0) * re, re)
            im = np.where(np.abs(im) < FP16_MIN_NORMAL, np.float16(0) * im, im)
        out = np.empty(v.shape, dtype=np.complex128)
        out.real = re.astype(np.float64)
        out.imag = im.astype(np.float64)
        return out
    if prec == BF16:
        re, im = round_bf16(v.real), round_bf16(v.imag)
        if ftz:
            re = np.where(np.abs(re) < BF16_MIN_NORMAL, 0.0 * re, re)
            im = np.where(np.abs(im) < BF16_MIN_NORMAL, 0.0 * im, im)
        return re + 1j * im
    raise ValueError(f"unknown precision {prec!r}")


def norm2(v: np.ndarray) -> float:
    """|v|^2 in FP64."""
    return float(np.vdot(v, v).real)


def dot(a: np.ndarray, b: np.ndarray) -> complex:
    """(a, b) = sum conj(a) b in FP64."""
    return complex(np.vdot(a, b))


class LowPrecWilson:
    """A~ of Alg. 3: the Wilson matrix with links stored in ``prec`` applied
    to a stored vector, its result rounded to ``prec``."""

    def __init__(self, U, kappa, dims, prec, ftz=False):
        shape = U.shape
        self.U = lowp(U.reshape(-1), prec).reshape(shape)
        self.kappa, self.dims, self.prec, self.ftz = kappa, tuple(dims), prec, ftz
        self.count = 0

    def __call__(self, v):
        self.count += 1
        return lowp(dslash(self.U, v, self.kappa, self.dims, OP_D), self.prec, self.ftz)


@dataclass
class BicgstabInfo:
    iterations: int = 0
    matvecs: int = 0
    converged: bool = False
    nonfinite: bool = False
    breakdown: bool = False                        # rho = 0 or (r*, v) = 0
    history: list = field(default_factory=list)   # (|r| / gamma')^2 at each loop test
    betas: list = field(default_factory=list)
    gamma_cum: float = 1.0
    lambda_cum: float = 1.0


def bicgstab(A, b, prec=FP64, tol2=1e-24, maxiter=10000, sigma=None, recalc_gamma=True,
             sigma_lambda=None, omega0=0.7, rho_init=None, ftz=False, x_stored_out=None):
    """Rescaled BiCGStab of Alg. 4 (``sigma_lambda`` None) or Alg. 5.

    * ``sigma`` None keeps gamma = 1 at every step, which is the standard
      BiCGStab (Alg. 4 caption).
    * ``omega0`` is the omega prescription of the cited improvement.
    * ``rho_init`` None uses rho' = |r|^2 so that beta = 1 in the first
      iteration; a number reproduces other initialisations (e.g. 1.0).
    * x0 = 0, as in the paper's runs.
    Stops when (|r|/gamma')^2 <= tol2 * |b|^2.
    Returns (x, info) with x the unscaled solution in FP64.
    """
    st = lambda v: lowp(v, prec, ftz)
    b = st(b)
    x = np.zeros_like(b)
    r = b.copy()                       # r = b - A x0 with x0 = 0
    rstar = r.copy()
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    rho_prev = norm2(r) if rho_init is None else float(rho_init)
    omega_prev = alpha_prev = gamma_cum = 1.0
    lam_cum = 1.0
    bn2 = norm2(b)
    info = BicgstabInfo()
    rn2 = norm2(r)
    while True:
        res2 = rn2 / gamma_cum ** 2
        info.history.append(res2)
        if res2 <= tol2 * bn2:
            info.converged = True
            break
        if info.iterations >= maxiter:
            break
        rho = dot(rstar, r)
        if rho == 0:
            info.breakdown = True
            break
        beta = rho * alpha_prev / (rho_prev * omega_prev)
        info.betas.append(beta)
        p = st(beta * (p - omega_prev * v) + r)
        v = A(p)
        rv = dot(rstar, v)
        if rv == 0:
            info.breakdown = True
            break
        alpha = rho / rv
        r = st(r - alpha * v)
        t = A(r)
        tr, tt, rr = dot(t, r), norm2(t), norm2(r)
        omega = tr / tt
        omega_hat = abs(tr) / math.sqrt(tt * rr)
        if omega_hat < omega0:
            omega = omega * omega0 / omega_hat
        c = lam_cum / gamma_cum
        x = st(x + c * omega * r + c * alpha * p)
        r = st(r - omega * t)
        info.matvecs += 2
        info.iterations += 1
        if sigma is not None:
            g = math.sqrt(norm2(r))
            gamma = sigma / g
            r = st(gamma * r)
            if recalc_gamma:
                gamma = math.sqrt(norm2(r)) / g
            p = st(gamma * p)
            v = st(gamma * v)
        else:
            gamma = 1.0
        omega_prev, alpha_prev, rho_prev = omega, alpha, gamma * rho
        gamma_cum *= gamma
        if sigma_lambda is not None:
            lam = sigma_lambda / math.sqrt(norm2(x))
            x = st(lam * x)
            lam_cum *= lam
        rn2 = norm2(r)
        scal = (beta, alpha, omega, gamma_cum, lam_cum, rn2)
        if not all(np.isfinite(complex(z)) for z in scal):
            info.nonfinite = True
            break
    info.gamma_cum, info.lambda_cum = gamma_cum, lam_cum
    if x_stored_out is not None:
        x_stored_out.append(x.copy())
    return x / lam_cum, info


@dataclass
class IRInfo:
    outer: int = 0
    inner_iterations: int = 0
    matvec_low: int = 0
    matvec_fp64: int = 0
    converged: bool = False
    true_rel_residual: float = float("nan")
    history: list = field(default_factory=list)     # outer |r|/|b|
    shat_over_s: list = field(default_factory=list)
    zeros: list = field(default_factory=list)       # zero reals in y~ per outer step
    inner_infos: list = field(default_factory=list)


def solve_mixed_ir(U, kappa, dims, b, inner_prec=FP16, s=128.0, recalc_shat=True, inner_tol2=1e-4,
                   sigma=64.0, recalc_gamma=True, sigma_lambda=None, omega0=0.7, tol=1e-12,
                   max_outer=200, inner_maxiter=10000, ftz=False, inner_solver=None):
    """FP64 iterative refinement around a low-precision rescaled BiCGStab.

    Alg. 3 with ``recalc_shat``; Alg. 2 is s = 1 without it.  The outer
    residual r = b - D x is recomputed in FP64 after every correction.
    Stops when |b - D x| / |b| <= tol.
    """
    b = np.asarray(b, dtype=np.complex128)
    A_low = LowPrecWilson(U, kappa, dims, inner_prec, ftz)
    x = np.zeros_like(b)
    r = b.copy()
    bn = math.sqrt(norm2(b))
    info = IRInfo()
    if bn == 0.0:
        info.converged, info.true_rel_residual = True, 0.0
        return x, info
    rn = bn
    while True:
        info.history.append(rn / bn)
        if rn / bn <= tol:
            info.converged = True
            break
        if info.outer >= max_outer:
            break
        scale = s / rn
        y = scale * r
        yt = lowp(y, inner_prec, ftz)
        info.zeros.append(int(np.count_nonzero(yt.real == 0) + np.count_nonzero(yt.imag == 0)))
        shat = math.sqrt(norm2(yt)) if recalc_shat else s
        info.shat_over_s.append(shat / s)
        if inner_solver is None:
            t, ii = bicgstab(A_low, yt, inner_prec, tol2=inner_tol2, maxiter=inner_maxiter, sigma=sigma,
                             recalc_gamma=recalc_gamma, sigma_lambda=sigma_lambda, omega0=omega0, ftz=ftz)
        else:
            t, ii = inner_solver(yt)
        info.inner_infos.append(ii)
        info.inner_iterations += ii.iterations
        info.matvec_low += ii.matvecs
        x = x + (rn / shat) * t
        r = b - dslash(U, x, kappa, dims, OP_D)
        info.matvec_fp64 += 1
        info.outer += 1
        rn = math.sqrt(norm2(r))
        if not math.isfinite(rn):
            break
    info.true_rel_residual = rn / bn
    return x, info


def solve_fp64(U, kappa, dims, b, tol=1e-12, maxiter=20000, omega0=0.7):
    """Plain FP64 BiCGStab (Alg. 4 with gamma = 1) on the full Wilson matrix."""
    A = lambda v: dslash(U, v, kappa, dims, OP_D)
    return bicgstab(A, b, FP64, tol2=tol * tol, maxiter=maxiter, sigma=None, omega0=omega0)
