"""Python binding of libqcd (Wilson-Dirac mixed-precision solver for MI355X).

Argument marshalling only: every step runs in the HIP kernels of libqcd.so,
reached through its C ABI (``include/qcd.h``).  PyTorch supplies device
memory and the current stream.  There is no fallback: importing this module
without the built library raises.

Functions keep the C names without the ``qcd_`` prefix: :func:`gauge_upload`,
:func:`dslash`, :func:`bicgstab`, :func:`solve_mixed_ir`, :func:`convert`,
:func:`unconvert`, :func:`residual`.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqcd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2602_14450_amd/build.py (or __graft_entry__.build())")

_lib = ctypes.CDLL(LIB_PATH)

FP64, FP32, FP16, BF16 = 0, 1, 2, 3
PREC = {"fp64": FP64, "fp32": FP32, "fp16": FP16, "bf16": BF16, FP64: FP64, FP32: FP32, FP16: FP16,
        BF16: BF16}
CANONICAL, NATIVE = 0, 1
LINKS_FULL = 1 << 8
OP_D, OP_H, OP_DDAG, OP_HDAG, OP_SCHUR = 0, 1, 2, 3, 4
STATUS = {0: "ok", 1: "not_converged", -1: "err_arg", -2: "err_hip", -3: "err_nonfinite", -4: "err_workspace",
          -5: "err_unsupported", -6: "err_breakdown"}


class BicgstabParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("sigma", ctypes.c_double),
                ("sigma_lambda", ctypes.c_double), ("recalc_gamma", ctypes.c_int), ("omega0", ctypes.c_double),
                ("ftz", ctypes.c_int), ("check_every", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("even_odd", ctypes.c_int)]


class IRParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_outer", ctypes.c_int), ("inner_prec", ctypes.c_int),
                ("s", ctypes.c_double), ("recalc_shat", ctypes.c_int), ("inner", BicgstabParams),
                ("precond", ctypes.c_void_p), ("precond_scale", ctypes.c_double)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("inner_iters", ctypes.c_int), ("matvec_low", ctypes.c_int),
                ("matvec_fp64", ctypes.c_int), ("true_rel_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("inner_status", ctypes.c_int), ("first_shat_over_s", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int),
                ("history_len", ctypes.c_int), ("outer_history", ctypes.POINTER(ctypes.c_double)),
                ("outer_history_cap", ctypes.c_int), ("zeros", ctypes.POINTER(ctypes.c_double)),
                ("precond_steps", ctypes.c_int), ("precond_fallback", ctypes.c_int),
                ("precond_scale", ctypes.c_double)]


_vp, _i, _d, _sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
_lib.qcd_last_error.restype = ctypes.c_char_p
_lib.qcd_gauge_upload.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(_i), _vp, _i, _vp]
_lib.qcd_gauge_free.argtypes = [_vp]
_lib.qcd_gauge_link_reals.argtypes = [_vp, _i]
_lib.qcd_gauge_link_reals.restype = _i
_lib.qcd_spinor_bytes.argtypes = [_vp, _i]
_lib.qcd_spinor_bytes.restype = _sz
_lib.qcd_workspace_bytes.argtypes = [_vp, _i, _i, _i, _i]
_lib.qcd_workspace_bytes.restype = _sz
_lib.qcd_convert.argtypes = [_vp, _i, _i, _vp, _vp, _d, _i, ctypes.POINTER(_d), _vp]
_lib.qcd_gaussian_spinors.argtypes = [_vp, ctypes.c_int64, ctypes.c_uint64, _vp]
_lib.qcd_unconvert.argtypes = [_vp, _i, _i, _vp, _vp, _d, _vp]
_lib.qcd_dslash.argtypes = [_vp, _d, _i, _i, _i, _i, _vp, _vp, _vp]
_lib.qcd_residual.argtypes = [_vp, _d, _i, _vp, _vp, _vp, ctypes.POINTER(_d), _vp]
_lib.qcd_bicgstab.argtypes = [_vp, _d, _i, _i, _vp, _vp, ctypes.POINTER(BicgstabParams), ctypes.POINTER(SolveInfo),
                              _vp, _sz, _vp]
_lib.qcd_solve_mixed_ir.argtypes = [_vp, _d, _i, _vp, _vp, ctypes.POINTER(IRParams), ctypes.POINTER(SolveInfo), _vp,
                                    _sz, _vp]
_lib.qcd_solve_mixed_ir_static.argtypes = [_vp, _d, _i, _vp, _vp, ctypes.POINTER(IRParams),
                                           ctypes.POINTER(SolveInfo), _vp]
_lib.qcd_solve_mixed_ir_static.restype = _i
_lib.qcd_solve_mixed_ir_batched.argtypes = [_i, ctypes.POINTER(_vp), ctypes.POINTER(_d), ctypes.POINTER(_i),
                                            ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(IRParams),
                                            ctypes.POINTER(ctypes.POINTER(SolveInfo)), ctypes.POINTER(_vp),
                                            ctypes.POINTER(_sz), _vp]
_lib.qcd_solve_mixed_ir_batched.restype = _i
_lib.qcd_set_dslash_tuning.argtypes = [_vp, _i, _i, _i, _i]
_lib.qcd_stream_probe.argtypes = [_vp, _vp, _sz, _i, _i, ctypes.POINTER(_d), _vp]
_lib.qcd_stream_probe.restype = _i
_lib.qcd_autotune_dslash.argtypes = [_vp, _i, _i, _i, ctypes.c_char_p, ctypes.POINTER(_d), _vp]
_lib.qcd_get_dslash_tuning.argtypes = [_vp, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]
_lib.qcd_ptc_create.argtypes = [ctypes.POINTER(_vp), _vp, _i, ctypes.POINTER(_i), _i, _vp]
_lib.qcd_ptc_free.argtypes = [_vp]
_lib.qcd_ptc_num_weights.argtypes = [_vp]
_lib.qcd_ptc_num_weights.restype = _sz
_lib.qcd_ptc_set_weights.argtypes = [_vp, _vp, _vp]
_lib.qcd_ptc_get_weights.argtypes = [_vp, _vp, _vp]
_lib.qcd_ptc_apply.argtypes = [_vp, _i, _vp, _vp, _vp]
_lib.qcd_ptc_apply_prec.argtypes = [_vp, _i, _i, _vp, _vp, _vp]
_lib.qcd_eo_spectrum.argtypes = [_vp, _d, _i, _i, ctypes.c_uint64, ctypes.POINTER(_d), ctypes.POINTER(_d), _vp]
_lib.qcd_ptc_loss_grad.argtypes = [_vp, _i, _vp, _vp, ctypes.POINTER(_d), _vp, _vp]
_lib.qcd_ptc_train_step.argtypes = [_vp, _i, _vp, _vp, _d, ctypes.POINTER(_d), _vp]
_lib.qcd_ptc_set_gauge.argtypes = [_vp, _vp]
_lib.qcd_ptc_set_mixing.argtypes = [_vp, _i, _vp]
_lib.qcd_ptc_loss_grad_residual.argtypes = [_vp, _d, _i, _vp, ctypes.POINTER(_d), _vp, _vp]
_lib.qcd_ptc_train_step_residual.argtypes = [_vp, _d, _i, _vp, _d, ctypes.POINTER(_d), _vp]
_lib.qcd_ptc_init_neumann.argtypes = [_vp, _d, _vp]
for _f in ("qcd_ptc_create", "qcd_ptc_free", "qcd_ptc_set_weights", "qcd_ptc_get_weights", "qcd_ptc_apply",
           "qcd_ptc_apply_prec", "qcd_eo_spectrum",
           "qcd_ptc_loss_grad", "qcd_ptc_train_step", "qcd_ptc_set_gauge", "qcd_ptc_init_neumann",
           "qcd_ptc_set_mixing", "qcd_ptc_loss_grad_residual", "qcd_ptc_train_step_residual",
           "qcd_autotune_dslash", "qcd_set_dslash_tuning", "qcd_get_dslash_tuning", "qcd_gauge_upload", "qcd_gauge_free", "qcd_convert",
           "qcd_unconvert", "qcd_dslash", "qcd_residual", "qcd_bicgstab", "qcd_solve_mixed_ir"):
    getattr(_lib, _f).restype = _i

EXPORTED = ["qcd_last_error", "qcd_gauge_link_reals", "qcd_autotune_dslash", "qcd_set_dslash_tuning", "qcd_get_dslash_tuning", "qcd_gauge_upload", "qcd_gauge_free",
            "qcd_spinor_bytes", "qcd_workspace_bytes", "qcd_convert", "qcd_unconvert", "qcd_dslash", "qcd_residual", "qcd_bicgstab", "qcd_solve_mixed_ir", "qcd_solve_mixed_ir_static", "qcd_solve_mixed_ir_batched",
            "qcd_ptc_create", "qcd_ptc_free", "qcd_ptc_num_weights", "qcd_ptc_set_weights", "qcd_ptc_get_weights",
            "qcd_ptc_apply", "qcd_ptc_apply_prec", "qcd_ptc_loss_grad", "qcd_ptc_train_step", "qcd_ptc_set_gauge", "qcd_ptc_init_neumann",
            "qcd_ptc_set_mixing", "qcd_ptc_loss_grad_residual", "qcd_ptc_train_step_residual",
            "qcd_gaussian_spinors", "qcd_eo_spectrum", "qcd_stream_probe"]


class QcdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def _check(code, allow=(0,)):
    if code not in allow:
        raise QcdError(code, _lib.qcd_last_error().decode())
    return code


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    assert t.is_cuda and t.is_contiguous(), "expected a contiguous device tensor"
    return ctypes.c_void_p(t.data_ptr())


def _as_c128(t: torch.Tensor) -> torch.Tensor:
    assert t.dtype == torch.complex128, "canonical fields are complex128"
    return t.contiguous()


class Gauge:
    """A gauge field uploaded to the device in the native layout (FP64 plus
    the selected low-precision copies)."""

    def __init__(self, U: torch.Tensor, dims, precs=(FP64, FP32, FP16, BF16), full_links=False):
        U = _as_c128(U)
        self.dims = tuple(int(d) for d in dims)
        mask = LINKS_FULL if full_links else 0
        for p in precs:
            mask |= 1 << PREC[p]
        h = ctypes.c_void_p()
        d = (ctypes.c_int * 4)(*self.dims)
        _check(_lib.qcd_gauge_upload(ctypes.byref(h), d, _ptr(U), mask, _stream()))
        self.handle = h
        self.volume = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]

    def close(self):
        if self.handle:
            _lib.qcd_gauge_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def link_reals(self, prec) -> int:
        """Reals stored per link in prec: 12 (SU(3) rows 0, 1; row 2 rebuilt) or 18."""
        return int(_lib.qcd_gauge_link_reals(self.handle, PREC[prec]))

    def set_tuning(self, prec, sched: int, variant: int, rhs_tile: int = 0):
        _check(_lib.qcd_set_dslash_tuning(self.handle, PREC[prec], int(sched), int(variant), int(rhs_tile)))

    def get_tuning(self, prec):
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(_lib.qcd_get_dslash_tuning(self.handle, PREC[prec], ctypes.byref(a), ctypes.byref(b),
                                          ctypes.byref(c)))
        return a.value, b.value, c.value

    def eo_spectrum(self, kappa, power_iters=1000, inverse_iters=40, seed=1):
        """(largest, smallest) |eigenvalue| estimates of the even-odd matrix
        1 - kappa^2 H_eo H_oe (qcd_eo_spectrum); smallest is NaN when
        inverse_iters = 0."""
        hi, lo = _d(), _d()
        _check(_lib.qcd_eo_spectrum(self.handle, float(kappa), int(power_iters), int(inverse_iters),
                                    int(seed) & (2**64 - 1), ctypes.byref(hi), ctypes.byref(lo), _stream()))
        return hi.value, lo.value

    def autotune(self, prec, nrhs=1, reps=20, cache_path=None):
        """Time the launch choices of the Wilson operator and keep the fastest;
        cache_path defaults to $QCD_TUNE_CACHE.  Returns (sched, variant, rhs_tile, us)."""
        if cache_path is None:
            cache_path = os.environ.get("QCD_TUNE_CACHE")
        us = ctypes.c_double(0.0)
        _check(_lib.qcd_autotune_dslash(self.handle, PREC[prec], int(nrhs), int(reps),
                                        cache_path.encode() if cache_path else None, ctypes.byref(us), _stream()))
        return (*self.get_tuning(prec), us.value)

    def nrhs_of(self, t: torch.Tensor) -> int:
        """Number of canonical spinor fields a complex128 tensor holds."""
        per = self.volume * 12
        assert t.numel() % per == 0, "tensor is not a whole number of spinor fields"
        return t.numel() // per

    def spinor_bytes(self, prec) -> int:
        return int(_lib.qcd_spinor_bytes(self.handle, PREC[prec]))

    def workspace_bytes(self, what, prec, max_iter, nrhs=1) -> int:
        return int(_lib.qcd_workspace_bytes(self.handle, int(what), PREC[prec], int(max_iter), int(nrhs)))

    def native_spinor(self, prec, nrhs=1) -> torch.Tensor:
        """An uninitialised device buffer for nrhs native spinor fields."""
        return torch.empty(self.spinor_bytes(prec) * nrhs, dtype=torch.uint8, device="cuda")


def gauge_upload(U, dims, precs=(FP64, FP32, FP16, BF16), full_links=False) -> Gauge:
    return Gauge(U, dims, precs, full_links)


def _one_or_list(vals, n):
    return vals[0] if n == 1 else list(vals)


def stream_probe(nbytes=1 << 30, reps=20):
    """GB/s of plain 16-byte streaming sweeps (qcd_stream_probe): read-only,
    copy (bytes read + written) and write-only, on fresh device buffers."""
    nbytes -= nbytes % 16
    src = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = {}
    for mode, name, moved in ((0, "read", 1), (1, "copy", 2), (2, "write", 1)):
        us = ctypes.c_double()
        _check(_lib.qcd_stream_probe(_ptr(dst), _ptr(src), nbytes, mode, int(reps), ctypes.byref(us), _stream()))
        out[name + "_GBps"] = moved * nbytes / (us.value * 1e-6) / 1e9
    del src, dst
    return out


def gaussian_spinors(shape, seed: int) -> torch.Tensor:
    """A complex128 device tensor of the given shape (e.g. (n, V, 4, 3)) of
    complex normal values with E|z|^2 = 1, generated on the device from a
    counter-based stream keyed by seed."""
    out = torch.empty(shape, dtype=torch.complex128, device="cuda")
    _check(_lib.qcd_gaussian_spinors(_ptr(out), out.numel(), int(seed) & (2**64 - 1), _stream()))
    return out


def convert(g: Gauge, prec, native: torch.Tensor, canonical: torch.Tensor, scale=1.0, ftz=False, want_norm=True):
    """native = round_prec(scale * canonical); returns |native|^2 per right-hand side."""
    n = g.nrhs_of(canonical)
    n2 = (ctypes.c_double * n)()
    _check(_lib.qcd_convert(g.handle, PREC[prec], n, _ptr(native), _ptr(_as_c128(canonical)), float(scale), int(ftz),
                            n2 if want_norm else None, _stream()))
    return _one_or_list(n2, n) if want_norm else None


def unconvert(g: Gauge, prec, canonical: torch.Tensor, native: torch.Tensor, scale=1.0):
    n = g.nrhs_of(canonical)
    _check(_lib.qcd_unconvert(g.handle, PREC[prec], n, _ptr(canonical), _ptr(native), float(scale), _stream()))


def dslash(g: Gauge, kappa, out: torch.Tensor, inp: torch.Tensor, op=OP_D, prec=FP64, layout=CANONICAL, nrhs=None):
    """out = op(inp); nrhs defaults to the number of canonical fields in inp (native layout: 1)."""
    if nrhs is None:
        nrhs = g.nrhs_of(inp) if layout == CANONICAL else 1
    _check(_lib.qcd_dslash(g.handle, float(kappa), int(op), PREC[prec], int(layout), int(nrhs), _ptr(out), _ptr(inp),
                           _stream()))
    return out


def residual(g: Gauge, kappa, r: torch.Tensor, x: torch.Tensor, b: torch.Tensor):
    n = g.nrhs_of(b)
    n2 = (ctypes.c_double * n)()
    _check(_lib.qcd_residual(g.handle, float(kappa), n, _ptr(r), _ptr(_as_c128(x)), _ptr(_as_c128(b)), n2,
                             _stream()))
    return _one_or_list(n2, n)


@dataclass
class Info:
    status: str
    outer_iters: int
    inner_iters: int
    matvec_low: int
    matvec_fp64: int
    true_rel_residual: float
    seconds: float
    inner_status: int
    first_shat_over_s: float
    history: list = field(default_factory=list)
    outer_history: list = field(default_factory=list)
    zeros: list = field(default_factory=list)
    precond_steps: int = 0
    precond_fallback: int = -1
    precond_scale: float = 0.0


def _bicg_params(tol, max_iter, sigma, sigma_lambda, recalc_gamma, omega0, ftz, check_every, use_graph=False,
                 even_odd=False):
    return BicgstabParams(float(tol), int(max_iter), float(sigma or 0.0), float(sigma_lambda or 0.0),
                          int(bool(recalc_gamma)), float(omega0), int(bool(ftz)), int(check_every),
                          int(bool(use_graph)), int(bool(even_odd)))


def _make_infos(n, hist_cap, outer_cap):
    infos = (SolveInfo * n)()
    keep = []
    for i in range(n):
        hist = (ctypes.c_double * max(hist_cap, 1))()
        outer = (ctypes.c_double * max(outer_cap, 1))()
        zeros = (ctypes.c_double * max(outer_cap, 1))()
        infos[i].history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        infos[i].history_cap = hist_cap
        infos[i].outer_history = ctypes.cast(outer, ctypes.POINTER(ctypes.c_double))
        infos[i].outer_history_cap = outer_cap
        infos[i].zeros = ctypes.cast(zeros, ctypes.POINTER(ctypes.c_double))
        keep.append((hist, outer, zeros))
    return infos, keep


def _infos_out(code, infos, keep):
    out = []
    for info, (hist, outer, zeros) in zip(infos, keep):
        n_out = min(info.outer_iters, info.outer_history_cap)
        out.append(Info(STATUS.get(code, str(code)), info.outer_iters, info.inner_iters, info.matvec_low,
                        info.matvec_fp64, info.true_rel_residual, info.seconds, info.inner_status,
                        info.first_shat_over_s, list(hist[:info.history_len]), list(outer[:n_out]),
                        list(zeros[:n_out]), info.precond_steps, info.precond_fallback, info.precond_scale))
    return out[0] if len(out) == 1 else out


def bicgstab(g: Gauge, kappa, x: torch.Tensor, b: torch.Tensor, prec=FP64, tol=1e-12, max_iter=10000, sigma=0.0,
             sigma_lambda=0.0, recalc_gamma=True, omega0=0.7, ftz=False, check_every=0, workspace=None,
             history=True, raise_on_error=True, use_graph=False, even_odd=False):
    """Rescaled BiCGStab (Alg. 4 / 5) on canonical complex128 device vectors
    (one or several right-hand sides); returns an Info or a list of them.
    even_odd: solve the even-odd system of eq. (4)-(6)."""
    n = g.nrhs_of(b)
    p = _bicg_params(tol, max_iter, sigma, sigma_lambda, recalc_gamma, omega0, ftz, check_every, use_graph, even_odd)
    infos, keep = _make_infos(n, max_iter if history else 0, 1)
    ws = _ptr(workspace) if workspace is not None else None
    wsb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    code = _lib.qcd_bicgstab(g.handle, float(kappa), PREC[prec], n, _ptr(x), _ptr(_as_c128(b)), ctypes.byref(p),
                             infos, ws, wsb, _stream())
    if raise_on_error:
        _check(code, allow=(0, 1))
    return _infos_out(code, infos, keep)


def solve_mixed_ir(g: Gauge, kappa, x: torch.Tensor, b: torch.Tensor, inner_prec=FP16, tol=1e-12, max_outer=100,
                   s=128.0, recalc_shat=True, inner_tol=1e-2, inner_max_iter=10000, sigma=64.0, sigma_lambda=0.0,
                   recalc_gamma=True, omega0=0.7, ftz=False, check_every=0, workspace=None, history=False,
                   raise_on_error=True, use_graph=False, precond=None, precond_scale=0.0, even_odd=False):
    """FP64 iterative refinement (Alg. 3 / 2) around the rescaled BiCGStab,
    for one or several right-hand sides; returns an Info or a list of them.
    precond: a PTC network used as right preconditioner of the FP16 inner
    solve (flexible refinement with fallback to the plain step)."""
    n = g.nrhs_of(b)
    inner = _bicg_params(inner_tol, inner_max_iter, sigma, sigma_lambda, recalc_gamma, omega0, ftz, check_every,
                         use_graph, even_odd)
    p = IRParams(float(tol), int(max_outer), PREC[inner_prec], float(s), int(bool(recalc_shat)), inner,
                 precond.handle if precond is not None else None, float(precond_scale))
    infos, keep = _make_infos(n, inner_max_iter * 4 if history else 0, max_outer)
    ws = _ptr(workspace) if workspace is not None else None
    wsb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    code = _lib.qcd_solve_mixed_ir(g.handle, float(kappa), n, _ptr(x), _ptr(_as_c128(b)), ctypes.byref(p), infos,
                                   ws, wsb, _stream())
    if raise_on_error:
        _check(code, allow=(0, 1))
    return _infos_out(code, infos, keep)


def solve_mixed_ir_static(g: Gauge, kappa, x: torch.Tensor, b: torch.Tensor, inner_prec=FP16, tol=1e-12,
                          max_outer=100, s=128.0, recalc_shat=True, inner_tol=1e-2, inner_max_iter=10000, sigma=64.0,
                          sigma_lambda=0.0, recalc_gamma=True, omega0=0.7, ftz=False, check_every=0, history=False,
                          raise_on_error=True, even_odd=False):
    """solve_mixed_ir with the library's static device workspace (no device
    allocation; workspace of at most 64 MiB, no graph, no network)."""
    n = g.nrhs_of(b)
    inner = _bicg_params(inner_tol, inner_max_iter, sigma, sigma_lambda, recalc_gamma, omega0, ftz, check_every,
                         False, even_odd)
    p = IRParams(float(tol), int(max_outer), PREC[inner_prec], float(s), int(bool(recalc_shat)), inner, None, 0.0)
    infos, keep = _make_infos(n, inner_max_iter * 4 if history else 0, max_outer)
    code = _lib.qcd_solve_mixed_ir_static(g.handle, float(kappa), n, _ptr(x), _ptr(_as_c128(b)), ctypes.byref(p),
                                          infos, _stream())
    if raise_on_error:
        _check(code, allow=(0, 1))
    return _infos_out(code, infos, keep)


class PTC:
    """Gauge-covariant parallel-transport network on the lattice of a Gauge
    (which must hold FP32 links), usable as a right preconditioner.

    channels: fields per layer boundary, e.g. (1, 2, 2, 1).  Weights are a
    list of complex arrays (9, C_out, C_in, 4, 4), one per layer."""

    def __init__(self, g: Gauge, channels=(1, 2, 2, 1), max_batch=1):
        self.gauge = g
        self.channels = tuple(int(c) for c in channels)
        self.max_batch = int(max_batch)
        h = ctypes.c_void_p()
        ch = (ctypes.c_int * len(self.channels))(*self.channels)
        _check(_lib.qcd_ptc_create(ctypes.byref(h), g.handle, len(self.channels) - 1, ch, self.max_batch, _stream()))
        self.handle = h
        self.nweights = int(_lib.qcd_ptc_num_weights(h))

    def close(self):
        if self.handle is not None and self.handle.value:
            _lib.qcd_ptc_free(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_gauge(self, g: Gauge):
        """Bind the network to another gauge field of the same extents (keeps weights and Adam state)."""
        _check(_lib.qcd_ptc_set_gauge(self.handle, g.handle))
        self.gauge = g

    def init_neumann(self, kappa):
        """Weights of M = sum_{k<=3} (kappa H)^k (channels 1, 2, 2, 1)."""
        _check(_lib.qcd_ptc_init_neumann(self.handle, float(kappa), _stream()))

    def _shapes(self):
        return [(9, co, ci, 4, 4) for ci, co in zip(self.channels[:-1], self.channels[1:])]

    def set_weights(self, Ws):
        import numpy as np
        flat = np.concatenate([np.asarray(W, dtype=np.complex128).reshape(-1) for W in Ws])
        assert flat.size == self.nweights, (flat.size, self.nweights)
        flat = np.ascontiguousarray(flat)
        _check(_lib.qcd_ptc_set_weights(self.handle, flat.ctypes.data, _stream()))

    def _unflatten(self, flat):
        out, o = [], 0
        for sh in self._shapes():
            n = 9 * sh[1] * sh[2] * 16
            out.append(flat[o:o + n].reshape(sh).copy())
            o += n
        return out

    def get_weights(self):
        import numpy as np
        flat = np.empty(self.nweights, dtype=np.complex128)
        _check(_lib.qcd_ptc_get_weights(self.handle, flat.ctypes.data, _stream()))
        return self._unflatten(flat)

    def apply(self, out: torch.Tensor, inp: torch.Tensor):
        """out = M(inp) for one field (V, 4, 3) or a batch (B, V, 4, 3), complex128."""
        nb = 1 if inp.dim() == 3 else inp.shape[0]
        _check(_lib.qcd_ptc_apply(self.handle, nb, _ptr(out), _ptr(_as_c128(inp)), _stream()))
        return out

    def apply_prec(self, out: torch.Tensor, inp: torch.Tensor, prec: int):
        """out = M(inp) with activations stored in prec (FP32, or FP16 as the inner solver applies it)."""
        nb = 1 if inp.dim() == 3 else inp.shape[0]
        _check(_lib.qcd_ptc_apply_prec(self.handle, prec, nb, _ptr(out), _ptr(_as_c128(inp)), _stream()))
        return out

    def loss_grad(self, r: torch.Tensor, e: torch.Tensor, want_grad=True):
        import numpy as np
        nb = 1 if r.dim() == 3 else r.shape[0]
        loss = ctypes.c_double()
        flat = np.empty(self.nweights, dtype=np.complex128) if want_grad else None
        _check(_lib.qcd_ptc_loss_grad(self.handle, nb, _ptr(_as_c128(r)), _ptr(_as_c128(e)), ctypes.byref(loss),
                                      flat.ctypes.data if want_grad else None, _stream()))
        return (loss.value, self._unflatten(flat)) if want_grad else loss.value

    def set_mixing(self, prec):
        """Channel mixing of the two-pass form in BF16 (default) or FP32."""
        _check(_lib.qcd_ptc_set_mixing(self.handle, PREC[prec], _stream()))

    def loss_grad_residual(self, kappa, r: torch.Tensor, want_grad=True):
        """Residual loss mean |D M r - r|^2 / |r|^2 and (optionally) its weight gradient."""
        import numpy as np
        nb = 1 if r.dim() == 3 else r.shape[0]
        loss = ctypes.c_double()
        flat = np.empty(self.nweights, dtype=np.complex128) if want_grad else None
        _check(_lib.qcd_ptc_loss_grad_residual(self.handle, float(kappa), nb, _ptr(_as_c128(r)), ctypes.byref(loss),
                                               flat.ctypes.data if want_grad else None, _stream()))
        return (loss.value, self._unflatten(flat)) if want_grad else loss.value

    def train_step_residual(self, kappa, r: torch.Tensor, lr=1e-3):
        """One Adam step on the residual loss; returns the loss before the step."""
        nb = 1 if r.dim() == 3 else r.shape[0]
        loss = ctypes.c_double()
        _check(_lib.qcd_ptc_train_step_residual(self.handle, float(kappa), nb, _ptr(_as_c128(r)), float(lr),
                                                ctypes.byref(loss), _stream()))
        return loss.value

    def train_step(self, r: torch.Tensor, e: torch.Tensor, lr=1e-3):
        nb = 1 if r.dim() == 3 else r.shape[0]
        loss = ctypes.c_double()
        _check(_lib.qcd_ptc_train_step(self.handle, nb, _ptr(_as_c128(r)), _ptr(_as_c128(e)), float(lr),
                                       ctypes.byref(loss), _stream()))
        return loss.value


def solve_mixed_ir_batched(gauges, kappas, xs, bs, inner_prec=FP16, tol=1e-12, max_outer=100, s=128.0,
                           recalc_shat=True, inner_tol=1e-2, inner_max_iter=10000, sigma=64.0, sigma_lambda=0.0,
                           recalc_gamma=True, omega0=0.7, ftz=False, check_every=0, history=False,
                           raise_on_error=True, use_graph=False, even_odd=False, workspaces=None):
    """Several lattices (distinct Gauge handles, any extents) solved together:
    one refinement whose inner solves run concurrently.  xs[i], bs[i] hold one
    or several canonical fields of lattice i.  workspaces: None (the handles'
    own) or one device buffer per lattice (None entries: that handle's own).
    Returns a list (per lattice) of Info or lists of Info."""
    nl = len(gauges)
    ns = [g.nrhs_of(b) for g, b in zip(gauges, bs)]
    inner = _bicg_params(inner_tol, inner_max_iter, sigma, sigma_lambda, recalc_gamma, omega0, ftz, check_every,
                         use_graph, even_odd)
    p = IRParams(float(tol), int(max_outer), PREC[inner_prec], float(s), int(bool(recalc_shat)), inner, None, 0.0)
    made = [_make_infos(n, inner_max_iter * 4 if history else 0, max_outer) for n in ns]
    gh = (ctypes.c_void_p * nl)(*[g.handle.value for g in gauges])
    kp = (ctypes.c_double * nl)(*[float(k) for k in kappas])
    npp = (ctypes.c_int * nl)(*ns)
    bcs = [_as_c128(b) for b in bs]
    xp = (ctypes.c_void_p * nl)(*[_ptr(x).value for x in xs])
    bp = (ctypes.c_void_p * nl)(*[_ptr(b).value for b in bcs])
    ip = (ctypes.POINTER(SolveInfo) * nl)(*[ctypes.cast(m[0], ctypes.POINTER(SolveInfo)) for m in made])
    wsp = wsb = None
    if workspaces is not None:
        assert len(workspaces) == nl, "one workspace (or None) per lattice"
        wsp = (ctypes.c_void_p * nl)(*[(_ptr(w).value if w is not None else None) for w in workspaces])
        wsb = (ctypes.c_size_t * nl)(*[(w.numel() * w.element_size() if w is not None else 0) for w in workspaces])
    code = _lib.qcd_solve_mixed_ir_batched(nl, gh, kp, npp, xp, bp, ctypes.byref(p), ip, wsp, wsb, _stream())
    if raise_on_error:
        _check(code, allow=(0, 1))
    out = []
    for (infos, keep) in made:
        out.append(_infos_out(code, infos, keep))
    return out
