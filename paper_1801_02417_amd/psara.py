"""ctypes binding of libpsara.so (the C ABI declared in include/psara.h).

Argument marshalling only: every computation runs in the library's HIP kernels.  The
module-level functions carry the C names; `Solver` bundles them for convenience.  Host
arrays are numpy float64 (images N x 4, coefficients J x 4) or complex128 (visibilities
M x 4).  If the shared library has not been built this module raises on first use; there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsara.so")

PSARA_OK, PSARA_EINVAL, PSARA_ENOMEM, PSARA_EDEVICE, PSARA_ESTATE, PSARA_ENAN = 0, -1, -2, -3, -4, -5
PSARA_FP64, PSARA_FP32_MIXED = 0, 1
PSARA_CONSTRAINED, PSARA_NNLS_INIT, PSARA_UNCONSTRAINED = 0, 1, 2

ALL_BASES = 0x1FF      # Dirac + Db1..Db8

EXPORTS = (
    "psara_create", "psara_destroy", "psara_last_error", "psara_status_string", "psara_set_operator",
    "psara_set_data", "psara_set_data_dev", "psara_get_image_dev", "psara_set_prior", "psara_set_steps", "psara_opnorm", "psara_solve", "psara_reweight",
    "psara_coef_std", "psara_reweighted_solve", "psara_report_now", "psara_synchronize", "psara_get_image",
    "psara_state_bytes",
    "psara_get_state", "psara_set_state", "psara_reset_state", "psara_footprint", "psara_apply_phi",
    "psara_apply_phi_adjoint", "psara_apply_psi_adjoint", "psara_apply_psi", "psara_wavelet_filter",
    "psara_kb_beta", "psara_kb_value", "psara_kb_deapod", "psara_layout", "psara_profile_passes",
    "psara_batch_solve", "psara_batch_reweighted_solve", "psara_batch_profile_passes", "psara_data_gamma",
    "psara_set_gamma", "psara_set_mueller", "psara_set_prior_tv", "psara_solve_adaptive", "psara_reweighted_solve_adaptive", "psara_batch_solve_adaptive",
    "psara_server_create", "psara_server_submit", "psara_server_poll", "psara_server_drain",
    "psara_server_clock", "psara_server_last_error", "psara_server_destroy", "psara_runtime_check",
    "psara_step_sizes", "psara_set_steps_auto", "psara_capture", "psara_solve_noalloc", "psara_server_cancel",
    "psara_get_tuning", "psara_set_tuning", "psara_autotune", "psara_batch_autotune", "psara_tuning_lookup",
)

PSARA_TUNE_USE_CACHE, PSARA_TUNE_STORE = 1, 2

PSARA_SERVE_BATCHED, PSARA_SERVE_FIFO = 0, 1
PSARA_REQ_QUEUED, PSARA_REQ_RUNNING, PSARA_REQ_DONE, PSARA_REQ_FAILED, PSARA_REQ_CANCELLED = 0, 1, 2, 3, 4


class PsaraReport(C.Structure):
    _fields_ = [("residual", C.c_double), ("epsilon", C.c_double), ("rel_var", C.c_double * 4),
                ("zeta", C.c_double), ("n_p", C.c_double), ("objective", C.c_double),
                ("vnorm", C.c_double), ("iterations", C.c_int64)]

    def as_dict(self) -> dict:
        return {"residual": self.residual, "epsilon": self.epsilon, "rel_var": list(self.rel_var),
                "zeta": self.zeta, "n_p": self.n_p, "objective": self.objective, "vnorm": self.vnorm,
                "iterations": int(self.iterations)}


class PsaraTuning(C.Structure):
    _fields_ = [("grid_chunk", C.c_int), ("degrid_item", C.c_int), ("analysis_wide", C.c_int), ("fft_cells", C.c_int)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


DEFAULT_TUNING = {"grid_chunk": 1024, "degrid_item": 256, "analysis_wide": 1, "fft_cells": 0}


class PsaraStop(C.Structure):
    _fields_ = [("theta", C.c_double), ("rel_var", C.c_double), ("np_max", C.c_double)]


# the stopping criteria of the paper's simulations (theta, relative variation, N_p in percent)
PAPER_STOP = (5e-3, 1e-5, 0.5)


class PsaraRequest(C.Structure):
    _fields_ = [("n", C.c_int), ("M", C.c_int64), ("uv", C.POINTER(C.c_double)), ("Y", C.POINTER(C.c_double)),
                ("epsilon", C.c_double), ("taps", C.c_int), ("levels", C.c_int), ("basis_mask", C.c_uint32),
                ("precision", C.c_int), ("mode", C.c_int), ("cycles", C.c_int),
                ("iters_per_stage", C.POINTER(C.c_int)), ("delta_decay", C.c_double),
                ("gamma_factor", C.c_double), ("opnorm_iters", C.c_int), ("opnorm_rtol", C.c_double),
                ("check_every", C.c_int), ("stop", PsaraStop)]


class PsaraResult(C.Structure):
    _fields_ = [("state", C.c_int), ("status", C.c_int), ("t_submit", C.c_double), ("t_start", C.c_double),
                ("t_done", C.c_double), ("n", C.c_int), ("report", PsaraReport)]


class PsaraError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"psara error {status}: {message}")
        self.status = status


_lib_handle = None


def lib() -> C.CDLL:
    """Load libpsara.so (raises if it has not been built)."""
    global _lib_handle
    if _lib_handle is not None:
        return _lib_handle
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1801_02417_amd.build`")
    L = C.CDLL(LIB_PATH)
    P, D, I, I64, U32, S = C.c_void_p, C.POINTER(C.c_double), C.c_int, C.c_int64, C.c_uint32, C.c_size_t
    sig = {
        "psara_create": (I, [C.POINTER(P), I, P]),
        "psara_destroy": (None, [P]),
        "psara_last_error": (C.c_char_p, [P]),
        "psara_status_string": (C.c_char_p, [I]),
        "psara_set_operator": (I, [P, I, I64, D, I, I, I]),
        "psara_set_data": (I, [P, D, C.c_double]),
        "psara_set_data_dev": (I, [P, P, C.c_double]),
        "psara_get_image_dev": (I, [P, P]),
        "psara_set_prior": (I, [P, U32, I, D, C.c_double]),
        "psara_set_steps": (I, [P, C.c_double, C.c_double, C.c_double, C.c_double]),
        "psara_runtime_check": (I, [C.POINTER(I), C.POINTER(I)]),
        "psara_step_sizes": (I, [I, C.c_double, C.c_double, D]),
        "psara_set_steps_auto": (I, [P, C.c_double, D]),
        "psara_capture": (I, [P, I, I, I]),
        "psara_solve_noalloc": (I, [P, I, I]),
        "psara_get_tuning": (I, [P, C.POINTER(PsaraTuning)]),
        "psara_set_tuning": (I, [P, C.POINTER(PsaraTuning)]),
        "psara_autotune": (I, [P, I, I, C.POINTER(PsaraTuning), D]),
        "psara_batch_autotune": (I, [C.POINTER(P), I, I, C.POINTER(PsaraTuning), D]),
        "psara_tuning_lookup": (I, [I, I64, I, I, U32, I, C.POINTER(PsaraTuning)]),
        "psara_opnorm": (I, [P, I, C.c_double, D]),
        "psara_solve": (I, [P, I, I, I, C.POINTER(PsaraReport)]),
        "psara_set_mueller": (I, [P, D]),
        "psara_set_prior_tv": (I, [P, I, D, D]),
        "psara_solve_adaptive": (I, [P, I, I, I, C.POINTER(PsaraStop), C.POINTER(C.c_int), C.POINTER(PsaraReport)]),
        "psara_reweighted_solve_adaptive": (I, [P, I, I, I, I, C.POINTER(PsaraStop), C.c_double,
                                                C.POINTER(C.c_int), C.POINTER(PsaraReport)]),
        "psara_batch_solve_adaptive": (I, [C.POINTER(P), I, I, I, I, C.POINTER(PsaraStop), C.POINTER(C.c_int),
                                           C.POINTER(PsaraReport)]),
        "psara_reweight": (I, [P, C.c_double]),
        "psara_coef_std": (I, [P, D]),
        "psara_reweighted_solve": (I, [P, I, I, C.POINTER(C.c_int), C.c_double, C.POINTER(PsaraReport)]),
        "psara_report_now": (I, [P, C.POINTER(PsaraReport)]),
        "psara_synchronize": (I, [P]),
        "psara_get_image": (I, [P, D]),
        "psara_state_bytes": (S, [P]),
        "psara_get_state": (I, [P, P, S]),
        "psara_set_state": (I, [P, P, S]),
        "psara_reset_state": (I, [P]),
        "psara_footprint": (S, [I, I64, I, I, U32, I]),
        "psara_apply_phi": (I, [P, D, D]),
        "psara_apply_phi_adjoint": (I, [P, D, D]),
        "psara_apply_psi_adjoint": (I, [P, D, D]),
        "psara_apply_psi": (I, [P, D, D]),
        "psara_wavelet_filter": (I, [I, D]),
        "psara_kb_beta": (C.c_double, [I, C.c_double]),
        "psara_kb_value": (C.c_double, [I, C.c_double, C.c_double]),
        "psara_kb_deapod": (C.c_double, [I, C.c_double, C.c_double]),
        "psara_layout": (I, [P, C.POINTER(C.c_int64)]),
        "psara_profile_passes": (I, [P, I, I, D]),
        "psara_batch_solve": (I, [C.POINTER(P), I, I, I, C.POINTER(PsaraReport)]),
        "psara_batch_profile_passes": (I, [C.POINTER(P), I, I, I, D]),
        "psara_data_gamma": (I, [P, C.c_double, D]),
        "psara_set_gamma": (I, [P, C.c_double]),
        "psara_server_create": (I, [C.POINTER(P), I, S, I, I, I]),
        "psara_server_submit": (I, [P, C.POINTER(PsaraRequest), C.POINTER(C.c_uint64)]),
        "psara_server_poll": (I, [P, C.c_uint64, C.POINTER(PsaraResult), D]),
        "psara_server_drain": (I, [P]),
        "psara_server_cancel": (I, [P, C.c_uint64]),
        "psara_server_clock": (C.c_double, [P]),
        "psara_server_last_error": (C.c_char_p, [P]),
        "psara_server_destroy": (None, [P]),
        "psara_batch_reweighted_solve": (I, [C.POINTER(P), I, I, I, C.POINTER(C.c_int), C.c_double,
                                             C.POINTER(PsaraReport)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib_handle = L
    return L


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None) -> np.ndarray:
    out = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and out.shape != tuple(shape):
        out = out.reshape(shape)
    return out


def _vis(a: np.ndarray) -> np.ndarray:
    """complex (M, 4) -> interleaved float64 (M, 8)."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a.view(np.float64).reshape(a.shape[0], 8)


def _check(ctx, status: int):
    if status != PSARA_OK:
        msg = lib().psara_last_error(ctx).decode() if ctx else lib().psara_status_string(status).decode()
        raise PsaraError(status, msg)


# ---- C-named functions --------------------------------------------------------------------------
def psara_runtime_check():
    """(status, built, running): the HIP runtime versions the library was built for and runs on."""
    built, running = C.c_int(), C.c_int()
    st = lib().psara_runtime_check(C.byref(built), C.byref(running))
    return st, built.value, running.value


def _create_error(st: int) -> PsaraError:
    msg = lib().psara_status_string(st).decode()
    rc, built, running = psara_runtime_check()
    if rc != PSARA_OK:
        msg += f" (HIP runtime {running} in this process, library built for {built})"
    return PsaraError(st, msg)


def psara_create(device: int = 0, hip_stream: Optional[int] = None):
    ctx = C.c_void_p()
    st = lib().psara_create(C.byref(ctx), device, C.c_void_p(hip_stream) if hip_stream else None)
    if st != PSARA_OK:
        raise _create_error(st)
    return ctx


def psara_destroy(ctx) -> None:
    lib().psara_destroy(ctx)


def psara_set_operator(ctx, n: int, uv: np.ndarray, oversample: int = 2, taps: int = 8,
                       precision: int = PSARA_FP32_MIXED) -> None:
    uv = _f64(uv)
    _check(ctx, lib().psara_set_operator(ctx, n, uv.shape[0], _dptr(uv), oversample, taps, precision))


def psara_set_data(ctx, Y: np.ndarray, epsilon: float) -> None:
    y = _vis(Y)
    _check(ctx, lib().psara_set_data(ctx, _dptr(y), float(epsilon)))


def psara_set_data_dev(ctx, Y_dev: int, epsilon: float) -> None:
    """Y_dev: the device address (an integer, e.g. a tensor's data_ptr()) of M x 4 complex128."""
    _check(ctx, lib().psara_set_data_dev(ctx, C.c_void_p(int(Y_dev)), float(epsilon)))


def psara_set_prior(ctx, basis_mask: int, levels: int, weights: Optional[np.ndarray], gamma: float) -> None:
    if weights is None:
        _check(ctx, lib().psara_set_prior(ctx, basis_mask, levels, None, float(gamma)))
    else:
        w = _f64(weights)
        _check(ctx, lib().psara_set_prior(ctx, basis_mask, levels, _dptr(w), float(gamma)))


def psara_set_steps(ctx, tau: float, rho1: float, rho2: float, rho3: float) -> None:
    _check(ctx, lib().psara_set_steps(ctx, tau, rho1, rho2, rho3))


def psara_step_sizes(prior: int, phi_norm_sq: float, margin: float = 0.99):
    """(tau, rho1, rho2, rho3) the library picks for prior 0 (SARA), 1 (TV) or 2 (l1 + TV)."""
    out = np.zeros(4)
    st = lib().psara_step_sizes(int(prior), float(phi_norm_sq), float(margin), _dptr(out))
    if st != PSARA_OK:
        raise PsaraError(st, lib().psara_status_string(st).decode())
    return tuple(float(v) for v in out)


def psara_set_steps_auto(ctx, margin: float = 0.99):
    out = np.zeros(4)
    _check(ctx, lib().psara_set_steps_auto(ctx, float(margin), _dptr(out)))
    return tuple(float(v) for v in out)


def psara_opnorm(ctx, max_iter: int = 500, rtol: float = 1e-10) -> float:
    out = C.c_double()
    _check(ctx, lib().psara_opnorm(ctx, max_iter, rtol, C.byref(out)))
    return out.value


def psara_solve(ctx, mode: int, iters: int, check_every: int = 0, report: bool = True):
    rep = PsaraReport()
    _check(ctx, lib().psara_solve(ctx, mode, iters, check_every, C.byref(rep) if report else None))
    return rep.as_dict() if report else None


def psara_solve_noalloc(ctx, mode: int, iters: int) -> None:
    _check(ctx, lib().psara_solve_noalloc(ctx, mode, iters))


def psara_get_tuning(ctx) -> dict:
    t = PsaraTuning()
    _check(ctx, lib().psara_get_tuning(ctx, C.byref(t)))
    return t.as_dict()


def psara_set_tuning(ctx, tuning: Optional[dict] = None) -> None:
    """Launch shapes from a dict with the keys of DEFAULT_TUNING (missing keys: defaults), or
    None for the defaults."""
    if tuning is None:
        _check(ctx, lib().psara_set_tuning(ctx, None))
        return
    t = PsaraTuning(**{**DEFAULT_TUNING, **tuning})
    _check(ctx, lib().psara_set_tuning(ctx, C.byref(t)))


def psara_autotune(ctx, mode: int = PSARA_CONSTRAINED, flags: int = 0):
    """(chosen shapes, [ms per iteration of the starting shapes, of the chosen ones])."""
    t, ms = PsaraTuning(), np.zeros(2)
    _check(ctx, lib().psara_autotune(ctx, mode, flags, C.byref(t), _dptr(ms)))
    return t.as_dict(), [float(v) for v in ms]


def psara_batch_autotune(ctxs, mode: int = PSARA_CONSTRAINED):
    t, ms = PsaraTuning(), np.zeros(2)
    _batch_check(ctxs, lib().psara_batch_autotune(_ctx_array(ctxs), len(ctxs), mode, C.byref(t), _dptr(ms)))
    return t.as_dict(), [float(v) for v in ms]


def psara_tuning_lookup(n: int, M: int, taps: int, levels: int, basis_mask: int = ALL_BASES,
                        precision: int = PSARA_FP32_MIXED) -> Optional[dict]:
    t = PsaraTuning()
    st = lib().psara_tuning_lookup(n, M, taps, levels, basis_mask, precision, C.byref(t))
    return t.as_dict() if st == PSARA_OK else None


def psara_capture(ctx, mode: int, iters: int, check_every: int = 0) -> None:
    _check(ctx, lib().psara_capture(ctx, mode, iters, check_every))


def psara_solve_adaptive(ctx, mode: int, max_iters: int, check_every: int, stop=PAPER_STOP):
    """Iterations until the criteria stop = (theta, rel_var, np_max) hold (checked on the device
    every check_every iterations) or max_iters; returns (iterations run, report)."""
    st, rep, it = PsaraStop(*[float(v) for v in stop]), PsaraReport(), C.c_int(0)
    _check(ctx, lib().psara_solve_adaptive(ctx, mode, max_iters, check_every, C.byref(st), C.byref(it),
                                           C.byref(rep)))
    return it.value, rep.as_dict()


def psara_reweighted_solve_adaptive(ctx, mode: int, cycles: int, max_iters_per_stage: int, check_every: int,
                                    stop=PAPER_STOP, delta_decay: float = 10.0):
    """Algorithm 2 with adaptive stages; returns (iterations per stage, report)."""
    st, rep = PsaraStop(*[float(v) for v in stop]), PsaraReport()
    its = (C.c_int * (cycles + 1))()
    _check(ctx, lib().psara_reweighted_solve_adaptive(ctx, mode, cycles, max_iters_per_stage, check_every,
                                                      C.byref(st), float(delta_decay), its, C.byref(rep)))
    return list(its), rep.as_dict()


def psara_batch_solve_adaptive(ctxs, mode: int, max_iters: int, check_every: int, stop=PAPER_STOP):
    """Batched adaptive stage; returns (iterations per member, reports)."""
    st = PsaraStop(*[float(v) for v in stop])
    its = (C.c_int * len(ctxs))()
    reps = (PsaraReport * len(ctxs))()
    _batch_check(ctxs, lib().psara_batch_solve_adaptive(_ctx_array(ctxs), len(ctxs), mode, max_iters, check_every,
                                                        C.byref(st), its, reps))
    return list(its), [r.as_dict() for r in reps]


def psara_set_prior_tv(ctx, tv_weight, l1_weight=None) -> None:
    """TV (l1_weight None) or l1 + TV prior of Algorithm 3; weights: 4 per-Stokes values."""
    tw = _f64(np.asarray(tv_weight, dtype=np.float64).reshape(4))
    lw = None if l1_weight is None else _f64(np.asarray(l1_weight, dtype=np.float64).reshape(4))
    _check(ctx, lib().psara_set_prior_tv(ctx, 0 if lw is None else 1, _dptr(tw), _dptr(lw) if lw is not None else None))


def psara_set_mueller(ctx, D) -> None:
    """Known direction-independent Mueller matrices (M, 4, 4) complex of the rows, or None."""
    if D is None:
        _check(ctx, lib().psara_set_mueller(ctx, None))
        return
    d = np.ascontiguousarray(np.asarray(D, dtype=np.complex128))
    if d.ndim != 3 or d.shape[1:] != (4, 4):
        raise ValueError("D must be (M, 4, 4)")
    flat = np.ascontiguousarray(d.view(np.float64).reshape(-1))
    _check(ctx, lib().psara_set_mueller(ctx, _dptr(flat)))


def psara_reweight(ctx, delta: float) -> None:
    _check(ctx, lib().psara_reweight(ctx, float(delta)))


def psara_coef_std(ctx) -> float:
    out = C.c_double()
    _check(ctx, lib().psara_coef_std(ctx, C.byref(out)))
    return out.value


def psara_reweighted_solve(ctx, mode: int, iters_per_stage: Sequence[int], delta_decay: float = 10.0):
    arr = (C.c_int * len(iters_per_stage))(*[int(v) for v in iters_per_stage])
    rep = PsaraReport()
    _check(ctx, lib().psara_reweighted_solve(ctx, mode, len(iters_per_stage) - 1, arr, delta_decay, C.byref(rep)))
    return rep.as_dict()


def psara_report_now(ctx) -> dict:
    rep = PsaraReport()
    _check(ctx, lib().psara_report_now(ctx, C.byref(rep)))
    return rep.as_dict()


def psara_synchronize(ctx) -> None:
    _check(ctx, lib().psara_synchronize(ctx))


def psara_get_image(ctx, N: int) -> np.ndarray:
    out = np.empty((N, 4))
    _check(ctx, lib().psara_get_image(ctx, _dptr(out)))
    return out


def psara_get_image_dev(ctx, S_dev: int) -> None:
    """S_dev: the device address of N x 4 doubles."""
    _check(ctx, lib().psara_get_image_dev(ctx, C.c_void_p(int(S_dev))))


def psara_state_bytes(ctx) -> int:
    return int(lib().psara_state_bytes(ctx))


def psara_get_state(ctx) -> np.ndarray:
    nb = psara_state_bytes(ctx)
    buf = np.empty(nb // 8)
    _check(ctx, lib().psara_get_state(ctx, buf.ctypes.data_as(C.c_void_p), nb))
    return buf


def psara_set_state(ctx, buf: np.ndarray) -> None:
    buf = _f64(buf)
    _check(ctx, lib().psara_set_state(ctx, buf.ctypes.data_as(C.c_void_p), buf.nbytes))


def psara_reset_state(ctx) -> None:
    _check(ctx, lib().psara_reset_state(ctx))


def psara_footprint(n: int, M: int, taps: int, levels: int, basis_mask: int = ALL_BASES,
                    precision: int = PSARA_FP32_MIXED) -> int:
    return int(lib().psara_footprint(n, M, taps, levels, basis_mask, precision))


def psara_apply_phi(ctx, S: np.ndarray, M: int) -> np.ndarray:
    S = _f64(S)
    out = np.empty((M, 8))
    _check(ctx, lib().psara_apply_phi(ctx, _dptr(S), _dptr(out)))
    return out.view(np.complex128).reshape(M, 4)


def psara_apply_phi_adjoint(ctx, B: np.ndarray, N: int) -> np.ndarray:
    b = _vis(B)
    out = np.empty((N, 4))
    _check(ctx, lib().psara_apply_phi_adjoint(ctx, _dptr(b), _dptr(out)))
    return out


def psara_apply_psi_adjoint(ctx, S: np.ndarray, J: int) -> np.ndarray:
    S = _f64(S)
    out = np.empty((J, 4))
    _check(ctx, lib().psara_apply_psi_adjoint(ctx, _dptr(S), _dptr(out)))
    return out


def psara_apply_psi(ctx, A: np.ndarray, N: int) -> np.ndarray:
    A = _f64(A)
    out = np.empty((N, 4))
    _check(ctx, lib().psara_apply_psi(ctx, _dptr(A), _dptr(out)))
    return out


def psara_wavelet_filter(p: int) -> np.ndarray:
    out = np.zeros(16)
    k = lib().psara_wavelet_filter(p, _dptr(out))
    if k == 0:
        raise ValueError(f"bad wavelet order {p}")
    return out[:k].copy()


def psara_kb_beta(taps: int, alpha: float) -> float:
    return lib().psara_kb_beta(taps, alpha)


def psara_kb_value(taps: int, beta: float, t: float) -> float:
    return lib().psara_kb_value(taps, beta, t)


def psara_kb_deapod(taps: int, beta: float, nu: float) -> float:
    return lib().psara_kb_deapod(taps, beta, nu)


def psara_layout(ctx, M: int):
    perm = np.empty(M, dtype=np.int64)
    ts = lib().psara_layout(ctx, perm.ctypes.data_as(C.POINTER(C.c_int64)))
    if ts < 0:
        raise PsaraError(ts, "layout unavailable")
    return ts, perm


PASS_NAMES = ("P1+P4 primal/epigraph/Dirac dual + zero-pad + row FFT", "P2+P3 SARA analysis + dual A + synthesis",
              "(in P2+P3)", "(in P1+P4)", "P5 column FFT", "P6 de-grid + dual B", "P7 grid",
              "P8 column inverse FFT (+ split-tile sums)", "P9 row inverse FFT + crop",
              "P9+P1+P4 fused (row inverse FFT, primal step, row FFT)",
              "P6+P7 fused (de-grid + dual B + grid)")
N_PASSES = len(PASS_NAMES)


def psara_profile_passes(ctx, mode: int, iters: int) -> np.ndarray:
    out = np.zeros(N_PASSES)
    _check(ctx, lib().psara_profile_passes(ctx, mode, iters, _dptr(out)))
    return out


def _ctx_array(ctxs):
    arr = (C.c_void_p * len(ctxs))(*[c.value if isinstance(c, C.c_void_p) else c for c in ctxs])
    return arr


def _batch_check(ctxs, status: int):
    if status != PSARA_OK:
        raise PsaraError(status, lib().psara_last_error(ctxs[0]).decode() if ctxs else "empty batch")


def psara_batch_solve(ctxs, mode: int, iters: int, report: bool = True):
    """One batched stage over several contexts; returns one report per context (or None)."""
    reps = (PsaraReport * len(ctxs))()
    st = lib().psara_batch_solve(_ctx_array(ctxs), len(ctxs), mode, iters, reps if report else None)
    _batch_check(ctxs, st)
    return [r.as_dict() for r in reps] if report else None


def psara_batch_profile_passes(ctxs, mode: int, iters: int) -> np.ndarray:
    """Per-pass milliseconds of one batched launch of each pass (as psara_profile_passes)."""
    out = np.zeros(N_PASSES)
    _batch_check(ctxs, lib().psara_batch_profile_passes(_ctx_array(ctxs), len(ctxs), mode, iters, _dptr(out)))
    return out


def psara_batch_reweighted_solve(ctxs, mode: int, iters_per_stage: Sequence[int], delta_decay: float = 10.0):
    arr = (C.c_int * len(iters_per_stage))(*[int(v) for v in iters_per_stage])
    reps = (PsaraReport * len(ctxs))()
    st = lib().psara_batch_reweighted_solve(_ctx_array(ctxs), len(ctxs), mode, len(iters_per_stage) - 1, arr,
                                            delta_decay, reps)
    _batch_check(ctxs, st)
    return [r.as_dict() for r in reps]


def psara_data_gamma(ctx, factor: float = 1e-3) -> float:
    out = C.c_double()
    _check(ctx, lib().psara_data_gamma(ctx, float(factor), C.byref(out)))
    return out.value


def psara_set_gamma(ctx, gamma: float) -> None:
    _check(ctx, lib().psara_set_gamma(ctx, float(gamma)))


def psara_server_create(device: int = 0, hbm_budget: int = 64 << 30, max_slots: int = 64, quantum: int = 25,
                        policy: int = PSARA_SERVE_BATCHED):
    srv = C.c_void_p()
    st = lib().psara_server_create(C.byref(srv), device, int(hbm_budget), max_slots, quantum, policy)
    if st != PSARA_OK:
        raise _create_error(st)
    return srv


def _server_check(srv, status: int):
    if status != PSARA_OK:
        raise PsaraError(status, lib().psara_server_last_error(srv).decode())


def psara_server_submit(srv, n: int, uv: np.ndarray, Y: np.ndarray, epsilon: float, taps: int = 8, levels: int = 4,
                        basis_mask: int = ALL_BASES, precision: int = PSARA_FP32_MIXED,
                        mode: int = PSARA_CONSTRAINED, iters_per_stage: Sequence[int] = (100, 100, 100),
                        delta_decay: float = 10.0, gamma_factor: float = 1e-3, opnorm_iters: int = 200,
                        opnorm_rtol: float = 1e-6, check_every: int = 0, stop=PAPER_STOP) -> int:
    """Queue a request; with check_every > 0 its stages end when `stop` holds on the device
    (iters_per_stage are then the bounds, multiples of check_every)."""
    uv = _f64(uv)
    y = _vis(Y)
    stages = (C.c_int * len(iters_per_stage))(*[int(v) for v in iters_per_stage])
    req = PsaraRequest(n, uv.shape[0], _dptr(uv), _dptr(y), float(epsilon), taps, levels, basis_mask, precision,
                       mode, len(iters_per_stage) - 1, stages, float(delta_decay), float(gamma_factor),
                       opnorm_iters, float(opnorm_rtol), int(check_every), PsaraStop(*[float(v) for v in stop]))
    ticket = C.c_uint64()
    _server_check(srv, lib().psara_server_submit(srv, C.byref(req), C.byref(ticket)))
    return ticket.value


def psara_server_poll(srv, ticket: int, image: Optional[np.ndarray] = None) -> dict:
    """State of a request; with `image` (n*n x 4 float64) a finished request's image is copied
    there and the request is forgotten."""
    res = PsaraResult()
    ptr = _dptr(image) if image is not None else None
    _server_check(srv, lib().psara_server_poll(srv, C.c_uint64(ticket), C.byref(res), ptr))
    return {"state": res.state, "status": res.status, "t_submit": res.t_submit, "t_start": res.t_start,
            "t_done": res.t_done, "n": res.n, "report": res.report.as_dict()}


def psara_server_cancel(srv, ticket: int) -> None:
    _server_check(srv, lib().psara_server_cancel(srv, C.c_uint64(ticket)))


def psara_server_drain(srv) -> None:
    _server_check(srv, lib().psara_server_drain(srv))


def psara_server_clock(srv) -> float:
    return lib().psara_server_clock(srv)


def psara_server_destroy(srv) -> None:
    lib().psara_server_destroy(srv)


# ---- convenience wrapper ------------------------------------------------------------------------
def basis_count(mask: int) -> int:
    return bin(mask & 0x1FF).count("1")


class Solver:
    """One Polarized SARA solve on the GPU (owns a psara context)."""

    def __init__(self, n: int, uv: np.ndarray, taps: int = 8, precision: int = PSARA_FP32_MIXED,
                 device: int = 0, hip_stream: Optional[int] = None):
        self.ctx = psara_create(device, hip_stream)
        self.n, self.N, self.M = n, n * n, int(np.shape(uv)[0])
        psara_set_operator(self.ctx, n, uv, 2, taps, precision)
        self.mask = 0
        self.J = 0
        self.phi_norm_sq = None

    def close(self):
        if self.ctx:
            psara_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_data(self, Y, epsilon):
        psara_set_data(self.ctx, Y, epsilon)

    def set_prior(self, levels: int, gamma: float, basis_mask: int = ALL_BASES, weights=None):
        self.mask = basis_mask
        self.J = basis_count(basis_mask) * self.N
        self.tv_kind = 0
        psara_set_prior(self.ctx, basis_mask, levels, weights, gamma)

    def opnorm(self, max_iter: int = 500, rtol: float = 1e-10) -> float:
        self.phi_norm_sq = psara_opnorm(self.ctx, max_iter, rtol)
        return self.phi_norm_sq

    def set_steps(self, tau=None, rho1=None, rho2=None, rho3=None):
        """The given step sizes, or with none given the library's choice (psara_set_steps_auto)."""
        if tau is None:
            return psara_set_steps_auto(self.ctx)
        psara_set_steps(self.ctx, tau, rho1, rho2, rho3)
        return tau, rho1, rho2, rho3

    def set_prior_tv(self, tv_weight, l1_weight=None) -> None:
        psara_set_prior_tv(self.ctx, tv_weight, l1_weight)
        self.tv_kind = 1 if l1_weight is None else 2
        self.J = (2 if l1_weight is None else 3) * self.N

    def solve(self, mode: int, iters: int, check_every: int = 0, report: bool = True):
        return psara_solve(self.ctx, mode, iters, check_every, report)

    def capture(self, mode: int, iters: int, check_every: int = 0) -> None:
        psara_capture(self.ctx, mode, iters, check_every)

    def tuning(self) -> dict:
        return psara_get_tuning(self.ctx)

    def set_tuning(self, tuning: Optional[dict] = None) -> None:
        psara_set_tuning(self.ctx, tuning)

    def autotune(self, mode: int = PSARA_CONSTRAINED, flags: int = 0):
        return psara_autotune(self.ctx, mode, flags)

    def reweighted_solve(self, mode: int, iters_per_stage, delta_decay: float = 10.0):
        return psara_reweighted_solve(self.ctx, mode, iters_per_stage, delta_decay)

    def set_mueller(self, D) -> None:
        psara_set_mueller(self.ctx, D)

    def solve_adaptive(self, mode: int, max_iters: int, check_every: int, stop=PAPER_STOP):
        return psara_solve_adaptive(self.ctx, mode, max_iters, check_every, stop)

    def reweighted_solve_adaptive(self, mode: int, cycles: int, max_iters_per_stage: int, check_every: int,
                                  stop=PAPER_STOP, delta_decay: float = 10.0):
        return psara_reweighted_solve_adaptive(self.ctx, mode, cycles, max_iters_per_stage, check_every, stop,
                                               delta_decay)

    def image(self) -> np.ndarray:
        return psara_get_image(self.ctx, self.N)

    def phi(self, S):
        return psara_apply_phi(self.ctx, S, self.M)

    def phi_adjoint(self, B):
        return psara_apply_phi_adjoint(self.ctx, B, self.N)

    def psi_adjoint(self, S):
        return psara_apply_psi_adjoint(self.ctx, S, self.J)

    def psi(self, A):
        return psara_apply_psi(self.ctx, A, self.N)

    def state(self) -> dict:
        buf = psara_get_state(self.ctx)
        N, J, M = self.N, self.J, self.M
        o = 0
        out = {}
        for name, cnt, shape in (("S", 4 * N, (N, 4)), ("Z", 2 * N, (N, 2)), ("A", 4 * J, (J, 4)),
                                 ("B", 8 * M, None), ("C", 4 * N, (N, 4)), ("D", 2 * N, (N, 2))):
            v = buf[o:o + cnt]
            out[name] = v.view(np.complex128).reshape(M, 4).copy() if shape is None else v.reshape(shape).copy()
            o += cnt
        return out

    def set_state(self, S, Z, A, B, C, D):
        parts = [np.ravel(np.asarray(S, float)), np.ravel(np.asarray(Z, float)), np.ravel(np.asarray(A, float)),
                 np.ascontiguousarray(B, dtype=np.complex128).view(np.float64).ravel(),
                 np.ravel(np.asarray(C, float)), np.ravel(np.asarray(D, float))]
        psara_set_state(self.ctx, np.concatenate(parts))

    def report(self) -> dict:
        return psara_report_now(self.ctx)

    def synchronize(self) -> None:
        psara_synchronize(self.ctx)

    def reset(self):
        psara_reset_state(self.ctx)

    def profile_passes(self, mode: int, iters: int) -> np.ndarray:
        return psara_profile_passes(self.ctx, mode, iters)


def batch_solve(solvers: Sequence[Solver], mode: int, iters: int, report: bool = True):
    return psara_batch_solve([s.ctx for s in solvers], mode, iters, report)


def batch_solve_adaptive(solvers: Sequence[Solver], mode: int, max_iters: int, check_every: int, stop=PAPER_STOP):
    return psara_batch_solve_adaptive([s.ctx for s in solvers], mode, max_iters, check_every, stop)


def batch_autotune(solvers: Sequence[Solver], mode: int = PSARA_CONSTRAINED):
    return psara_batch_autotune([s.ctx for s in solvers], mode)


def batch_reweighted_solve(solvers: Sequence[Solver], mode: int, iters_per_stage, delta_decay: float = 10.0):
    return psara_batch_reweighted_solve([s.ctx for s in solvers], mode, iters_per_stage, delta_decay)
