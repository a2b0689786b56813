"""Python binding of the MI355X Smolyak library (libsg.so, C ABI in
include/sg.h).

Argument marshalling only: every step of the operator action and of the
propagation runs in the library's HIP kernels.  Device vectors are torch
complex128 tensors on a ROCm device; streams are torch streams.  There is no
fallback: if the native library is missing every call raises.

The function names are the C ABI's; `Problem` is a small convenience owner of
a problem handle.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

__all__ = [
    "SG_OK", "SG_EINVAL", "SG_ENOMEM", "SG_EDEVICE", "SG_EAGAIN", "SG_ENOTFOUND",
    "SG_ECANCELED", "SG_ETOL", "SG_FP64", "SG_MIXED", "SgError", "lib",
    "library_path", "sg_count_sizes", "sg_build_terms", "sg_build_terms_host",
    "sg_free", "sg_problem_info", "sg_basis_indices", "sg_term_levels",
    "sg_mapping_table", "sg_init_gaussian", "sg_apply_H", "sg_spectral_bounds",
    "sg_propagate_chebyshev", "sg_propagate", "sg_propagate_noalloc",
    "sg_noalloc_scratch_bytes", "SG_PROP_TAYLOR", "SG_PROP_RK", "SG_PROP_SIL",
    "SG_PROP_BS",
    "sg_set_timing", "sg_get_timing", "sg_set_mixed_threshold",
    "sg_tune_mixed", "sg_set_operator_form", "sg_set_schedule", "sg_tune_schedule",
    "sg_eigensolve", "sg_embed_basis",
    "sg_batch_create", "sg_batch_size", "sg_batch_propagate", "sg_batch_tune_schedule",
    "sg_batch_free",
    "ServeConfig", "sg_serve_create", "sg_serve_submit", "sg_serve_poll", "sg_serve_cancel",
    "sg_serve_counters", "sg_serve_destroy", "Problem",
    "VibronicDesc", "sg_vibronic_build", "sg_vibronic_free", "sg_vibronic_problem",
    "sg_vibronic_figures", "sg_vibronic_init", "sg_vibronic_apply", "sg_vibronic_bounds",
    "sg_vibronic_propagate", "Vibronic", "sg_set_potential",
]

SG_OK, SG_EINVAL, SG_ENOMEM, SG_EDEVICE = 0, -1, -2, -3
SG_EAGAIN, SG_ENOTFOUND, SG_ECANCELED, SG_ETOL = -4, -5, -6, -7
SG_FP64, SG_MIXED = 0, 1
SG_PROP_TAYLOR, SG_PROP_RK, SG_PROP_SIL, SG_PROP_BS = 1, 2, 3, 4

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def library_path() -> str:
    return os.path.join(_HERE, "libsg.so")


class SgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"sg status {status}: {message}")
        self.status = status


class ProblemDesc(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int32), ("L", ctypes.c_int32),
                ("nb_A", ctypes.c_int32), ("nb_B", ctypes.c_int32),
                ("nq_A", ctypes.c_int32), ("nq_B", ctypes.c_int32),
                ("omega", ctypes.POINTER(ctypes.c_double)),
                ("c", ctypes.POINTER(ctypes.c_double)),
                ("k", ctypes.POINTER(ctypes.c_double))]


class VibronicDesc(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int32), ("L", ctypes.c_int32),
                ("omega", ctypes.POINTER(ctypes.c_double)),
                ("E", ctypes.POINTER(ctypes.c_double)),
                ("kappa", ctypes.POINTER(ctypes.c_double)),
                ("lam", ctypes.POINTER(ctypes.c_double)),
                ("c2", ctypes.POINTER(ctypes.c_double))]


class Info(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int64), ("L", ctypes.c_int64),
                ("n_terms", ctypes.c_int64), ("n_cs", ctypes.c_int64),
                ("n_s", ctypes.c_int64), ("grid_literal", ctypes.c_int64),
                ("grid_active", ctypes.c_int64), ("max_term_basis", ctypes.c_int64),
                ("max_term_grid", ctypes.c_int64), ("flops_fp64", ctypes.c_double),
                ("flops_mixed", ctypes.c_double), ("sweep_flops_fp64", ctypes.c_double),
                ("sweep_flops_mixed", ctypes.c_double), ("bytes_fp64", ctypes.c_double),
                ("device_bytes", ctypes.c_int64), ("fp64_split", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("sweep_bytes", ctypes.c_double),
                ("reduce_bytes", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class PropStats(ctypes.Structure):
    _fields_ = [("steps_done", ctypes.c_int32), ("cheb_terms", ctypes.c_int32),
                ("applies", ctypes.c_int64), ("emin", ctypes.c_double),
                ("emax", ctypes.c_double), ("norm0", ctypes.c_double),
                ("energy0", ctypes.c_double), ("norm_last", ctypes.c_double),
                ("energy_last", ctypes.c_double), ("max_norm_drift", ctypes.c_double),
                ("max_energy_drift", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Timing(ctypes.Structure):
    _fields_ = [("sweep_ms", ctypes.c_double), ("sweep_launches", ctypes.c_int64),
                ("reduce_ms", ctypes.c_double), ("reduce_launches", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_P = ctypes.c_void_p
class ServeConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("prec", ctypes.c_int), ("check_every", ctypes.c_int32),
                ("tol", ctypes.c_double), ("mixed_threshold", ctypes.c_int32),
                ("compile_threads", ctypes.c_int32)]


class EigStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("applies", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("converged", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("D", ctypes.c_int32), ("L", ctypes.c_int32),
                ("n_cs", ctypes.c_int64), ("psi_host", ctypes.c_void_p),
                ("psi_capacity", ctypes.c_int64), ("stats", PropStats),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


# V(n, Q [n][D], out [n], user)
POTENTIAL_FN = ctypes.CFUNCTYPE(None, ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)

_SIGNATURES = {
    "sg_set_potential": (ctypes.c_int, [_P, POTENTIAL_FN, ctypes.c_void_p]),
    "sg_set_timing": (ctypes.c_int, [_P, ctypes.c_int32]),
    "sg_set_operator_form": (ctypes.c_int, [_P, ctypes.c_int32]),
    "sg_set_schedule": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32]),
    "sg_tune_schedule": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32), _P]),
    "sg_set_mixed_threshold": (ctypes.c_int, [_P, ctypes.c_int32]),
    "sg_tune_mixed": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_double), _P]),
    "sg_get_timing": (ctypes.c_int, [_P, ctypes.POINTER(Timing)]),
    "sg_last_error": (ctypes.c_char_p, []),
    "sg_count_sizes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "sg_build_terms": (ctypes.c_int, [ctypes.POINTER(ProblemDesc), ctypes.POINTER(_P)]),
    "sg_build_terms_host": (ctypes.c_int, [ctypes.POINTER(ProblemDesc), ctypes.POINTER(_P)]),
    "sg_free": (ctypes.c_int, [_P]),
    "sg_problem_info": (ctypes.c_int, [_P, ctypes.POINTER(Info)]),
    "sg_basis_indices": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "sg_term_levels": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32)]),
    "sg_mapping_table": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "sg_init_gaussian": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), _P,
                                        ctypes.POINTER(ctypes.c_double), _P]),
    "sg_apply_H": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P]),
    "sg_spectral_bounds": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double), _P]),
    "sg_propagate_chebyshev": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_int32,
                                              ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_int, ctypes.c_int32,
                                              ctypes.POINTER(PropStats),
                                              ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double), _P]),
    "sg_propagate": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_double, ctypes.c_int, ctypes.c_int32,
                                    ctypes.POINTER(PropStats), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double), _P]),
    "sg_propagate_noalloc": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                            ctypes.c_int, ctypes.c_int32,
                                            ctypes.POINTER(PropStats),
                                            ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_double), _P]),
    "sg_noalloc_scratch_bytes": (ctypes.c_int64, []),
    "sg_vibronic_build": (ctypes.c_int, [ctypes.POINTER(VibronicDesc), ctypes.POINTER(_P)]),
    "sg_vibronic_free": (ctypes.c_int, [_P]),
    "sg_vibronic_problem": (ctypes.c_int, [_P, ctypes.POINTER(_P)]),
    "sg_vibronic_figures": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double)]),
    "sg_vibronic_init": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, _P,
                                        _P]),
    "sg_vibronic_apply": (ctypes.c_int, [_P, _P, _P, _P]),
    "sg_vibronic_bounds": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double), _P]),
    "sg_vibronic_propagate": (ctypes.c_int, [_P, _P, ctypes.c_double, ctypes.c_int32,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_int32, ctypes.POINTER(PropStats),
                                             ctypes.POINTER(ctypes.c_double), _P]),
    "sg_batch_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int32, ctypes.POINTER(_P)]),
    "sg_batch_tune_schedule": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.c_int32,
                                              ctypes.c_int32, ctypes.c_int32,
                                              ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_double), _P]),
    "sg_batch_size": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int64)]),
    "sg_batch_propagate": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_double),
                                          ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                          ctypes.c_int, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(PropStats), _P]),
    "sg_batch_free": (ctypes.c_int, [_P]),
    "sg_eigensolve": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_double, _P, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_double), _P,
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(EigStats),
                                     _P]),
    "sg_embed_basis": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "sg_serve_create": (ctypes.c_int, [ctypes.POINTER(ServeConfig), ctypes.POINTER(_P)]),
    "sg_serve_submit": (ctypes.c_int, [_P, ctypes.POINTER(ProblemDesc),
                                       ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]),
    "sg_serve_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(Result)]),
    "sg_serve_cancel": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "sg_serve_counters": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "sg_serve_destroy": (ctypes.c_int, [_P]),
}


def lib() -> ctypes.CDLL:
    """Loads libsg.so (raises if it was not built)."""
    global _LIB
    if _LIB is None:
        # torch ships its own HIP runtime with the same SONAME as the system
        # one libsg.so links; loading torch first makes the dynamic loader
        # resolve libsg.so's HIP dependency to that already-loaded runtime, so
        # the process holds a single HIP runtime and device pointers and
        # streams from torch are valid in the library.
        import torch  # noqa: F401
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(
                f"native library {path} is missing: build it with "
                "`python -m paper_2111_13655_amd.build` (no fallback exists)")
        L = ctypes.CDLL(path)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _check(status: int):
    if status != SG_OK:
        msg = lib().sg_last_error()
        raise SgError(status, msg.decode() if msg else "")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _vec_ptr(t, n_cs: int, name: str):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous complex128 device tensor")
    if t.numel() != n_cs:
        raise ValueError(f"{name} has {t.numel()} entries, expected N_cs = {n_cs}")
    return ctypes.c_void_p(t.data_ptr())


def _make_desc(D, L, omega, c, k, nb, nq):
    omega = np.ascontiguousarray(omega, dtype=np.float64).reshape(D)
    c = np.ascontiguousarray(c, dtype=np.float64).reshape(D * D)
    kk = None if k is None else np.ascontiguousarray(k, dtype=np.float64).reshape(D * D)
    desc = ProblemDesc(D, L, nb[0], nb[1], nq[0], nq[1], _dptr(omega), _dptr(c),
                       _dptr(kk) if kk is not None else ctypes.POINTER(ctypes.c_double)())
    return desc, (omega, c, kk)  # keep arrays alive


# ---------------------------------------------------------------------------
# C ABI, one function each
# ---------------------------------------------------------------------------

def sg_count_sizes(D: int, L: int, nb_A: int = 1, nb_B: int = 2):
    out = (ctypes.c_int64 * 3)()
    _check(lib().sg_count_sizes(D, L, nb_A, nb_B, out))
    return int(out[0]), int(out[1]), int(out[2])


def sg_build_terms(D, L, omega, c, k=None, nb=(1, 2), nq=(2, 2)) -> ctypes.c_void_p:
    desc, keep = _make_desc(D, L, omega, c, k, nb, nq)
    h = _P()
    _check(lib().sg_build_terms(ctypes.byref(desc), ctypes.byref(h)))
    return h


def sg_build_terms_host(D, L, omega, c, k=None, nb=(1, 2), nq=(2, 2)) -> ctypes.c_void_p:
    desc, keep = _make_desc(D, L, omega, c, k, nb, nq)
    h = _P()
    _check(lib().sg_build_terms_host(ctypes.byref(desc), ctypes.byref(h)))
    return h


def sg_free(h) -> None:
    _check(lib().sg_free(h))


def sg_problem_info(h) -> dict:
    info = Info()
    _check(lib().sg_problem_info(h, ctypes.byref(info)))
    return info.as_dict()


def sg_basis_indices(h) -> np.ndarray:
    inf = sg_problem_info(h)
    out = np.zeros(inf["n_cs"] * inf["D"], dtype=np.int32)
    _check(lib().sg_basis_indices(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return out.reshape(inf["n_cs"], inf["D"])


def sg_term_levels(h):
    inf = sg_problem_info(h)
    lev = np.zeros(inf["n_terms"] * inf["D"], dtype=np.int32)
    co = np.zeros(inf["n_terms"], dtype=np.int32)
    _check(lib().sg_term_levels(h, lev.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                co.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return lev.reshape(inf["n_terms"], inf["D"]), co


def sg_mapping_table(h) -> np.ndarray:
    inf = sg_problem_info(h)
    mb = np.zeros(inf["n_s"], dtype=np.int32)
    _check(lib().sg_mapping_table(h, mb.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return mb


def sg_init_gaussian(h, shift, psi, stream=None) -> float:
    n_cs = sg_problem_info(h)["n_cs"]
    shift = np.ascontiguousarray(shift, dtype=np.float64)
    cap = ctypes.c_double()
    _check(lib().sg_init_gaussian(h, _dptr(shift), _vec_ptr(psi, n_cs, "psi"),
                                  ctypes.byref(cap), _stream_ptr(stream)))
    return cap.value


def sg_apply_H(h, psi_in, psi_out, precision: int = SG_FP64, stream=None, n_cs=None) -> None:
    if n_cs is None:
        n_cs = sg_problem_info(h)["n_cs"]
    _check(lib().sg_apply_H(h, _vec_ptr(psi_in, n_cs, "psi_in"),
                            _vec_ptr(psi_out, n_cs, "psi_out"), int(precision),
                            _stream_ptr(stream)))


def sg_spectral_bounds(h, iters: int = 40, stream=None):
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _check(lib().sg_spectral_bounds(h, iters, ctypes.byref(lo), ctypes.byref(hi),
                                    _stream_ptr(stream)))
    return lo.value, hi.value


def sg_propagate_chebyshev(h, psi, dt: float, nsteps: int, emin=math.nan, emax=math.nan,
                           tol: float = 1e-8, precision: int = SG_FP64,
                           check_every: int = 0, stream=None, traces: bool = False):
    """Returns (status, stats dict, norm trace, energy trace)."""
    n_cs = sg_problem_info(h)["n_cs"]
    st = PropStats()
    ntr = (nsteps // check_every + 2) if check_every > 0 else 2
    ntr = max(ntr, 2)
    nt = np.zeros(ntr)
    et = np.zeros(ntr)
    status = lib().sg_propagate_chebyshev(
        h, _vec_ptr(psi, n_cs, "psi"), float(dt), int(nsteps), float(emin), float(emax),
        float(tol), int(precision), int(check_every), ctypes.byref(st), _dptr(nt), _dptr(et),
        _stream_ptr(stream))
    if status not in (SG_OK, SG_ETOL):
        _check(status)
    d = st.as_dict()
    n = min(ntr, (d["steps_done"] // check_every + 2) if check_every > 0 else 2)
    return status, d, nt[:n], et[:n]


def sg_propagate(h, psi, dt: float, nsteps: int, method: int, order: int, tol: float = 0.0,
                 precision: int = SG_FP64, check_every: int = 0, stream=None):
    """Taylor / Runge-Kutta / short-iterative-Lanczos / Bulirsch-Stoer
    propagation in place.
    Returns (status, stats dict, norm trace, energy trace)."""
    return _propagate("sg_propagate", h, psi, dt, nsteps, method, order, tol, precision,
                      check_every, stream)


def sg_propagate_noalloc(h, psi, dt: float, nsteps: int, method: int, order: int,
                         tol: float = 0.0, precision: int = SG_FP64, check_every: int = 0,
                         stream=None):
    """sg_propagate with its work buffers in the library's fixed device array
    (no device allocation).  Same returns."""
    return _propagate("sg_propagate_noalloc", h, psi, dt, nsteps, method, order, tol, precision,
                      check_every, stream)


def sg_noalloc_scratch_bytes() -> int:
    return int(lib().sg_noalloc_scratch_bytes())


def _propagate(entry, h, psi, dt, nsteps, method, order, tol, precision, check_every, stream):
    n_cs = sg_problem_info(h)["n_cs"]
    st = PropStats()
    ntr = max((nsteps // check_every + 2) if check_every > 0 else 2, 2)
    nt = np.zeros(ntr)
    et = np.zeros(ntr)
    status = getattr(lib(), entry)(
        h, _vec_ptr(psi, n_cs, "psi"), float(dt), int(nsteps), int(method), int(order),
        float(tol), int(precision), int(check_every), ctypes.byref(st), _dptr(nt), _dptr(et),
        _stream_ptr(stream))
    if status not in (SG_OK, SG_ETOL):
        _check(status)
    d = st.as_dict()
    done = d["steps_done"]
    if done < nsteps:
        # stopped by the drift check at step `done`: checks at 0, ce, .., done
        n = 1 + (done // check_every if check_every > 0 else 0)
    else:
        # checks inside the loop, then the final one
        n = (0 if nsteps == 0 else 1 + ((nsteps - 1) // check_every if check_every > 0 else 0)) + 1
    n = min(n, ntr)
    return status, d, nt[:n], et[:n]


def sg_set_mixed_threshold(h, max_fp32_coeff: int) -> None:
    _check(lib().sg_set_mixed_threshold(h, int(max_fp32_coeff)))


def sg_tune_mixed(h, psi, tol: float = 1e-6, reps: int = 3, stream=None):
    """Returns (chosen threshold, its measured relative error)."""
    n_cs = sg_problem_info(h)["n_cs"]
    ch = ctypes.c_int32()
    er = ctypes.c_double()
    _check(lib().sg_tune_mixed(h, _vec_ptr(psi, n_cs, "psi"), float(tol), int(reps),
                               ctypes.byref(ch), ctypes.byref(er), _stream_ptr(stream)))
    return ch.value, er.value


def sg_set_potential(h, V) -> None:
    """Replaces the problem's polynomial couplings by the potential V: a
    function taking an (n, D) float64 array of points (mode 1 first) and
    returning their n values.  The library calls it only during this call;
    V=None restores the polynomial couplings.  An exception raised by V is
    re-raised here."""
    if V is None:
        _check(lib().sg_set_potential(h, POTENTIAL_FN(), None))
        return
    D = sg_problem_info(h)["D"]
    raised = []

    def thunk(n, Q, out, _user):
        res = np.ctypeslib.as_array(out, shape=(n,))
        if raised:
            res[:] = np.nan
            return
        try:
            pts = np.ctypeslib.as_array(Q, shape=(n, D))
            res[:] = np.asarray(V(pts), dtype=np.float64).reshape(n)
        except BaseException as exc:   # reported after the library returns
            raised.append(exc)
            res[:] = np.nan

    cb = POTENTIAL_FN(thunk)
    status = lib().sg_set_potential(h, cb, None)
    if raised:
        raise raised[0]
    _check(status)


def sg_set_operator_form(h, grid_kinetic: bool) -> None:
    _check(lib().sg_set_operator_form(h, int(grid_kinetic)))


def sg_set_schedule(h, block_min_grid: int = 0, packs_per_cu: int = 1) -> None:
    _check(lib().sg_set_schedule(h, int(block_min_grid), int(packs_per_cu)))


def sg_tune_schedule(h, psi, precision: int = SG_FP64, reps: int = 20, stream=None):
    """Returns the chosen (block_min_grid, packs_per_cu)."""
    n_cs = sg_problem_info(h)["n_cs"]
    g = ctypes.c_int32()
    s = ctypes.c_int32()
    _check(lib().sg_tune_schedule(h, _vec_ptr(psi, n_cs, "psi"), int(precision), int(reps),
                                  ctypes.byref(g), ctypes.byref(s), _stream_ptr(stream)))
    return g.value, s.value


def sg_set_timing(h, enable: bool) -> None:
    _check(lib().sg_set_timing(h, 1 if enable else 0))


def sg_get_timing(h) -> dict:
    t = Timing()
    _check(lib().sg_get_timing(h, ctypes.byref(t)))
    return t.as_dict()


def sg_eigensolve(h, nev: int, max_basis: int = 0, max_iter: int = 200, tol: float = 1e-9,
                  guess=None, evecs=None, stream=None):
    """Returns (status, eigenvalues, residual norms, stats).  guess: optional
    device complex128 tensor [nguess, N_cs]; evecs: optional device complex128
    tensor [nev, N_cs] that receives the eigenvectors."""
    n_cs = sg_problem_info(h)["n_cs"]
    if max_basis <= 0:
        max_basis = min(max(4 * nev, 16), 256)
    ev = np.zeros(nev)
    rn = np.zeros(nev)
    st = EigStats()
    g, ng = None, 0
    if guess is not None:
        if guess.dim() != 2 or guess.shape[1] != n_cs:
            raise ValueError("guess must be [nguess, N_cs]")
        _vec_ptr(guess.reshape(-1), guess.numel(), "guess")
        g, ng = ctypes.c_void_p(guess.data_ptr()), guess.shape[0]
    out = None
    if evecs is not None:
        _vec_ptr(evecs.reshape(-1), nev * n_cs, "evecs")
        out = ctypes.c_void_p(evecs.data_ptr())
    status = lib().sg_eigensolve(h, int(nev), int(max_basis), int(max_iter), float(tol), g, ng,
                                 _dptr(ev), out, _dptr(rn), ctypes.byref(st), _stream_ptr(stream))
    if status not in (SG_OK, SG_ETOL):
        _check(status)
    return status, ev, rn, st.as_dict()


def sg_embed_basis(h_from, h_to, x, y, stream=None) -> None:
    nf = sg_problem_info(h_from)["n_cs"]
    nt = sg_problem_info(h_to)["n_cs"]
    _check(lib().sg_embed_basis(h_from, h_to, _vec_ptr(x, nf, "x"), _vec_ptr(y, nt, "y"),
                                _stream_ptr(stream)))


def sg_batch_create(handles) -> ctypes.c_void_p:
    arr = (_P * len(handles))(*[h.value if isinstance(h, _P) else h for h in handles])
    b = _P()
    _check(lib().sg_batch_create(arr, len(handles), ctypes.byref(b)))
    return b


def sg_batch_size(b):
    """(number of instances, list of their N_cs)."""
    n = ctypes.c_int32(0)
    _check(lib().sg_batch_size(b, ctypes.byref(n), None))
    ncs = (ctypes.c_int64 * max(n.value, 1))()
    _check(lib().sg_batch_size(b, ctypes.byref(n), ncs))
    return n.value, [int(ncs[i]) for i in range(n.value)]


def sg_batch_propagate(b, psis, dts, nsteps: int, emins=None, emaxs=None, tol: float = 1e-8,
                       precision: int = SG_FP64, check_every: int = 0, use_graph: bool = False,
                       stream=None):
    """psis: list of device complex128 tensors, one per instance in batch order,
    each of that instance's N_cs (propagated in place).  Returns (status, list
    of stats dicts)."""
    n_inst, n_cs = sg_batch_size(b)
    n = len(psis)
    if n != n_inst:
        raise ValueError(f"{n} states for a batch of {n_inst} instances")
    for i, t in enumerate(psis):
        _vec_ptr(t, n_cs[i], f"psi[{i}]")
    ptrs = (_P * n)(*[t.data_ptr() for t in psis])
    dt = np.ascontiguousarray(dts, dtype=np.float64).reshape(n)
    lo = None if emins is None else np.ascontiguousarray(emins, dtype=np.float64).reshape(n)
    hi = None if emaxs is None else np.ascontiguousarray(emaxs, dtype=np.float64).reshape(n)
    null = ctypes.POINTER(ctypes.c_double)()
    st = (PropStats * n)()
    status = lib().sg_batch_propagate(
        b, ptrs, n, _dptr(dt), int(nsteps), _dptr(lo) if lo is not None else null,
        _dptr(hi) if hi is not None else null, float(tol), int(precision), int(check_every),
        1 if use_graph else 0, st, _stream_ptr(stream))
    if status not in (SG_OK, SG_ETOL):
        _check(status)
    return status, [st[i].as_dict() for i in range(n)]


def sg_batch_tune_schedule(b, psis, precision: int = SG_FP64, reps: int = 3, stream=None):
    """Tunes the batch's term schedule on its instances' states; returns
    (chosen block_min_grid, best ms per batched apply)."""
    n_inst, n_cs = sg_batch_size(b)
    if len(psis) != n_inst:
        raise ValueError(f"{len(psis)} states for a batch of {n_inst} instances")
    for i, t in enumerate(psis):
        _vec_ptr(t, n_cs[i], f"psi[{i}]")
    ptrs = (_P * n_inst)(*[t.data_ptr() for t in psis])
    g, ms = ctypes.c_int32(0), ctypes.c_double(0.0)
    _check(lib().sg_batch_tune_schedule(b, ptrs, n_inst, int(precision), int(reps),
                                        ctypes.byref(g), ctypes.byref(ms), _stream_ptr(stream)))
    return g.value, ms.value


def sg_batch_free(b) -> None:
    _check(lib().sg_batch_free(b))


def sg_serve_create(max_slots: int = 64, hbm_budget_bytes: int = 0, precision: int = SG_FP64,
                    check_every: int = 0, tol: float = 0.0, mixed_threshold: int = -1,
                    compile_threads: int = 0) -> ctypes.c_void_p:
    cfg = ServeConfig(int(hbm_budget_bytes), int(max_slots), int(precision), int(check_every),
                      float(tol), int(mixed_threshold), int(compile_threads))
    s = _P()
    _check(lib().sg_serve_create(ctypes.byref(cfg), ctypes.byref(s)))
    return s


def sg_serve_submit(s, D, L, omega, c, k, shift, dt: float, nsteps: int,
                    nb=(1, 2), nq=(2, 2)) -> int:
    desc, keep = _make_desc(D, L, omega, c, k, nb, nq)
    sh = np.ascontiguousarray(shift, dtype=np.float64).reshape(D)
    t = ctypes.c_uint64()
    _check(lib().sg_serve_submit(s, ctypes.byref(desc), _dptr(sh), float(dt), int(nsteps),
                                 ctypes.byref(t)))
    return t.value


def sg_serve_poll(s, ticket: int, n_cs_capacity: int = 0):
    """None while the request runs; else a dict with status, stats, times and
    (when n_cs_capacity suffices) the final state as a numpy complex128 array.
    Raises SgError(SG_ENOTFOUND) for an unknown ticket."""
    buf = np.zeros(max(int(n_cs_capacity), 0), dtype=np.complex128)
    r = Result()
    r.psi_host = buf.ctypes.data if buf.size else None
    r.psi_capacity = buf.size
    status = lib().sg_serve_poll(s, ctypes.c_uint64(ticket), ctypes.byref(r))
    if status == SG_EAGAIN:
        return None
    _check(status)
    out = {"status": r.status, "D": r.D, "L": r.L, "n_cs": r.n_cs, "stats": r.stats.as_dict(),
           "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done}
    out["psi"] = buf[: r.n_cs] if buf.size >= r.n_cs > 0 else None
    return out


def sg_serve_cancel(s, ticket: int) -> None:
    _check(lib().sg_serve_cancel(s, ctypes.c_uint64(ticket)))


def sg_serve_counters(s) -> dict:
    out = (ctypes.c_int64 * 4)()
    _check(lib().sg_serve_counters(s, out))
    return {"queued": out[0], "resident": out[1], "finished": out[2], "ticks": out[3]}


def sg_serve_destroy(s) -> None:
    _check(lib().sg_serve_destroy(s))


class Problem:
    """Owns one problem handle built on the current device."""

    def __init__(self, D, L, omega, c, k=None, nb=(1, 2), nq=(2, 2), host_only=False):
        self.handle = (sg_build_terms_host if host_only else sg_build_terms)(
            D, L, omega, c, k, nb, nq)
        self.info = sg_problem_info(self.handle)
        self.n_cs = self.info["n_cs"]

    @classmethod
    def from_instance(cls, inst, host_only=False):
        return cls(inst.D, inst.L, inst.omega, inst.c, inst.k,
                   (inst.nb_A, inst.nb_B), (inst.nq_A, inst.nq_B), host_only=host_only)

    def apply(self, psi_in, psi_out, precision=SG_FP64, stream=None):
        sg_apply_H(self.handle, psi_in, psi_out, precision, stream, self.n_cs)

    def close(self):
        if self.handle is not None:
            sg_free(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Two-state (vibronic) problems
# ---------------------------------------------------------------------------

def sg_vibronic_build(D, L, omega, E, kappa, lam, c2=None):
    omega = np.ascontiguousarray(omega, dtype=np.float64).reshape(D)
    E = np.ascontiguousarray(E, dtype=np.float64).reshape(2)
    kappa = np.ascontiguousarray(kappa, dtype=np.float64).reshape(2 * D)
    lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(D)
    c2a = None if c2 is None else np.ascontiguousarray(c2, dtype=np.float64).reshape(2 * D * D)
    d = VibronicDesc(int(D), int(L), _dptr(omega), _dptr(E), _dptr(kappa), _dptr(lam),
                     _dptr(c2a) if c2a is not None else ctypes.POINTER(ctypes.c_double)())
    h = _P()
    _check(lib().sg_vibronic_build(ctypes.byref(d), ctypes.byref(h)))
    return h


def sg_vibronic_free(v) -> None:
    _check(lib().sg_vibronic_free(v))


def sg_vibronic_problem(v):
    """The one-state structure handle (owned by v)."""
    h = _P()
    _check(lib().sg_vibronic_problem(v, ctypes.byref(h)))
    return h


def sg_vibronic_figures(v):
    f, b = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().sg_vibronic_figures(v, ctypes.byref(f), ctypes.byref(b)))
    return f.value, b.value


def sg_vibronic_init(v, n_cs, shift, state, psi, stream=None) -> None:
    shift = np.ascontiguousarray(shift, dtype=np.float64)
    _check(lib().sg_vibronic_init(v, _dptr(shift), int(state), _vec_ptr(psi, 2 * n_cs, "psi"),
                                  _stream_ptr(stream)))


def sg_vibronic_apply(v, n_cs, psi_in, psi_out, stream=None) -> None:
    _check(lib().sg_vibronic_apply(v, _vec_ptr(psi_in, 2 * n_cs, "psi_in"),
                                   _vec_ptr(psi_out, 2 * n_cs, "psi_out"), _stream_ptr(stream)))


def sg_vibronic_bounds(v, iters: int = 40, stream=None):
    lo, hi = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().sg_vibronic_bounds(v, int(iters), ctypes.byref(lo), ctypes.byref(hi),
                                    _stream_ptr(stream)))
    return lo.value, hi.value


def sg_vibronic_propagate(v, n_cs, psi, dt: float, nsteps: int, emin=math.nan, emax=math.nan,
                          tol: float = 0.0, check_every: int = 0, stream=None):
    """Returns (status, stats dict, population of state 1 at the checks)."""
    st = PropStats()
    ntr = max((nsteps // check_every + 2) if check_every > 0 else 2, 2)
    pop = np.zeros(ntr)
    status = lib().sg_vibronic_propagate(v, _vec_ptr(psi, 2 * n_cs, "psi"), float(dt),
                                         int(nsteps), float(emin), float(emax), float(tol),
                                         int(check_every), ctypes.byref(st), _dptr(pop),
                                         _stream_ptr(stream))
    if status not in (SG_OK, SG_ETOL):
        _check(status)
    d = st.as_dict()
    done = d["steps_done"]
    n = (1 + (done // check_every if check_every > 0 else 0)) if done < nsteps else \
        ((0 if nsteps == 0 else 1 + ((nsteps - 1) // check_every if check_every > 0 else 0)) + 1)
    return status, d, pop[:min(n, ntr)]


class Vibronic:
    """Owns one two-state problem handle built on the current device."""

    def __init__(self, D, L, omega, E, kappa, lam, c2=None):
        self.handle = sg_vibronic_build(D, L, omega, E, kappa, lam, c2)
        self.problem = sg_vibronic_problem(self.handle)
        self.info = sg_problem_info(self.problem)
        self.n_cs = self.info["n_cs"]

    @classmethod
    def from_instance(cls, inst):
        return cls(inst.D, inst.L, inst.omega, inst.E, inst.kappa, inst.lam, inst.c2)

    def apply(self, psi_in, psi_out, stream=None):
        sg_vibronic_apply(self.handle, self.n_cs, psi_in, psi_out, stream)

    def close(self):
        if self.handle is not None:
            sg_vibronic_free(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
