"""ctypes binding of libfdtd (include/fdtd.h), the gfx950 imaginary-time FDTD
library (Strickland & Yager-Elorriaga, arXiv:0904.0939).

Every function of the C ABI is exposed under its own name with the same
arguments; failures raise FdtdError carrying the status and the library's
message.  This module only marshals arguments: all arithmetic runs in the HIP
kernels.  torch is imported first so that the library binds to the same HIP
runtime as torch (one runtime per process); torch supplies device memory
(workspaces, fields) and streams.  There is no CPU fallback: without the
built library or a GPU the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import torch  # noqa: F401  (must precede loading libfdtd)

_HERE = os.path.dirname(os.path.abspath(__file__))
# FDTD_LIB_PATH: load another build of the same sources (the sanitizer build)
LIB_PATH = os.environ.get("FDTD_LIB_PATH") or os.path.join(_HERE, "libfdtd.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "fdtd.h")

OK, EINVAL, ENOMEM, EHIP, EUNSTABLE, ENOTREADY, ENONFINITE = range(7)
F64, F32, BF16 = 0, 1, 2
POT_CONST, POT_HO, POT_COULOMB, POT_COULOMB_REG, POT_CORNELL, POT_WELLS, POT_DODECA = range(7)
INIT_UNIFORM, INIT_GAUSS, INIT_USER = 0, 1, 2
EVOLVE_ASYNC = 1


def parity(px: int = 0, py: int = 0, pz: int = 0) -> int:
    """Parity word: 2 bits per axis, 0 free, 1 S_i, 2 A_i (Sec. IV)."""
    return (px & 3) | ((py & 3) << 2) | ((pz & 3) << 4)


class fdtd_config(C.Structure):
    _fields_ = [("n", C.c_int32), ("psi_dtype", C.c_int32), ("box_len", C.c_double),
                ("mass", C.c_double), ("dt", C.c_double), ("v_inf", C.c_double),
                ("device", C.c_int32), ("history", C.c_int32), ("stream", C.c_void_p)]


class fdtd_obs(C.Structure):
    _fields_ = [("norm2", C.c_double), ("energy", C.c_double), ("kinetic", C.c_double),
                ("potential", C.c_double), ("r_rms", C.c_double), ("binding", C.c_double),
                ("tau", C.c_double), ("step", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class fdtd_evolve_opts(C.Structure):
    _fields_ = [("max_steps", C.c_int64), ("renorm_every", C.c_int32),
                ("check_every", C.c_int32), ("reimpose_parity_every", C.c_int32),
                ("use_graph", C.c_int32), ("rel_tol", C.c_double),
                ("project_every", C.c_int32), ("flags", C.c_int32)]


class fdtd_tuning(C.Structure):
    _fields_ = [("vz", C.c_int32), ("ry", C.c_int32), ("xchunk", C.c_int32),
                ("grid", C.c_int32), ("xcd_remap", C.c_int32), ("depth", C.c_int32),
                ("variant", C.c_int32), ("persist", C.c_int32), ("vfuse", C.c_int32),
                ("tblock", C.c_int32), ("tile", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class fdtd_counters(C.Structure):
    _fields_ = [("graph_captures", C.c_int64), ("graph_replays", C.c_int64),
                ("allocations", C.c_int64), ("reserved", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class FdtdError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func}: status {status}: {msg}")
        self.status = status


_P = C.c_void_p
_SIGS = {
    "fdtd_create": [C.POINTER(fdtd_config), C.POINTER(_P)],
    "fdtd_create_batch": [C.POINTER(fdtd_config), C.c_int32, C.POINTER(_P)],
    "fdtd_workspace_size": [_P, C.POINTER(C.c_size_t)],
    "fdtd_bind_workspace": [_P, _P, C.c_size_t],
    "fdtd_destroy": [_P],
    "fdtd_set_potential": [_P, C.c_int32, _P, C.c_int32, C.c_int32],
    "fdtd_set_potential_analytic": [_P, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_int32],
    "fdtd_set_initial": [_P, C.c_int32, C.c_int32, C.c_uint64, C.c_uint32, _P, C.c_int32,
                         C.c_int32],
    "fdtd_set_projection_states": [_P, C.c_int32, _P, C.c_int32, C.c_int32, C.c_int32],
    "fdtd_project": [_P, C.c_int32, C.POINTER(C.c_double)],
    "fdtd_evolve": [_P, C.POINTER(fdtd_evolve_opts), C.POINTER(C.c_int64), C.POINTER(C.c_int32)],
    "fdtd_observables": [_P, C.POINTER(fdtd_obs)],
    "fdtd_history": [_P, C.c_int32, C.POINTER(fdtd_obs), C.c_int64, C.POINTER(C.c_int64)],
    "fdtd_get_psi": [_P, C.c_int32, _P, C.c_int32, C.c_int32],
    "fdtd_get_state": [_P, C.c_int32, _P, C.c_int32, C.POINTER(C.c_int64)],
    "fdtd_checkpoint_size": [_P, C.c_int32, C.POINTER(C.c_size_t)],
    "fdtd_checkpoint_save": [_P, C.c_int32, _P, C.c_int32],
    "fdtd_checkpoint_load": [_P, C.c_int32, _P, C.c_int32],
    "fdtd_upsample": [_P, C.c_int32, _P, C.c_int32],
    "fdtd_upsample_noalloc": [_P, C.c_int32, _P, C.c_int32],
    "fdtd_energy_grad": [_P, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_int32,
                         C.POINTER(C.c_int32), C.c_int32, _P, C.POINTER(C.c_double),
                         C.POINTER(C.c_double)],
    "fdtd_grad_workspace_size": [_P, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)],
    "fdtd_bind_grad_workspace": [_P, _P, C.c_size_t],
    "fdtd_get_tuning": [_P, C.POINTER(fdtd_tuning)],
    "fdtd_set_tuning": [_P, C.POINTER(fdtd_tuning)],
    "fdtd_autotune": [_P, C.c_int32, C.POINTER(fdtd_tuning), C.POINTER(C.c_double)],
    "fdtd_tune_cache_save": [C.c_char_p],
    "fdtd_tune_cache_load": [C.c_char_p],
    "fdtd_synchronize": [_P],
    "fdtd_info": [_P, C.POINTER(C.c_int32), C.POINTER(_P)],
    "fdtd_get_counters": [_P, C.POINTER(fdtd_counters)],
}

_lib = None


def header_functions():
    """Names of the functions include/fdtd.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:fdtd_status|const char\*)\s+(fdtd_\w+)\s*\(", text, re.M)))


def lib():
    """Load libfdtd.so (built in-tree by paper_0904_0939_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FdtdError(EHIP, "load", f"{LIB_PATH} is missing: run paper_0904_0939_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.fdtd_status_string.argtypes = [C.c_int]
        L.fdtd_status_string.restype = C.c_char_p
        L.fdtd_last_error.argtypes = []
        L.fdtd_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _call(name, *args):
    st = getattr(lib(), name)(*args)
    if st != OK:
        raise FdtdError(st, name, lib().fdtd_last_error().decode())
    return st


# ------------------------------------------------ C ABI, one wrapper each --
def fdtd_create(cfg: fdtd_config) -> int:
    h = _P()
    _call("fdtd_create", C.byref(cfg), C.byref(h))
    return h.value


def fdtd_create_batch(cfgs) -> int:
    arr = (fdtd_config * len(cfgs))(*cfgs)
    h = _P()
    _call("fdtd_create_batch", arr, len(cfgs), C.byref(h))
    return h.value


def fdtd_workspace_size(h) -> int:
    n = C.c_size_t()
    _call("fdtd_workspace_size", h, C.byref(n))
    return n.value


def fdtd_bind_workspace(h, ptr: int, nbytes: int):
    _call("fdtd_bind_workspace", h, ptr, nbytes)


def fdtd_destroy(h):
    _call("fdtd_destroy", h)


def fdtd_set_potential(h, member: int, ptr: int, dtype: int, on_device: int):
    _call("fdtd_set_potential", h, member, ptr, dtype, on_device)


def fdtd_set_potential_analytic(h, member: int, kind: int, params):
    p = (C.c_double * max(len(params), 1))(*[float(v) for v in params])
    _call("fdtd_set_potential_analytic", h, member, kind, p, len(params))


def fdtd_set_initial(h, member: int, kind: int, seed: int, parity_word: int = 0, user_ptr=None,
                     dtype: int = F64, on_device: int = 0):
    _call("fdtd_set_initial", h, member, kind, seed & (2**64 - 1), parity_word, user_ptr, dtype,
          on_device)


def fdtd_set_projection_states(h, member: int, states_ptr, n: int, dtype: int, on_device: int):
    _call("fdtd_set_projection_states", h, member, states_ptr, n, dtype, on_device)


def fdtd_project(h, member: int, n: int):
    coef = (C.c_double * max(n, 1))()
    _call("fdtd_project", h, member, coef)
    return [coef[i] for i in range(n)]


def fdtd_evolve(h, opts: fdtd_evolve_opts):
    done, conv = C.c_int64(), C.c_int32()
    _call("fdtd_evolve", h, C.byref(opts), C.byref(done), C.byref(conv))
    return done.value, bool(conv.value)


def fdtd_observables(h, count: int = 1):
    out = (fdtd_obs * count)()
    _call("fdtd_observables", h, out)
    return [o.as_dict() for o in out]


def fdtd_history(h, member: int, max_records: int):
    out = (fdtd_obs * max(max_records, 1))()
    n = C.c_int64()
    _call("fdtd_history", h, member, out, max_records, C.byref(n))
    return [out[i].as_dict() for i in range(n.value)]


def fdtd_get_psi(h, member: int, ptr: int, dtype: int, on_device: int):
    _call("fdtd_get_psi", h, member, ptr, dtype, on_device)


def fdtd_get_state(h, member: int, ptr: int, on_device: int) -> int:
    st = C.c_int64()
    _call("fdtd_get_state", h, member, ptr, on_device, C.byref(st))
    return st.value


def fdtd_checkpoint_size(h, member: int) -> int:
    n = C.c_size_t()
    _call("fdtd_checkpoint_size", h, member, C.byref(n))
    return n.value


def fdtd_checkpoint_save(h, member: int, ptr: int, on_device: int):
    _call("fdtd_checkpoint_save", h, member, ptr, on_device)


def fdtd_checkpoint_load(h, member: int, ptr: int, on_device: int):
    _call("fdtd_checkpoint_load", h, member, ptr, on_device)


def fdtd_upsample(coarse, cm: int, fine, fm: int):
    _call("fdtd_upsample", coarse, cm, fine, fm)


def fdtd_upsample_noalloc(coarse, cm: int, fine, fm: int):
    _call("fdtd_upsample_noalloc", coarse, cm, fine, fm)


def fdtd_energy_grad(h, steps: int, checkpoint_every: int, theta=None, wrt=None, dE_dV_ptr=None):
    th = (C.c_double * len(theta))(*theta) if theta is not None else None
    nt = len(theta) if theta is not None else 0
    w = (C.c_int32 * len(wrt))(*wrt) if wrt else None
    nw = len(wrt) if wrt else 0
    g = (C.c_double * max(nw, 1))()
    e = C.c_double()
    _call("fdtd_energy_grad", h, steps, checkpoint_every, th, nt, w, nw, dE_dV_ptr, g, C.byref(e))
    return e.value, [g[i] for i in range(nw)]


def fdtd_grad_workspace_size(h, steps: int, checkpoint_every: int) -> int:
    n = C.c_size_t()
    _call("fdtd_grad_workspace_size", h, steps, checkpoint_every, C.byref(n))
    return n.value


def fdtd_bind_grad_workspace(h, ptr, nbytes: int):
    _call("fdtd_bind_grad_workspace", h, ptr, nbytes)


def fdtd_get_tuning(h) -> fdtd_tuning:
    t = fdtd_tuning()
    _call("fdtd_get_tuning", h, C.byref(t))
    return t


def fdtd_set_tuning(h, t: fdtd_tuning):
    _call("fdtd_set_tuning", h, C.byref(t))


def fdtd_autotune(h, steps_per_trial: int = 10):
    t = fdtd_tuning()
    ms = C.c_double()
    _call("fdtd_autotune", h, steps_per_trial, C.byref(t), C.byref(ms))
    return t, ms.value


def fdtd_tune_cache_save(path: str):
    _call("fdtd_tune_cache_save", os.fsencode(path))


def fdtd_tune_cache_load(path: str):
    _call("fdtd_tune_cache_load", os.fsencode(path))


def fdtd_synchronize(h):
    _call("fdtd_synchronize", h)


def fdtd_get_counters(h) -> dict:
    c = fdtd_counters()
    _call("fdtd_get_counters", h, C.byref(c))
    return c.as_dict()


def fdtd_info(h):
    n, s = C.c_int32(), _P()
    _call("fdtd_info", h, C.byref(n), C.byref(s))
    return n.value, s.value


def fdtd_status_string(s: int) -> str:
    return lib().fdtd_status_string(s).decode()


def fdtd_last_error() -> str:
    return lib().fdtd_last_error().decode()
