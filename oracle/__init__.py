"""FP64 CPU oracle for imaginary-time FDTD relaxation (arXiv:0904.0939).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  The product path never imports this
package.  It wraps ``fdtd_oracle.c`` (plain C, double precision) with ctypes;
numpy arrays are laid out as psi[x, y, z] with z fastest.  Nothing here is
shared with the GPU library.

Parity pins live in ``tests/test_oracle_*.py``: closed-form box modes, the
dense operator (I - dt D^-1 H) on small lattices, the generalised eigenproblem
H psi = mu D psi, separable harmonic-oscillator eigenvalues, the paper's own
printed energies, brute-force finite differences for the gradient.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FDTD_ORACLE_LIB: load another build of the same source (the sanitizer build)
_LIB_PATH = os.environ.get("FDTD_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

POT_CONST, POT_HO, POT_COULOMB, POT_COULOMB_REG, POT_CORNELL, POT_WELLS, POT_DODECA = range(7)
INIT_UNIFORM, INIT_GAUSS = 0, 1
PAR_FREE, PAR_S, PAR_A = 0, 1, 2

_dp = C.POINTER(C.c_double)


def parity_word(x: int = 0, y: int = 0, z: int = 0) -> int:
    """2 bits per axis: 0 free, 1 symmetric (S_i), 2 antisymmetric (A_i)."""
    return (x & 3) | ((y & 3) << 2) | ((z & 3) << 4)


def lib():
    global _lib
    if _lib is None:
        if not os.environ.get("FDTD_ORACLE_LIB") and (not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(os.path.join(_HERE, "fdtd_oracle.c"))
        )):
            from . import build as _b

            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.orc_potential.argtypes = [C.c_int, _dp, C.c_int, C.c_int, C.c_double, _dp]
        L.orc_potential.restype = C.c_int
        L.orc_initial.argtypes = [C.c_uint64, C.c_uint32, C.c_int, C.c_uint32, C.c_int, _dp]
        L.orc_initial.restype = C.c_int
        L.orc_reimpose.argtypes = [C.c_int, C.c_uint32, _dp]
        L.orc_reimpose.restype = C.c_int
        L.orc_step.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _dp, _dp, _dp]
        L.orc_step.restype = None
        L.orc_hpsi.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp, _dp]
        L.orc_hpsi.restype = None
        L.orc_observables.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp, C.c_double, _dp]
        L.orc_observables.restype = None
        L.orc_evolve.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _dp, _dp,
                                 C.c_int64, C.c_int, C.c_int, C.c_double, C.c_double,
                                 C.POINTER(C.c_int), _dp]
        L.orc_evolve.restype = C.c_int64
        L.orc_evolve_deflated.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _dp,
                                          _dp, C.c_int64, C.c_int, C.c_int, C.c_double,
                                          C.c_double, C.POINTER(C.c_int), _dp, _dp, C.c_int,
                                          C.c_int]
        L.orc_evolve_deflated.restype = C.c_int64
        L.orc_project_out.argtypes = [C.c_int64, _dp, C.c_int, _dp, _dp]
        L.orc_project_out.restype = None
        L.orc_upsample.argtypes = [C.c_int, C.c_double, _dp, C.c_int, _dp]
        L.orc_upsample.restype = None
        L.orc_energy_grad_v.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _dp, _dp,
                                        C.c_int, _dp]
        L.orc_energy_grad_v.restype = C.c_double
        L.orc_wells_dv.argtypes = [_dp, C.c_int, C.c_int, C.c_double, C.c_int, _dp]
        L.orc_wells_dv.restype = C.c_int
        L.orc_potential_dv.argtypes = [C.c_int, _dp, C.c_int, C.c_int, C.c_double, C.c_int, _dp]
        L.orc_potential_dv.restype = C.c_int
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_set_num_threads.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _field(N: int) -> np.ndarray:
    return np.zeros((N, N, N), dtype=np.float64)


def coords(N: int, L: float) -> np.ndarray:
    """Site coordinates x_i = (2 i - (N - 1)) a / 2 of one axis."""
    a = L / N
    return (2.0 * np.arange(N) - (N - 1)) * (0.5 * a)


def potential(kind: int, params, N: int, L: float) -> np.ndarray:
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1))
    V = _field(N)
    rc = lib().orc_potential(int(kind), _ptr(p), int(p.size), int(N), float(L), _ptr(V))
    if rc != 0:
        raise ValueError("oracle: bad potential parameters")
    return V


def initial(N: int, seed: int, kind: int = INIT_UNIFORM, parity: int = 0, member: int = 0):
    psi = _field(N)
    rc = lib().orc_initial(int(seed) & (2**64 - 1), int(member), int(kind), int(parity), int(N),
                           _ptr(psi))
    if rc != 0:
        raise ValueError("oracle: bad initial-state arguments")
    return psi


def reimpose(psi: np.ndarray, parity: int) -> np.ndarray:
    """The Sec. IV symmetry operators applied to a copy of psi (orc_reimpose)."""
    out = np.ascontiguousarray(psi, dtype=np.float64).copy()
    if lib().orc_reimpose(out.shape[0], int(parity), _ptr(out)) != 0:
        raise ValueError("oracle: bad parity word")
    return out


def step(psi: np.ndarray, V: np.ndarray, L: float, dt: float, mass: float = 1.0) -> np.ndarray:
    N = psi.shape[0]
    out = _field(N)
    lib().orc_step(N, float(L), float(mass), float(dt), _ptr(V), _ptr(psi), _ptr(out))
    return out


def hpsi(psi: np.ndarray, V: np.ndarray, L: float, mass: float = 1.0) -> np.ndarray:
    N = psi.shape[0]
    out = _field(N)
    lib().orc_hpsi(N, float(L), float(mass), _ptr(V), _ptr(psi), _ptr(out))
    return out


def observables(psi: np.ndarray, V: np.ndarray, L: float, mass: float = 1.0, v_inf: float = 0.0):
    """dict(norm2, energy, kinetic, potential, r_rms, binding)."""
    out = np.zeros(6)
    lib().orc_observables(psi.shape[0], float(L), float(mass), _ptr(V), _ptr(psi), float(v_inf),
                          _ptr(out))
    keys = ("norm2", "energy", "kinetic", "potential", "r_rms", "binding")
    return dict(zip(keys, (float(v) for v in out)))


def evolve(psi: np.ndarray, V: np.ndarray, L: float, dt: float, steps: int, mass: float = 1.0,
           renorm_every: int = 1, check_every: int = 0, rel_tol: float = 0.0,
           v_inf: float = 0.0, deflate=None, project_every: int = 0):
    """Evolve psi in place.  Returns (steps_done, converged, checked_energies).
    deflate: optional list of states projected out after every
    project_every-th step (orc_evolve_deflated)."""
    N = psi.shape[0]
    conv = C.c_int(0)
    nchk = steps // check_every if check_every > 0 else 0
    hist = np.zeros(max(nchk, 1))
    if deflate:
        st = np.ascontiguousarray(np.stack([np.asarray(d, dtype=np.float64) for d in deflate]))
        done = lib().orc_evolve_deflated(N, float(L), float(mass), float(dt), _ptr(V), _ptr(psi),
                                         int(steps), int(renorm_every), int(check_every),
                                         float(rel_tol), float(v_inf), C.byref(conv), _ptr(hist),
                                         st.ctypes.data_as(_dp), len(deflate), int(project_every))
    else:
        done = lib().orc_evolve(N, float(L), float(mass), float(dt), _ptr(V), _ptr(psi),
                                int(steps), int(renorm_every), int(check_every), float(rel_tol),
                                float(v_inf), C.byref(conv), _ptr(hist))
    if done < 0:
        raise MemoryError("oracle: allocation failed")
    used = done // check_every if check_every > 0 else 0
    return int(done), bool(conv.value), hist[:used].copy()


def project_out(psi: np.ndarray, states) -> np.ndarray:
    """psi minus its components along `states`, removed one after the other
    (orc_project_out, Sec. III).  Returns (new psi, coefficients)."""
    out = np.ascontiguousarray(psi, dtype=np.float64).copy()
    st = np.ascontiguousarray(np.stack([np.asarray(d, dtype=np.float64) for d in states]))
    coef = np.zeros(len(states))
    lib().orc_project_out(out.size, st.ctypes.data_as(_dp), len(states), _ptr(out), _ptr(coef))
    return out, coef


def upsample(psi_c: np.ndarray, Nf: int, L: float) -> np.ndarray:
    out = _field(Nf)
    lib().orc_upsample(psi_c.shape[0], float(L), _ptr(np.ascontiguousarray(psi_c)), int(Nf),
                       _ptr(out))
    return out


def energy_grad_v(psi0: np.ndarray, V: np.ndarray, L: float, dt: float, steps: int,
                  mass: float = 1.0):
    """(E_T, dE_T/dV field) for psi_T = T renormalised steps from psi0."""
    N = psi0.shape[0]
    G = _field(N)
    E = lib().orc_energy_grad_v(N, float(L), float(mass), float(dt), _ptr(V),
                                _ptr(np.ascontiguousarray(psi0)), int(steps), _ptr(G))
    if not np.isfinite(E):
        raise MemoryError("oracle: allocation failed")
    return float(E), G


def wells_dv(params, N: int, L: float, j: int) -> np.ndarray:
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1))
    out = _field(N)
    if lib().orc_wells_dv(_ptr(p), int(p.size), int(N), float(L), int(j), _ptr(out)) != 0:
        raise ValueError("oracle: bad well-parameter index")
    return out


def potential_dv(kind: int, params, N: int, L: float, j: int) -> np.ndarray:
    """dV/dparams[j] at every site for an analytic potential kind."""
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1))
    out = _field(N)
    if lib().orc_potential_dv(int(kind), _ptr(p), int(p.size), int(N), float(L), int(j),
                              _ptr(out)) != 0:
        raise ValueError("oracle: the potential kind has no parameter j")
    return out


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of later sweeps (timing only; results do not depend on it)."""
    lib().orc_set_num_threads(int(n))


def normalized(psi: np.ndarray, L: float) -> np.ndarray:
    a = L / psi.shape[0]
    return psi / np.sqrt(np.sum(psi * psi) * a ** 3)
