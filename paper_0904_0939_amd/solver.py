"""Convenience wrappers over the C ABI: a Solver for one lattice, a Batch of
lattices advancing together, the multi-resolution chain of Sec. VI and an
autograd Function for energy gradients.  They own handles, bind a torch
tensor as the device workspace, pass torch's current stream, and move arrays
between numpy/torch and the library.  No arithmetic of the method happens
here.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import fdtd as F

_DT = {"f64": F.F64, "f32": F.F32, "bf16": F.BF16, F.F64: F.F64, F.F32: F.F32, F.BF16: F.BF16}
_NP = {F.F64: np.float64, F.F32: np.float32}


def dtype_code(d) -> int:
    return _DT[d]


def _stream(device: int) -> int:
    if not torch.cuda.is_available():
        raise F.FdtdError(F.EHIP, "stream", "no GPU visible to torch; the library has no CPU path")
    return torch.cuda.current_stream(device).cuda_stream


class _Handle:
    def __init__(self, cfgs: List[F.fdtd_config], bind_torch_workspace: bool = True):
        self.cfgs = cfgs
        self.count = len(cfgs)
        self.device = cfgs[0].device
        self.h = F.fdtd_create(cfgs[0]) if self.count == 1 else F.fdtd_create_batch(cfgs)
        self._ws = None
        if bind_torch_workspace:
            nbytes = F.fdtd_workspace_size(self.h)
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.device}")
            F.fdtd_bind_workspace(self.h, self._ws.data_ptr(), nbytes)

    def close(self):
        if self.h:
            F.fdtd_destroy(self.h)
            self.h = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def evolve(self, steps: int, renorm_every: int = 1, check_every: int = 0, rel_tol: float = 0.0,
               use_graph: bool = True, reimpose_parity_every: int = 0, project_every: int = 0,
               async_launch: bool = False):
        o = F.fdtd_evolve_opts(int(steps), int(renorm_every), int(check_every),
                               int(reimpose_parity_every), 1 if use_graph else 0, float(rel_tol),
                               int(project_every), F.EVOLVE_ASYNC if async_launch else 0)
        return F.fdtd_evolve(self.h, o)

    def counters(self) -> Dict:
        return F.fdtd_get_counters(self.h)

    def set_projection_states(self, states, member: int = 0):
        """Keep `states` (a sequence of N^3 arrays or tensors, or one stacked
        array / tensor; empty: drop them) for projection (Sec. III)."""
        if isinstance(states, (list, tuple)):
            if len(states) == 0:
                F.fdtd_set_projection_states(self.h, member, None, 0, F.F64, 0)
                return
            if isinstance(states[0], torch.Tensor):
                states = torch.stack([t.to(states[0].dtype) for t in states])
            else:
                states = np.stack([np.asarray(t, dtype=np.float64) for t in states])
        n = states.shape[0]
        if isinstance(states, torch.Tensor):
            t = states.contiguous()
            code = {torch.float64: F.F64, torch.float32: F.F32, torch.bfloat16: F.BF16}[t.dtype]
            F.fdtd_set_projection_states(self.h, member, t.data_ptr(), n, code, 1 if t.is_cuda else 0)
            if t.is_cuda:
                torch.cuda.current_stream(self.device).synchronize()
        else:
            a = np.ascontiguousarray(states, dtype=np.float64)
            F.fdtd_set_projection_states(self.h, member, a.ctypes.data, n, F.F64, 0)
        self._nproj = getattr(self, "_nproj", {})
        self._nproj[member] = n

    def project(self, member: int = 0):
        """Project the kept states out of the current state; returns the
        coefficients <phi_k|psi>/<phi_k|phi_k>."""
        return F.fdtd_project(self.h, member, getattr(self, "_nproj", {}).get(member, 0))

    def observables(self) -> List[Dict]:
        return F.fdtd_observables(self.h, self.count)

    def tuning(self) -> Dict:
        return F.fdtd_get_tuning(self.h).as_dict()

    def set_tuning(self, vz: int, ry: int, xchunk: int, grid: int = 0, xcd_remap: int = 1,
                   depth: int = 1, variant: int = 0, persist: int = 0, vfuse: int = 1,
                   tblock: int = 0, tile: int = 0):
        F.fdtd_set_tuning(self.h, F.fdtd_tuning(vz, ry, xchunk, grid, xcd_remap, depth, variant,
                                                persist, vfuse, tblock, tile))

    def autotune(self, steps_per_trial: int = 10):
        t, ms = F.fdtd_autotune(self.h, steps_per_trial)
        return t.as_dict(), ms

    def synchronize(self):
        F.fdtd_synchronize(self.h)

    def history(self, member: int = 0, max_records: int = 4096) -> List[Dict]:
        return F.fdtd_history(self.h, member, max_records)

    def psi(self, member: int = 0, dtype=np.float64) -> np.ndarray:
        N = self.cfgs[member].n
        code = F.F64 if np.dtype(dtype) == np.float64 else F.F32
        out = np.empty((N, N, N), dtype=_NP[code])
        F.fdtd_get_psi(self.h, member, out.ctypes.data, code, 0)
        return out

    def state(self, member: int = 0) -> np.ndarray:
        """The stored state as held on the device (storage dtype, bf16 as uint16)."""
        N = self.cfgs[member].n
        code = self.cfgs[member].psi_dtype
        out = np.empty((N, N, N), dtype={F.F64: np.float64, F.F32: np.float32, F.BF16: np.uint16}[code])
        F.fdtd_get_state(self.h, member, out.ctypes.data, 0)
        return out

    def checkpoint(self, member: int = 0) -> np.ndarray:
        """A checkpoint record of the member (header + stored state) in host memory."""
        buf = np.empty(F.fdtd_checkpoint_size(self.h, member), dtype=np.uint8)
        F.fdtd_checkpoint_save(self.h, member, buf.ctypes.data, 0)
        return buf

    def restore(self, record: np.ndarray, member: int = 0):
        """Continue from a record written by checkpoint() (same N, dtype, L, dt)."""
        a = np.ascontiguousarray(record, dtype=np.uint8)
        F.fdtd_checkpoint_load(self.h, member, a.ctypes.data, 0)

    def psi_tensor(self, member: int = 0, dtype=torch.float32) -> torch.Tensor:
        N = self.cfgs[member].n
        code = {torch.float64: F.F64, torch.float32: F.F32, torch.bfloat16: F.BF16}[dtype]
        out = torch.empty((N, N, N), dtype=dtype, device=f"cuda:{self.device}")
        F.fdtd_get_psi(self.h, member, out.data_ptr(), code, 1)
        return out

    def set_potential(self, kind: int, params: Sequence[float], member: int = -1):
        F.fdtd_set_potential_analytic(self.h, member, kind, list(params))

    def set_potential_array(self, V, member: int = 0):
        if isinstance(V, torch.Tensor):
            t = V.contiguous()
            code = F.F64 if t.dtype == torch.float64 else F.F32
            if t.dtype not in (torch.float64, torch.float32):
                t = t.float()
            if t.is_cuda:
                F.fdtd_set_potential(self.h, member, t.data_ptr(), code, 1)
                torch.cuda.current_stream(self.device).synchronize()
            else:
                F.fdtd_set_potential(self.h, member, t.data_ptr(), code, 0)
        else:
            a = np.ascontiguousarray(V, dtype=np.float64)
            F.fdtd_set_potential(self.h, member, a.ctypes.data, F.F64, 0)

    def set_initial(self, seed: int, kind: int = F.INIT_UNIFORM, parity: int = 0, member: int = -1):
        F.fdtd_set_initial(self.h, member, kind, seed, parity)

    def set_initial_array(self, psi, member: int = 0):
        if isinstance(psi, torch.Tensor):
            t = psi.contiguous()
            code = {torch.float64: F.F64, torch.float32: F.F32, torch.bfloat16: F.BF16}[t.dtype]
            F.fdtd_set_initial(self.h, member, F.INIT_USER, 0, 0, t.data_ptr(), code,
                               1 if t.is_cuda else 0)
        else:
            a = np.ascontiguousarray(psi, dtype=np.float64)
            F.fdtd_set_initial(self.h, member, F.INIT_USER, 0, 0, a.ctypes.data, F.F64, 0)


def make_config(N: int, L: float, dt: Optional[float] = None, mass: float = 1.0, dtype="f32",
                v_inf: float = 0.0, device: int = 0, history: int = 0, stream=None,
                dt_over_a2: float = 0.125) -> F.fdtd_config:
    a = L / N
    if dt is None:
        dt = dt_over_a2 * a * a
    s = _stream(device) if stream is None else stream
    return F.fdtd_config(int(N), dtype_code(dtype), float(L), float(mass), float(dt), float(v_inf),
                         int(device), int(history), s)


class Solver(_Handle):
    """One N^3 lattice."""

    def __init__(self, N: int, L: float, dt: Optional[float] = None, mass: float = 1.0,
                 dtype="f32", v_inf: float = 0.0, device: int = 0, history: int = 0,
                 dt_over_a2: float = 0.125, bind_torch_workspace: bool = True):
        super().__init__([make_config(N, L, dt, mass, dtype, v_inf, device, history,
                                      dt_over_a2=dt_over_a2)], bind_torch_workspace)
        self.N, self.L = N, L

    def energy_grad(self, steps: int, checkpoint_every: int, theta=None, wrt=None,
                    want_field: bool = False):
        """(E_T, dE/dtheta list, dE/dV device tensor or None).  The driver's
        checkpoints live in a torch tensor bound to the handle, kept between
        calls and grown when a call needs more."""
        need = F.fdtd_grad_workspace_size(self.h, steps, checkpoint_every)
        gws = getattr(self, "_gws", None)
        if gws is None or gws.numel() < need:
            self._gws = None
            F.fdtd_bind_grad_workspace(self.h, None, 0)
            self._gws = torch.empty(need, dtype=torch.uint8, device=f"cuda:{self.device}")
            F.fdtd_bind_grad_workspace(self.h, self._gws.data_ptr(), need)
        G = None
        ptr = None
        if want_field:
            G = torch.empty((self.N,) * 3, dtype=torch.float64, device=f"cuda:{self.device}")
            ptr = G.data_ptr()
        E, g = F.fdtd_energy_grad(self.h, steps, checkpoint_every, theta, wrt, ptr)
        return E, g, G


class Batch(_Handle):
    """Lattices of uneven size advancing together, one launch per step."""

    def __init__(self, lattices: Sequence, dtype="f32", device: int = 0, history: int = 0):
        cfgs = [make_config(l.N, l.L, l.dt, l.mass, dtype, l.v_inf, device, history)
                for l in lattices]
        super().__init__(cfgs)
        self.lattices = list(lattices)


def multires(levels: Sequence[int], L: float, kind: int, params: Sequence[float],
             dtypes: Sequence[str], seed: int = 0, rel_tol: Sequence[float] = (1e-7,),
             max_steps: Sequence[int] = (200000,), check_every: int = 100,
             dt_over_a2: float = 0.125, mass: float = 1.0, parity: int = 0,
             use_graph: bool = True, v_inf: float = 0.0, project: Optional[Dict] = None,
             project_every: int = 10, keep: bool = False, two_step: bool = False):
    """Multi-resolution chain (Sec. VI): relax from noise on levels[0], then
    reseed each finer level by trilinear interpolation of the previous one.
    project: optional {N: [states]} projected out every project_every steps
    on level N (excited states, Sec. III).  keep: also return each level's
    final state (FP32 device tensor) in a dict.  two_step: every level whose
    side the dtype's vector width divides runs two steps per pass over HBM
    (prefetch depth 5 for F32 states, 3 otherwise; 16 x 128 tiles for F32
    levels of side 512 or more that read the V table).  Returns (final Solver,
    per-level [(N, steps, converged)][, kept states])."""
    prev = None
    log = []
    kept = {}
    for i, N in enumerate(levels):
        s = Solver(N, L, mass=mass, dtype=dtypes[i], dt_over_a2=dt_over_a2, v_inf=v_inf)
        s.set_potential(kind, params)
        vw = {"f32": 4, "f64": 2, "bf16": 8}[dtypes[i]]
        if two_step and N % vw == 0:
            # a step that streams the V table (kinds past CORNELL) from HBM:
            # F32 lattices from 512^3 on take the 16 x 128 tiles, which re-read
            # fewer frame bytes
            vfuse = s.tuning()["vfuse"]
            table_v = kind > F.POT_CORNELL or not vfuse
            tile = 1 if dtypes[i] == "f32" and table_v and N >= 512 else 0
            s.set_tuning(vw, 1, 0, 0, 1, 5 if dtypes[i] == "f32" else 3, 0, 0, vfuse, 2, tile)
        if prev is None:
            s.set_initial(seed, parity=parity)
        else:
            F.fdtd_upsample(prev.h, 0, s.h, 0)
            prev.close()
        pe = 0
        if project and N in project:
            s.set_projection_states(project[N])
            pe = project_every
        tol = rel_tol[min(i, len(rel_tol) - 1)]
        mx = max_steps[min(i, len(max_steps) - 1)]
        done, conv = s.evolve(mx, check_every=check_every, rel_tol=tol, use_graph=use_graph,
                              project_every=pe)
        log.append((N, done, conv))
        if keep:
            kept[N] = s.psi_tensor(0, dtype=torch.float32)
        prev = s
    return (prev, log, kept) if keep else (prev, log)


class EnergyOfPotential(torch.autograd.Function):
    """E[psi_T](V) for a Solver whose state is the fixed start psi_0: forward
    sets V and, when V needs a gradient, runs the adjoint driver once and
    keeps dE/dV (otherwise it only relaxes and reads E); backward returns
    grad_output * dE/dV, so torch's autograd can chain through any V(theta)."""

    @staticmethod
    def forward(ctx, V: torch.Tensor, solver: Solver, psi0: torch.Tensor, steps: int,
                checkpoint_every: int):
        solver.set_potential_array(V.detach())
        solver.set_initial_array(psi0)
        if not ctx.needs_input_grad[0]:
            solver.evolve(steps, renorm_every=1, use_graph=False)
            E = solver.observables()[0]["energy"]
            ctx.save_for_backward(None)
            return torch.tensor(E, dtype=torch.float64, device=V.device)
        E, _, G = solver.energy_grad(steps, checkpoint_every, want_field=True)
        ctx.save_for_backward(G)
        return torch.tensor(E, dtype=torch.float64, device=V.device)

    @staticmethod
    def backward(ctx, grad_out):
        (G,) = ctx.saved_tensors
        return (grad_out * G).to(torch.float64), None, None, None, None
