"""Python front end of the HIP solver: one context per case, workspace and
stream from torch, everything else done by libdvm_hip.so."""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import _lib as L
from .cases import Case


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Solver:
    """Iterative DVM solver for one ``Case`` on one GPU.

    precision: "f64" (default) or "f32" (f stored and updated in FP32, the
    equilibrium evaluated in FP32 from per-cell parameters computed in FP64;
    moments accumulated in FP64; finalisation and residual in FP64)."""

    def __init__(self, case: Case, precision: str = "f64", device: str = "cuda:0",
                 stream: Optional[torch.cuda.Stream] = None, velocity_groups: Optional[int] = None,
                 memory_fraction: float = 0.9, schedule: Optional[dict] = None,
                 static_workspace: bool = False, parameter_bits: int = 0, sweep_streams: int = 0):
        """velocity_groups: sweep the velocity set in that many parts per
        iteration (None: the fewest parts whose workspace fits
        memory_fraction of the device's free memory).  schedule: a sweep
        kernel shape in place of the library's choice, any of the keys vl
        (velocities per lane), bx, by, bz (brick cells) and pipelined
        (True / False, or "dyn": the pipelined body in one dependency-driven
        launch); see dvm_set_schedule.  static_workspace: bind the
        library's static device workspace (no allocation; small contexts
        only, one context per device at a time; see
        dvm_bind_static_workspace) instead of a torch buffer.
        parameter_bits: 64 with precision "f32" keeps the per-cell
        parameters, Gaussian tables and the equilibrium evaluation in FP64
        (see dvm_set_parameter_precision); 0 keeps the default.
        sweep_streams: streams for the per-diagonal sweep launches (see
        dvm_set_sweep_streams); 0 keeps the default."""
        if not torch.cuda.is_available():
            raise RuntimeError("the HIP solver needs a GPU")
        self.case = case
        self.device = torch.device(device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        self.precision = {"f64": L.DVM_F64, "f32": L.DVM_F32}[precision]
        lib = L.lib()
        g = L.Grid(*case.n, *case.L)
        vg = L.VGrid((C.c_int * 3)(*case.m), (C.c_double * 3)(*case.vmax))
        gas = L.Gas(case.kn, case.omega, case.pr, int(case.correction))
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            L.check(lib.dvm_create(C.byref(g), C.byref(vg), C.byref(gas), self.precision,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        for f, face in enumerate(case.faces):
            bc = L.FaceBC(face.code, (C.c_double * 3)(*face.u), face.T, face.rho)
            L.check(lib.dvm_set_face_bc(h, f, C.byref(bc)))
        if case.solid is not None:
            self._solid = case.solid_flat()
            u = np.ascontiguousarray(case.solid_u, dtype=np.float64)
            L.check(lib.dvm_set_solid(h, self._solid.ctypes.data_as(C.c_void_p), _ptr(u), case.solid_T))
        L.check(lib.dvm_set_closed(h, int(case.closed)))
        if case.spacing is not None:
            self._spacing = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in case.spacing]
            L.check(lib.dvm_set_spacing(h, *[None if a is None else _ptr(a) for a in self._spacing]))
        if case.velocity_axes is not None:
            args = []
            self._vax = []
            for ax in case.velocity_axes:
                if ax is None:
                    args += [None, None]
                    continue
                xi, w = (np.ascontiguousarray(a, dtype=np.float64) for a in ax)
                self._vax.append((xi, w))
                args += [_ptr(xi), _ptr(w)]
            L.check(lib.dvm_set_velocity_axes(h, *args))
        if case.model != "shakhov":
            if case.model != "esbgk":
                raise ValueError(f"unknown model {case.model}")
            L.check(lib.dvm_set_model(h, 1))
        if case.order != 1:
            L.check(lib.dvm_set_order(h, int(case.order)))
        if parameter_bits:
            L.check(lib.dvm_set_parameter_precision(h, int(parameter_bits)))
        if sweep_streams:
            L.check(lib.dvm_set_sweep_streams(h, int(sweep_streams)))
        if schedule:
            unknown = set(schedule) - {"vl", "bx", "by", "bz", "pipelined"}
            if unknown:
                raise ValueError(f"unknown schedule keys {sorted(unknown)}")
            body = schedule.get("pipelined")
            code = 0 if body is None else (3 if body == "dyn" else 2 if body else 1)
            L.check(lib.dvm_set_schedule(h, int(schedule.get("vl", 0)), int(schedule.get("bx", 0)),
                                         int(schedule.get("by", 0)), int(schedule.get("bz", 0)), code))
        nbytes = C.c_size_t()
        groups = 1 if velocity_groups is None else int(velocity_groups)
        L.check(lib.dvm_set_velocity_groups(h, groups))
        L.check(lib.dvm_required_workspace(h, C.byref(nbytes)))
        if velocity_groups is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            # memory torch holds in its cache is free for this allocation too
            free += torch.cuda.memory_reserved(self.device) - torch.cuda.memory_allocated(self.device)
            info = L.Info()
            L.check(lib.dvm_get_info(h, C.byref(info)))
            while nbytes.value > memory_fraction * free and groups < info.tiles_per_octant:
                groups += 1
                L.check(lib.dvm_set_velocity_groups(h, groups))
                L.check(lib.dvm_required_workspace(h, C.byref(nbytes)))
        if static_workspace:
            self.workspace = None
            with torch.cuda.device(self.device):
                L.check(lib.dvm_bind_static_workspace(h))
        else:
            self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
            with torch.cuda.device(self.device):
                L.check(lib.dvm_bind_workspace(h, C.c_void_p(self.workspace.data_ptr()), nbytes.value))
        self.N = case.ncells

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                L.lib().dvm_destroy(h)
            except Exception:  # interpreter shutdown: module state already torn down
                pass
            self._h = None

    # ---- state
    def init_uniform(self, rho=None, u=None, T=None):
        c = self.case
        u = np.ascontiguousarray(c.init_u if u is None else u, dtype=np.float64)
        L.check(L.lib().dvm_init_uniform(self._h, c.init_rho if rho is None else rho, _ptr(u),
                                         c.init_T if T is None else T))

    def init_fields(self, rho, u, T, target_mass: float = 0.0):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(3, -1)
        T = np.ascontiguousarray(T, dtype=np.float64)
        L.check(L.lib().dvm_init_fields(self._h, _ptr(rho), _ptr(u), _ptr(T), target_mass))

    def iterate(self, n: int = 1, tol: float = 0.0):
        """Run up to n iterations (stop at residual <= tol if tol > 0).
        Returns (iterations done, residual, converged)."""
        it = C.c_int()
        r = C.c_double()
        st = L.check(L.lib().dvm_iterate(self._h, n, tol, C.byref(it), C.byref(r)))
        return it.value, r.value, st == L.DVM_OK

    def run(self, max_iters: int, tol: float = 0.0, log=None, diverge_window: int = 0):
        """Iterate one step at a time up to max_iters (or residual <= tol),
        writing one JSON line per iteration to the open file ``log`` if given
        (iteration, residual per field, total mass, wall seconds, GPt/s), and
        stopping with ``diverged`` set when the residual has grown for
        ``diverge_window`` iterations in a row above its starting value.
        Returns a dict: iterations, residual, converged, diverged, seconds."""
        import json
        import time
        hist = []
        diverged = converged = False
        t_all = time.perf_counter()
        it = 0
        for it in range(1, max_iters + 1):
            t0 = time.perf_counter()
            _, r, ok = self.iterate(1, tol=tol)
            dt = time.perf_counter() - t0
            hist.append(r)
            if log is not None:
                W, _, _, M0 = self.state()
                rec = {"it": it, "residual": r, "residual_fields": [float(x) for x in self.residual(True)],
                       "mass_rel": float(self.total_mass(W) / M0) if M0 else None, "t_iter": dt,
                       "gpt_per_s": self.case.points / dt / 1e9}
                log.write(json.dumps(rec) + "\n")
                log.flush()
            if ok:
                converged = True
                break
            if diverge_window and diverging(hist, diverge_window):
                diverged = True
                break
        return {"iterations": it, "residual": hist[-1] if hist else float("nan"), "converged": converged,
                "diverged": diverged, "seconds": time.perf_counter() - t_all}

    def total_mass(self, W=None) -> float:
        """Sum of rho times cell volume over the fluid cells."""
        if W is None:
            W = self.state()[0]
        c = self.case
        if c.spacing is not None:
            hx, hy, hz = (np.full(n, L / n) if h is None else np.asarray(h) for n, L, h in zip(c.n, c.L, c.spacing))
        else:
            hx, hy, hz = (np.full(n, L / n) for n, L in zip(c.n, c.L))
        vol = (hz[:, None, None] * hy[None, :, None] * hx[None, None, :]).ravel()
        return float((W[0] * vol).sum())

    def residual(self, per_field: bool = False):
        r = np.zeros(5)
        L.check(L.lib().dvm_get_residuals(self._h, _ptr(r)))
        return r if per_field else float(r.max())

    def fields(self):
        N = self.N
        rho = np.empty(N); u = np.empty((3, N)); T = np.empty(N); q = np.empty((3, N))
        L.check(L.lib().dvm_get_fields(self._h, _ptr(rho), _ptr(u), _ptr(T), _ptr(q)))
        return {"rho": rho, "u": u, "T": T, "q": q}

    def stress(self):
        """ES-BGK: stress per unit mass of the current iterate, 6 x N."""
        P = np.empty((6, self.N))
        L.check(L.lib().dvm_get_stress(self._h, _ptr(P)))
        return P

    def set_stress(self, P):
        P = np.ascontiguousarray(P, dtype=np.float64).reshape(6, self.N)
        L.check(L.lib().dvm_set_stress(self._h, _ptr(P)))

    def state(self):
        N = self.N
        W = np.empty((5, N)); q = np.empty((3, N)); rw = np.empty((6, N)); M0 = C.c_double()
        L.check(L.lib().dvm_get_state(self._h, _ptr(W), _ptr(q), _ptr(rw), C.byref(M0)))
        return W, q, rw, M0.value

    def set_state(self, W, q, rho_w, M0):
        W = np.ascontiguousarray(W, dtype=np.float64)
        q = np.ascontiguousarray(q, dtype=np.float64)
        rho_w = np.ascontiguousarray(rho_w, dtype=np.float64)
        L.check(L.lib().dvm_set_state(self._h, _ptr(W), _ptr(q), _ptr(rho_w), M0))

    def info(self) -> dict:
        inf = L.Info()
        L.check(L.lib().dvm_get_info(self._h, C.byref(inf)))
        return {"cells": [inf.nx, inf.ny, inf.nz], "nfluid": inf.nfluid, "m": list(inf.m),
                "nvel": inf.nvel, "precision": inf.precision, "brick": list(inf.brick),
                "vel_per_lane": inf.vel_per_lane, "tiles_per_octant": inf.tiles_per_octant,
                "sweep_launches": inf.sweep_launches, "workspace_bytes": inf.workspace_bytes,
                "sweep_kernel": ("sweep_kernel", "sweep_kernel_pf", "sweep_kernel_dyn")[inf.pipelined],
                "velocity_groups": inf.velocity_groups, "parameter_bits": inf.parameter_bits,
                "sweep_streams": inf.sweep_streams}

    def set_timing(self, enable: int = 1):
        """1: per-phase events; 2: also every sweep launch (see dvm_set_timing)."""
        L.check(L.lib().dvm_set_timing(self._h, int(enable)))

    def launch_timings(self):
        ms = C.c_double()
        n = C.c_longlong()
        L.check(L.lib().dvm_get_launch_timings(self._h, C.byref(ms), C.byref(n)))
        return {"launch_ms_total": ms.value, "launches": n.value}

    def timings(self):
        a = C.c_double(); b = C.c_double(); d = C.c_double(); n = C.c_int()
        L.check(L.lib().dvm_get_timings(self._h, C.byref(a), C.byref(b), C.byref(d), C.byref(n)))
        return {"params_ms": a.value, "sweep_ms": b.value, "finalize_ms": d.value, "iterations": n.value}


def diverging(history, window: int) -> bool:
    """True when the last ``window`` residuals each grew and the latest is
    above the first of the run (a run that has started to blow up rather
    than a transient bump on the way down)."""
    if window <= 0 or len(history) < window + 1:
        return False
    tail = history[-(window + 1):]
    return all(b > a for a, b in zip(tail, tail[1:])) and history[-1] > history[0]


def selftest_wave_reduce(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(64, 13)
    out = np.zeros(13)
    L.check(L.lib().dvm_selftest_wave_reduce(_ptr(x), _ptr(out)))
    return out


def solve_fp32_then_fp64(case: Case, tol: float = 1e-6, max_iters: int = 4000, switch_factor: float = 20.0,
                         window: int = 10, progress: float = 0.8, stall_below: float = 1e-3,
                         device: str = "cuda:0", init=None, target_mass: float = 0.0):
    """Iterate with f in FP32 until the residual reaches switch_factor * tol
    (or tol itself, or stops improving), then continue from the same state
    (W, q, wall densities, reference mass and, for ES-BGK, the stress -- all
    FP64) with f in FP64 until tol.

    FP32 storage has a noise floor in the relative residual of a field whose
    norm is small against the others (the spanwise momentum of the cavity:
    about 1e-6 to 2e-5 there), so it may never reach a tight tolerance on its
    own.  Stalled means: the residual is below ``stall_below`` and the best
    of the last ``window`` iterations is not below ``progress`` times the best
    of the window before.

    init = (rho, u, T) starts from those fields (e.g. a learned prediction,
    with target_mass the total mass to rescale them to) instead of the
    uniform state.

    Returns a dict with the iterations and wall seconds of each phase."""
    import time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = Solver(case, precision="f32", device=device)
    if init is None:
        s.init_uniform()
    else:
        s.init_fields(*init, target_mass=target_mass)
    hist = []
    it32 = 0
    ok = False
    while it32 < max_iters:
        n, r, ok = s.iterate(1, tol=tol)
        it32 += n
        hist.append(r)
        if ok or r <= switch_factor * tol:
            break
        if (r < stall_below and len(hist) >= 2 * window
                and min(hist[-window:]) > progress * min(hist[-2 * window:-window])):
            break
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t0
    out = {"f32_iters": it32, "f32_seconds": t32, "f32_residual": hist[-1] if hist else float("nan"),
           "f64_iters": 0, "f64_seconds": 0.0}
    if not ok:
        t1 = time.perf_counter()
        state = s.state()
        stress = s.stress() if case.model == "esbgk" else None
        del s
        s = Solver(case, precision="f64", device=device)
        s.set_state(*state)
        if stress is not None:
            s.set_stress(stress)
        n, r, ok = s.iterate(max(1, max_iters - it32), tol=tol)
        torch.cuda.synchronize()
        out["f64_iters"] = n
        out["f64_seconds"] = time.perf_counter() - t1
        out["residual"] = r
    else:
        out["residual"] = hist[-1]
    out["converged"] = ok
    out["seconds"] = out["f32_seconds"] + out["f64_seconds"]
    out["iters"] = out["f32_iters"] + out["f64_iters"]
    out["fields"] = s.fields()
    return out
