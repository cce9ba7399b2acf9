"""ctypes binding of the plain FP64 CPU oracle (dvm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of the benchmark.  The product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dvm_oracle.c")
LIB = os.path.join(HERE, "libdvm_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, FP64, no fast-math)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", "-D_DEFAULT_SOURCE",
               "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Case(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
        ("m", C.c_int * 3),
        ("vmax", C.c_double * 3),
        ("kn", C.c_double), ("omega", C.c_double), ("pr", C.c_double),
        ("correction", C.c_int),
        ("face_kind", C.c_int * 6),
        ("face_u", (C.c_double * 3) * 6),
        ("face_T", C.c_double * 6),
        ("face_rho", C.c_double * 6),
        ("closed", C.c_int),
        ("solid_u", C.c_double * 3),
        ("solid_T", C.c_double),
        ("threads", C.c_int),
    ]


_lib = None
_P = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(_Case), C.c_void_p]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_init_uniform.argtypes = [C.c_void_p, C.c_double, _P, C.c_double]
        L.orc_init_fields.argtypes = [C.c_void_p, _P, _P, _P]
        L.orc_iterate.argtypes = [C.c_void_p]
        L.orc_residual.restype = C.c_double
        L.orc_residual.argtypes = [C.c_void_p, _P]
        L.orc_get_state.argtypes = [C.c_void_p, _P, _P, _P]
        L.orc_set_state.argtypes = [C.c_void_p, _P, _P, _P, C.c_double]
        L.orc_get_fields.argtypes = [C.c_void_p, _P, _P, _P, _P]
        L.orc_total_mass.restype = C.c_double
        L.orc_total_mass.argtypes = [C.c_void_p]
        L.orc_initial_mass.restype = C.c_double
        L.orc_initial_mass.argtypes = [C.c_void_p]
        L.orc_get_ghat.argtypes = [C.c_void_p, C.c_int, _P, _P]
        L.orc_sweep_one.argtypes = [C.c_void_p, C.c_int, _P, _P, _P, _P]
        L.orc_velocity_axis.argtypes = [C.c_int, C.c_double, _P, _P]
        L.orc_kappa.restype = C.c_double
        L.orc_kappa.argtypes = [C.c_double]
        L.orc_equilibrium.argtypes = [C.POINTER(C.c_int), C.POINTER(_P), C.POINTER(_P),
                                      C.c_double, _P, C.c_double, _P, C.c_double, C.c_int, _P]
        L.orc_num_threads.argtypes = [C.c_void_p]
        L.orc_set_spacing.argtypes = [C.c_void_p, _P, _P, _P]
        L.orc_set_order.argtypes = [C.c_void_p, C.c_int]
        L.orc_set_velocity_axis.argtypes = [C.c_void_p, C.c_int, _P, _P]
        L.orc_set_model.argtypes = [C.c_void_p, C.c_int]
        L.orc_get_stress.argtypes = [C.c_void_p, _P]
        L.orc_esbgk_gaussian.argtypes = [C.POINTER(C.c_int), C.POINTER(_P), C.c_double, _P, C.c_double,
                                         _P, C.c_double, _P]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_P)


def velocity_axis(M: int, V: float):
    xi = np.empty(M)
    w = np.empty(M)
    if lib().orc_velocity_axis(M, V, _ptr(xi), _ptr(w)) != 0:
        raise ValueError("bad velocity axis")
    return xi, w


def kappa(omega: float) -> float:
    return lib().orc_kappa(omega)


def equilibrium(m, vmax, rho, U, T, q=(0.0, 0.0, 0.0), pr=2.0 / 3.0, correct=True):
    """Corrected (or plain) Shakhov equilibrium on the full velocity grid,
    returned as an array [mz, my, mx]."""
    axes = [velocity_axis(m[d], vmax[d]) for d in range(3)]
    xis = [np.ascontiguousarray(a[0]) for a in axes]
    ws = [np.ascontiguousarray(a[1]) for a in axes]
    XI = (_P * 3)(*[_ptr(x) for x in xis])
    WW = (_P * 3)(*[_ptr(x) for x in ws])
    mm = (C.c_int * 3)(*m)
    out = np.empty(m[0] * m[1] * m[2])
    U = np.ascontiguousarray(U, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    st = lib().orc_equilibrium(mm, XI, WW, rho, _ptr(U), T, _ptr(q), pr, int(correct), _ptr(out))
    if st != 0:
        raise ValueError("non-physical equilibrium state")
    return out.reshape(m[2], m[1], m[0])


def esbgk_gaussian(m, vmax, rho, U, T, theta, pr=2.0 / 3.0):
    """The ES-BGK Gaussian (no correction) for stress per unit mass theta
    (xx, yy, zz, xy, xz, yz) on the uniform velocity grid, [mz, my, mx]."""
    axes = [velocity_axis(m[d], vmax[d]) for d in range(3)]
    xis = [np.ascontiguousarray(a[0]) for a in axes]
    XI = (_P * 3)(*[_ptr(x) for x in xis])
    mm = (C.c_int * 3)(*m)
    out = np.empty(m[0] * m[1] * m[2])
    U = np.ascontiguousarray(U, dtype=np.float64)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    if lib().orc_esbgk_gaussian(mm, XI, rho, _ptr(U), T, _ptr(th), pr, _ptr(out)) != 0:
        raise ValueError("non-physical ES-BGK state")
    return out.reshape(m[2], m[1], m[0])


class Oracle:
    """The plain FP64 iteration on one case."""

    def __init__(self, case, threads: int = 0):
        self.case = case
        cs = _Case()
        cs.nx, cs.ny, cs.nz = case.n
        cs.lx, cs.ly, cs.lz = case.L
        for d in range(3):
            cs.m[d] = case.m[d]
            cs.vmax[d] = case.vmax[d]
        cs.kn, cs.omega, cs.pr = case.kn, case.omega, case.pr
        cs.correction = int(case.correction)
        for f, face in enumerate(case.faces):
            cs.face_kind[f] = face.code
            for d in range(3):
                cs.face_u[f][d] = face.u[d]
            cs.face_T[f] = face.T
            cs.face_rho[f] = face.rho
        cs.closed = int(case.closed)
        for d in range(3):
            cs.solid_u[d] = case.solid_u[d]
        cs.solid_T = case.solid_T
        cs.threads = threads
        self._cs = cs
        solid = case.solid_flat()
        self._solid = solid
        sp = solid.ctypes.data_as(C.c_void_p) if solid is not None else None
        self._h = lib().orc_create(C.byref(cs), sp)
        if not self._h:
            raise ValueError("oracle rejected the case")
        self.N = case.ncells
        sp3 = getattr(case, "spacing", None)
        if sp3 is not None:
            self._sp = [None if h is None else np.ascontiguousarray(h, dtype=np.float64) for h in sp3]
            if lib().orc_set_spacing(self._h, *[None if h is None else _ptr(h) for h in self._sp]) != 0:
                raise ValueError("bad cell sizes")
        vax = getattr(case, "velocity_axes", None)
        if vax is not None:
            self._vax = []
            for d, ax in enumerate(vax):
                if ax is None:
                    continue
                xi, w = (np.ascontiguousarray(a, dtype=np.float64) for a in ax)
                self._vax.append((xi, w))
                if lib().orc_set_velocity_axis(self._h, d, _ptr(xi), _ptr(w)) != 0:
                    raise ValueError(f"bad velocity axis {d}")
        model = getattr(case, "model", "shakhov")
        if model != "shakhov":
            if model != "esbgk" or lib().orc_set_model(self._h, 1) != 0:
                raise ValueError(f"unknown model {model}")
        order = getattr(case, "order", 1)
        if order != 1 and lib().orc_set_order(self._h, order) != 0:
            raise ValueError("the upwind order must be 1 or 2")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    @property
    def threads(self) -> int:
        return lib().orc_num_threads(self._h)

    def init_uniform(self, rho=None, u=None, T=None):
        c = self.case
        rho = c.init_rho if rho is None else rho
        u = np.ascontiguousarray(c.init_u if u is None else u, dtype=np.float64)
        T = c.init_T if T is None else T
        if lib().orc_init_uniform(self._h, rho, _ptr(u), T) != 0:
            raise ValueError("non-physical initial state")

    def init_fields(self, rho, u, T):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(3, -1)
        T = np.ascontiguousarray(T, dtype=np.float64)
        if lib().orc_init_fields(self._h, _ptr(rho), _ptr(u), _ptr(T)) != 0:
            raise ValueError("non-physical initial state")

    def iterate(self, n: int = 1) -> float:
        for _ in range(n):
            if lib().orc_iterate(self._h) != 0:
                raise FloatingPointError("non-physical state during iteration")
        return self.residual()

    def residual(self, per_field: bool = False):
        r = np.zeros(5)
        m = lib().orc_residual(self._h, _ptr(r))
        return r if per_field else m

    def state(self):
        N = self.N
        W = np.empty((5, N)); q = np.empty((3, N)); rw = np.empty((6, N))
        lib().orc_get_state(self._h, _ptr(W), _ptr(q), _ptr(rw))
        return W, q, rw

    def set_state(self, W, q, rho_w, M0):
        W = np.ascontiguousarray(W, dtype=np.float64)
        q = np.ascontiguousarray(q, dtype=np.float64)
        rho_w = np.ascontiguousarray(rho_w, dtype=np.float64)
        lib().orc_set_state(self._h, _ptr(W), _ptr(q), _ptr(rho_w), M0)

    def fields(self):
        N = self.N
        rho = np.empty(N); u = np.empty((3, N)); T = np.empty(N); q = np.empty((3, N))
        lib().orc_get_fields(self._h, _ptr(rho), _ptr(u), _ptr(T), _ptr(q))
        return {"rho": rho, "u": u, "T": T, "q": q}

    def stress(self):
        """ES-BGK: the stress per unit mass of the current iterate, 6 x N
        (xx, yy, zz, xy, xz, yz)."""
        P = np.empty((6, self.N))
        lib().orc_get_stress(self._h, _ptr(P))
        return P

    def total_mass(self) -> float:
        return lib().orc_total_mass(self._h)

    def initial_mass(self) -> float:
        return lib().orc_initial_mass(self._h)

    def ghat(self, kind: int):
        g = np.empty(self.case.nvel)
        go = np.empty(6)
        if lib().orc_get_ghat(self._h, kind, _ptr(g), _ptr(go)) != 0:
            raise ValueError("no emission shape for that kind")
        return g, go

    def sweep_one(self, alpha: int, spec_mirror=None):
        N = self.N
        f = np.empty(N); feq = np.empty(N); nu = np.empty(N)
        sp = None
        if spec_mirror is not None:
            spec_mirror = np.ascontiguousarray(spec_mirror, dtype=np.float64)
            sp = _ptr(spec_mirror)
        if lib().orc_sweep_one(self._h, alpha, sp, _ptr(f), _ptr(feq), _ptr(nu)) != 0:
            raise ValueError("sweep failed")
        return f, feq, nu
