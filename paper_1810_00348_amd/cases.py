"""Workload definitions and seeded synthetic inputs.

This module only *describes* problems (grids, velocity grids, gas constants,
boundary conditions, initial fields).  It holds none of the method's
arithmetic, so both the HIP library binding and the CPU oracle can take their
inputs from it.

Units follow the normalisation of the solver: lengths in units of the
reference length L that defines the Knudsen number, velocities in units of
the most probable speed sqrt(2 R T0), temperature in units of T0, density in
units of rho0.

Workloads (all synthetic; the paper's DSMC data and figures are not used):

* ``cavity``: the 3D lid-driven cavity of Sec. 4.1 -- unit cube, all six
  walls diffuse at T = 1, the top wall (y = 1) moving along +x.
* ``cube``: supersonic flow past a cube (Sec. 4.2), re-parameterised as a
  symmetry half-domain: specular plane at z = 0, free stream on the other
  five faces, a diffuse cube wall.
* ``cube_paper``: the paper's own full-domain cube run (stretched
  191 x 181 x 181 mesh, 48^3 velocities, Ma 2, Kn 1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence, Tuple

import numpy as np

FACE_NAMES = ("x-", "x+", "y-", "y+", "z-", "z+")
WALL, FREE, SPECULAR = 0, 1, 2
KIND_CODES = {"wall": WALL, "free": FREE, "specular": SPECULAR}


@dataclasses.dataclass
class Face:
    """Boundary condition on one face of the box.

    kind: 'wall' (Maxwell diffuse wall with velocity u and temperature T),
          'free' (particles entering get the equilibrium of (rho, u, T)),
          'specular' (mirror reflection; only supported on z-).
    """

    kind: str = "wall"
    u: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    T: float = 1.0
    rho: float = 1.0

    @property
    def code(self) -> int:
        return KIND_CODES[self.kind]


@dataclasses.dataclass
class Case:
    name: str
    n: Tuple[int, int, int]
    L: Tuple[float, float, float]
    m: Tuple[int, int, int]
    vmax: Tuple[float, float, float]
    kn: float
    omega: float = 0.81
    pr: float = 2.0 / 3.0
    correction: bool = True
    faces: Sequence[Face] = dataclasses.field(default_factory=lambda: [Face() for _ in range(6)])
    closed: bool = True
    solid: Optional[np.ndarray] = None   # uint8 [nz, ny, nx], 1 = solid
    solid_u: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    solid_T: float = 1.0
    init_rho: float = 1.0
    init_u: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    init_T: float = 1.0
    # cell sizes along x, y, z (arrays of length nx, ny, nz summing to L),
    # None for a uniform mesh
    spacing: Optional[Tuple[Optional[np.ndarray], Optional[np.ndarray], Optional[np.ndarray]]] = None
    # spatial order of the upwind scheme: 1 (the paper's), or 2 (linear
    # upwind extrapolation from the cell and its upwind neighbour)
    order: int = 1
    # velocity nodes and quadrature weights per axis, (xi, w) pairs of
    # length m[d] (None: m[d] uniform nodes on [-vmax, vmax], trapezoid)
    velocity_axes: Optional[Tuple] = None
    # collision model: "shakhov" (the paper's) or "esbgk" (ellipsoidal
    # statistical BGK: anisotropic Gaussian, relaxation frequency Pr p / mu)
    model: str = "shakhov"

    @property
    def ncells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def nfluid(self) -> int:
        if self.solid is None:
            return self.ncells
        return int(self.ncells - int(np.count_nonzero(self.solid)))

    @property
    def nvel(self) -> int:
        return self.m[0] * self.m[1] * self.m[2]

    @property
    def points(self) -> int:
        """Phase-space points updated per iteration (fluid cells x velocities)."""
        return self.nfluid * self.nvel

    def solid_flat(self) -> Optional[np.ndarray]:
        if self.solid is None:
            return None
        return np.ascontiguousarray(self.solid.reshape(-1).astype(np.uint8))

    def describe(self) -> dict:
        return {
            "name": self.name,
            "cells": list(self.n),
            "velocities": list(self.m),
            "vmax": list(self.vmax),
            "kn": self.kn,
            "fluid_cells": self.nfluid,
            "points": self.points,
        }


def cavity(n: int | Tuple[int, int, int] = 16, m: int | Tuple[int, int, int] = 12,
           kn: float = 1.0, lid: float = 0.16, vmax: float = 5.0,
           omega: float = 0.81, pr: float = 2.0 / 3.0, correction: bool = True,
           name: Optional[str] = None) -> Case:
    """Lid-driven cubic cavity: all walls diffuse at T = 1; the y+ wall moves
    along +x with speed ``lid`` (z is the spanwise direction)."""
    nn = (n, n, n) if isinstance(n, int) else tuple(n)
    mm = (m, m, m) if isinstance(m, int) else tuple(m)
    faces = [Face("wall") for _ in range(6)]
    faces[3] = Face("wall", u=(lid, 0.0, 0.0))
    return Case(name=name or f"cavity_{nn[0]}x{nn[1]}x{nn[2]}_v{mm[0]}",
                n=nn, L=(1.0, 1.0, 1.0), m=mm, vmax=(vmax, vmax, vmax), kn=kn,
                omega=omega, pr=pr, correction=correction, faces=faces,
                closed=True)


def cube_half(nx: int = 64, ny: int = 48, nz: int = 48, edge: int = 8,
              x0: int = 16, m: int = 48, vmax: float = 12.0, mach: float = 5.0,
              kn: float = 0.1, T_inf: float = 1.0, T_wall: float = 1.0,
              name: Optional[str] = None) -> Case:
    """Supersonic flow past a cube, symmetry half-domain.

    The cube has ``edge`` cells per side; the length unit is the cube edge,
    so the cell size is 1/edge.  The cube is bisected by the specular plane
    z = 0 (solid cells z in [0, edge/2)), centred in y, its upstream face at
    cell x0.  Inflow along +x at Mach ``mach`` (gamma = 5/3, so the speed
    in units of sqrt(2 R T) is mach * sqrt(5/6) * sqrt(T_inf)).
    """
    if edge % 2:
        raise ValueError("cube edge must be an even number of cells")
    h = 1.0 / edge
    u_inf = mach * math.sqrt(5.0 / 6.0 * T_inf)
    solid = np.zeros((nz, ny, nx), dtype=np.uint8)
    y0 = (ny - edge) // 2
    solid[0:edge // 2, y0:y0 + edge, x0:x0 + edge] = 1
    free = Face("free", u=(u_inf, 0.0, 0.0), T=T_inf, rho=1.0)
    faces = [dataclasses.replace(free) for _ in range(6)]
    faces[4] = Face("specular")
    return Case(name=name or f"cube_half_{nx}x{ny}x{nz}_v{m}",
                n=(nx, ny, nz), L=(nx * h, ny * h, nz * h), m=(m, m, m),
                vmax=(vmax, vmax, vmax), kn=kn, faces=faces, closed=False,
                solid=solid, solid_u=(0.0, 0.0, 0.0), solid_T=T_wall,
                init_rho=1.0, init_u=(u_inf, 0.0, 0.0), init_T=T_inf)


def cube_full_mirror(half: Case) -> Case:
    """The full domain of which ``half`` is the z >= 0 half: the solid mask is
    mirrored about z = 0 and the z- face gets the z+ condition."""
    nx, ny, nz = half.n
    solid = np.concatenate([half.solid[::-1], half.solid], axis=0)
    faces = list(half.faces)
    faces[4] = dataclasses.replace(faces[5])
    return dataclasses.replace(half, name=half.name + "_full", n=(nx, ny, 2 * nz),
                               L=(half.L[0], half.L[1], 2 * half.L[2]), solid=solid,
                               faces=faces)


def graded_segment(length: float, n: int, h0: float) -> np.ndarray:
    """n cell sizes h0 r, h0 r^2, ..., h0 r^n (growing away from a cell of
    size h0) with the ratio r chosen so that they sum to ``length``."""
    if n < 1 or not (length > 0 and h0 > 0):
        raise ValueError("need n >= 1 cells, a positive length and a positive h0")
    k = np.arange(1, n + 1, dtype=np.float64)
    lo, hi = 0.25, 4.0
    for _ in range(200):
        r = 0.5 * (lo + hi)
        if h0 * np.sum(r ** k) > length:
            hi = r
        else:
            lo = r
    h = h0 * r ** k
    return h * (length / h.sum())


def body_fitted_axis(n_body: int, body_len: float, before: float, n_before: int, after: float,
                     n_after: int) -> np.ndarray:
    """Cell sizes along one axis of a mesh around a body: n_body equal cells
    across the body, graded geometrically away from it on both sides
    (``before`` / ``after``: lengths of the two sides)."""
    h0 = body_len / n_body
    return np.concatenate([graded_segment(before, n_before, h0)[::-1], np.full(n_body, h0),
                           graded_segment(after, n_after, h0)])


def cube_paper(n_body: int = 31, n_side: int = 75, n_front: int = 65, n_rear: int = 95,
               m: int = 48, vmax: float = 4.0, mach: float = 2.0, kn: float = 1.0,
               front: float = 4.5, rear: float = 8.5, side: float = 5.5,
               name: Optional[str] = None) -> Case:
    """The full-domain cube of Sec. 4.2: a unit cube in a 14 x 12 x 12 box,
    free stream at Mach ``mach`` along +x on all six faces, a diffuse cube
    wall at the free-stream temperature, 48^3 velocities on [-4, 4]^3 (units
    of sqrt(2 R T_wall)).  Mesh: ``n_body`` equal cells across the cube and
    cells growing geometrically away from it -- ``n_side`` cells over the
    ``side`` length on each lateral side, ``n_front`` over the ``front``
    length upstream and ``n_rear`` over the ``rear`` length downstream.  The
    defaults give 191 x 181 x 181 cells with growth ratios of about 1.02 in
    every direction (the paper's faster growth downstream, 1.03, would leave
    fewer than its 191 cells along x over this length)."""
    hx = body_fitted_axis(n_body, 1.0, front, n_front, rear, n_rear)
    hy = body_fitted_axis(n_body, 1.0, side, n_side, side, n_side)
    hz = hy.copy()
    nx, ny, nz = hx.size, hy.size, hz.size
    u_inf = mach * math.sqrt(5.0 / 6.0)
    solid = np.zeros((nz, ny, nx), dtype=np.uint8)
    solid[n_side:n_side + n_body, n_side:n_side + n_body, n_front:n_front + n_body] = 1
    free = Face("free", u=(u_inf, 0.0, 0.0), T=1.0, rho=1.0)
    return Case(name=name or f"cube_full_{nx}x{ny}x{nz}_v{m}",
                n=(nx, ny, nz), L=(float(hx.sum()), float(hy.sum()), float(hz.sum())),
                m=(m, m, m), vmax=(vmax, vmax, vmax), kn=kn,
                faces=[dataclasses.replace(free) for _ in range(6)], closed=False,
                solid=solid, solid_u=(0.0, 0.0, 0.0), solid_T=1.0,
                init_rho=1.0, init_u=(u_inf, 0.0, 0.0), init_T=1.0, spacing=(hx, hy, hz))


def gauss_hermite_axis(M: int, scale: float = 1.0):
    """M Gauss-Hermite nodes and weights for integrals over the whole line of
    functions that decay like exp(-xi^2 / scale^2) (the rest Maxwellian at
    T = scale^2): nodes scale * x_i, weights scale * w_i * exp(x_i^2), with
    (x_i, w_i) the rule for the weight exp(-x^2); symmetric about 0."""
    x, w = np.polynomial.hermite.hermgauss(M)
    xi = scale * x
    wt = scale * w * np.exp(x * x)
    return 0.5 * (xi - xi[::-1]), 0.5 * (wt + wt[::-1])


def graded_velocity_axis(M: int, vmax: float, ratio: float):
    """M nodes on [-vmax, vmax], spaced most finely around 0 and growing
    geometrically by ``ratio`` towards +-vmax, with trapezoid weights on
    those nodes."""
    if M < 2 or ratio <= 0:
        raise ValueError("need M >= 2 and a positive ratio")
    half = M // 2
    gaps = ratio ** np.arange(half, dtype=np.float64)    # outward from the centre
    if M % 2:
        pos = np.cumsum(gaps)                            # nodes 0 < ... on the + side
        pos = pos * (vmax / pos[-1])
        xi = np.concatenate([-pos[::-1], [0.0], pos])
    else:
        g = gaps.copy()
        g[0] *= 0.5                                      # the two central nodes at +-g0/2
        pos = np.cumsum(g)
        pos = pos * (vmax / pos[-1])
        xi = np.concatenate([-pos[::-1], pos])
    w = np.empty(M)
    w[1:-1] = 0.5 * (xi[2:] - xi[:-2])
    w[0] = 0.5 * (xi[1] - xi[0])
    w[-1] = 0.5 * (xi[-1] - xi[-2])
    return xi, 0.5 * (w + w[::-1])


# ---- the configurations the benchmark and the parity tests use ------------

def config(name: str, **kw) -> Case:
    """Named workloads.

    c1: cavity 16^3 cells x 12^3 velocities on [-5,5]^3, Kn=1, lid 0.16 (FP64)
    c2: cavity 64^3 x 32^3, lid 0.16, Kn from {0.1, 1, 10} (FP64)
    c3: cavity 96^3 x 28^3, Kn=0.5, lid 0.3 (FP32 storage form)
    c4: cube half-domain 64x48x48 cells, 48^3 velocities on [-12,12]^3,
        Ma=5, Kn=0.1 (FP32 storage form)
    c6: the full-domain cube of Sec. 4.2, 191x181x181 stretched cells x 48^3
        velocities on [-4,4]^3, Ma=2, Kn=1 (6.9e11 points; FP32 storage
        form, velocity groups to fit one device)
    """
    if name == "c1":
        return cavity(16, 12, kn=kw.get("kn", 1.0), lid=0.16, vmax=5.0, name="c1_cavity_16^3_v12^3")
    if name == "c2":
        kn = kw.get("kn", 1.0)
        return cavity(64, 32, kn=kn, lid=0.16, vmax=5.0, name=f"c2_cavity_64^3_v32^3_kn{kn:g}")
    if name == "c3":
        return cavity(96, 28, kn=0.5, lid=0.3, vmax=5.0, name="c3_cavity_96^3_v28^3")
    if name == "c4":
        return cube_half(64, 48, 48, edge=8, x0=16, m=48, vmax=12.0, mach=5.0, kn=0.1,
                         name="c4_cube_half_64x48x48_v48^3")
    if name == "c6":
        return cube_paper(name="c6_cube_full_191x181x181_v48^3")
    raise KeyError(name)


def random_fields(case: Case, seed: int, drho: float = 0.2, du: float = 0.2,
                  dT: float = 0.2):
    """Seeded smooth-ish positive random initial fields (rho, u[3], T), each a
    flat array in cell order i + nx*(j + ny*k)."""
    rng = np.random.default_rng(seed)
    N = case.ncells
    rho = case.init_rho * (1.0 + drho * (rng.random(N) - 0.5))
    u = np.empty((3, N))
    for d in range(3):
        u[d] = case.init_u[d] + du * (rng.random(N) - 0.5)
    T = case.init_T * (1.0 + dT * (rng.random(N) - 0.5))
    return rho, u, T


def stretched_axis(n: int, length: float, ratio: float, centre: Optional[float] = None) -> np.ndarray:
    """Cell sizes of a mesh line of n cells and the given length that grow
    geometrically by ``ratio`` away from the two ends (centre None: cells
    cluster at both walls, as next to the cavity walls) or away from the
    interior point ``centre`` (cells cluster there, as around a body)."""
    if ratio <= 0:
        raise ValueError("ratio must be positive")
    idx = np.arange(n, dtype=np.float64)
    if centre is None:
        k = np.minimum(idx, n - 1 - idx)
    else:
        pos = (idx + 0.5) / n * length
        k = np.floor(np.abs(pos - centre) / (length / n))
    h = ratio ** k
    return h * (length / h.sum())


def stretched(case: Case, ratio: float, centres=(None, None, None)) -> Case:
    """The same case on a mesh stretched along every axis (same cell counts
    and lengths)."""
    sp = tuple(stretched_axis(case.n[d], case.L[d], ratio, centres[d]) for d in range(3))
    return dataclasses.replace(case, spacing=sp, name=case.name + f"_stretch{ratio:g}")
