"""The C-ABI library loads and exports every entry point that include/*.h
declares; host-only calls (no GPU work) behave as documented."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols(header="dvm.h", prefix="dvm_"):
    src = open(os.path.join(ROOT, "include", header)).read()
    pat = r"^\s*(?:dvm_status|int|size_t|const char\*|void)\s+(" + prefix + r"\w+)\s*\("
    return sorted(set(re.findall(pat, src, re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_1810_00348_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1810_00348_amd import build
        build.build()
    return _lib


def test_every_declared_symbol_is_exported(L):
    lib = L.lib()
    syms = declared_symbols()
    assert len(syms) >= 18
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) <= set(L.EXPORTS), set(syms) - set(L.EXPORTS)


def test_every_warm_start_symbol_is_exported(L):
    lib = L.lib()
    syms = declared_symbols("wsn.h", "wsn_")
    assert len(syms) == 16, syms
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(os.listdir(os.path.join(ROOT, "include"))) == ["dvm.h", "wsn.h"]


def test_warm_start_argument_errors(L):
    from paper_1810_00348_amd import warmstart as W
    lib = W.wsn_lib()
    h = C.c_void_p()
    # rejected before any device call
    assert lib.wsn_create(3, 5, 12, 16, 16, 16, None, C.byref(h)) == -1
    assert b"multiple of 8" in lib.wsn_last_error()
    assert lib.wsn_create(3, 5, 32, 18, 16, 16, None, C.byref(h)) == -1
    assert lib.wsn_create(3, 5, 128, 16, 16, 16, None, C.byref(h)) == -1
    assert lib.wsn_create(3, 5, 32, 16, 16, 16, None, None) == -1
    assert not h.value
    assert lib.wsn_num_params(None) == 0
    assert lib.wsn_forward(None, None, 4, 4, 4, None) == -1
    assert lib.wsn_test_conv(4, 4, 4, 3, 5, 9, None, None, None, None, None, None, None, None) == -1


def _ctx(L, case, prec=0):
    lib = L.lib()
    g = L.Grid(*case.n, *case.L)
    vg = L.VGrid((C.c_int * 3)(*case.m), (C.c_double * 3)(*case.vmax))
    gas = L.Gas(case.kn, case.omega, case.pr, 1)
    h = C.c_void_p()
    assert lib.dvm_create(C.byref(g), C.byref(vg), C.byref(gas), prec, None, C.byref(h)) == 0
    return h


def test_workspace_sizes_fit_one_gpu(L):
    from paper_1810_00348_amd import cases
    lib = L.lib()
    for name, prec in (("c1", 0), ("c2", 0), ("c3", 1), ("c3", 0), ("c4", 1)):
        case = cases.config(name)
        h = _ctx(L, case, prec)
        for f, face in enumerate(case.faces):
            bc = L.FaceBC(face.code, (C.c_double * 3)(*face.u), face.T, face.rho)
            assert lib.dvm_set_face_bc(h, f, C.byref(bc)) == 0
        n = C.c_size_t()
        assert lib.dvm_required_workspace(h, C.byref(n)) == 0
        info = L.Info()
        assert lib.dvm_get_info(h, C.byref(info)) == 0
        assert info.nvel == case.nvel and info.ncells == case.ncells
        assert 0 < n.value < 200 * 2 ** 30, (name, n.value / 2 ** 30)
        lib.dvm_destroy(h)


def test_argument_errors(L):
    from paper_1810_00348_amd import cases
    lib = L.lib()
    case = cases.config("c1")
    g = L.Grid(0, 4, 4, 1.0, 1.0, 1.0)
    vg = L.VGrid((C.c_int * 3)(8, 8, 8), (C.c_double * 3)(5, 5, 5))
    gas = L.Gas(1.0, 0.81, 2 / 3, 1)
    h = C.c_void_p()
    assert lib.dvm_create(C.byref(g), C.byref(vg), C.byref(gas), 0, None, C.byref(h)) == -1
    assert b"grid" in lib.dvm_last_error()
    h = _ctx(L, case)
    bc = L.FaceBC(2, (C.c_double * 3)(0, 0, 0), 1.0, 1.0)
    assert lib.dvm_set_face_bc(h, 0, C.byref(bc)) == -1          # specular only on z-
    assert lib.dvm_set_face_bc(h, 4, C.byref(bc)) == 0
    assert lib.dvm_iterate(h, 1, 0.0, None, None) == -2           # not initialised
    assert lib.dvm_init_uniform(h, 1.0, (C.c_double * 3)(0, 0, 0), 1.0) == -2  # no workspace
    assert lib.dvm_bind_workspace(h, C.c_void_p(1024), 10) == -3  # too small
    lib.dvm_destroy(h)


def test_spacing_arguments(L):
    """dvm_set_spacing: host-side validation and the variant it selects."""
    import numpy as np
    from paper_1810_00348_amd import cases
    lib = L.lib()
    case = cases.cavity((6, 5, 4), 16, kn=1.0)
    h = _ctx(L, case)
    P = C.POINTER(C.c_double)
    good = np.full(6, 1.0 / 6)
    bad_sum = np.full(6, 0.2)
    neg = good.copy()
    neg[2] = -neg[2]
    assert lib.dvm_set_spacing(h, bad_sum.ctypes.data_as(P), None, None) == -1
    assert b"sum" in lib.dvm_last_error()
    assert lib.dvm_set_spacing(h, neg.ctypes.data_as(P), None, None) == -1
    hy = cases.stretched_axis(5, 1.0, 1.3)
    assert lib.dvm_set_spacing(h, good.ctypes.data_as(P), hy.ctypes.data_as(P), None) == 0
    inf = L.Info()
    assert lib.dvm_get_info(h, C.byref(inf)) == 0
    # FP64 with 8 nodes per x half on a stretched mesh: 4 per lane, 4x2
    # bricks, pipelined body
    assert (inf.vel_per_lane, inf.brick[0], inf.brick[1], inf.pipelined) == (4, 4, 2, 1)
    n = C.c_size_t()
    assert lib.dvm_required_workspace(h, C.byref(n)) == 0
    assert lib.dvm_bind_workspace(h, C.c_void_p(1 << 20), 16) == -3
    lib.dvm_destroy(h)


def test_velocity_groups_arguments_and_workspace(L):
    """dvm_set_velocity_groups: argument checks, the tile split it reports
    and the workspace it saves; the paper's full-domain cube fits one device
    only with groups."""
    import numpy as np
    from paper_1810_00348_amd import cases
    lib = L.lib()
    case = cases.config("c6")
    h = _ctx(L, case, 1)
    P = C.POINTER(C.c_double)
    sp = [np.ascontiguousarray(a) for a in case.spacing]
    assert lib.dvm_set_spacing(h, *[a.ctypes.data_as(P) for a in sp]) == 0
    assert lib.dvm_set_velocity_groups(h, 0) == -1
    assert b"groups" in lib.dvm_last_error()
    sizes = {}
    for groups in (1, 2, 3, 1000):
        assert lib.dvm_set_velocity_groups(h, groups) == 0
        n = C.c_size_t()
        assert lib.dvm_required_workspace(h, C.byref(n)) == 0
        info = L.Info()
        assert lib.dvm_get_info(h, C.byref(info)) == 0
        assert info.velocity_groups == min(groups, info.tiles_per_octant)
        assert info.tiles_per_octant == 54 and info.vel_per_lane == 4
        sizes[groups] = n.value
    assert sizes[1] > 288e9                   # one group: more than the device holds
    assert sizes[2] < 250e9 and sizes[3] < 0.7 * sizes[2]
    assert sizes[1000] < sizes[3]
    assert lib.dvm_bind_workspace(h, C.c_void_p(1 << 20), 16) == -3
    assert lib.dvm_set_velocity_groups(h, 2) == 0
    lib.dvm_destroy(h)


def test_order_arguments(L):
    """dvm_set_order: 1 or 2, before binding; the second order re-derives
    the schedule (FP64: 2 per lane, pipelined body) and doubles the face
    buffers; on a stretched mesh it adds the table of slope weights and
    needs the pipelined body."""
    import numpy as np
    from paper_1810_00348_amd import cases
    lib = L.lib()
    case = cases.cavity((6, 5, 4), 16, kn=1.0)
    h = _ctx(L, case)
    n1 = C.c_size_t()
    assert lib.dvm_required_workspace(h, C.byref(n1)) == 0
    assert lib.dvm_set_order(h, 3) == -1 and b"order" in lib.dvm_last_error()
    assert lib.dvm_set_order(h, 2) == 0
    info = L.Info()
    assert lib.dvm_get_info(h, C.byref(info)) == 0
    # the second-order FP64 form runs 2 per lane on 4x2 bricks
    assert info.pipelined == 1 and (info.vel_per_lane, info.brick[0], info.brick[1]) == (2, 4, 2)
    n2 = C.c_size_t()
    assert lib.dvm_required_workspace(h, C.byref(n2)) == 0
    assert n2.value > n1.value
    P = C.POINTER(C.c_double)
    hy = cases.stretched_axis(5, 1.0, 1.3)
    assert lib.dvm_set_spacing(h, None, hy.ctypes.data_as(P), None) == 0
    n3 = C.c_size_t()
    assert lib.dvm_required_workspace(h, C.byref(n3)) == 0
    assert n3.value > n2.value
    assert lib.dvm_set_order(h, 1) == 0
    assert lib.dvm_set_order(h, 2) == 0
    # the plain body has no stretched second-order form: binding refuses
    assert lib.dvm_set_schedule(h, 0, 0, 0, 0, 1) == 0
    assert lib.dvm_bind_workspace(h, C.c_void_p(1 << 20), 1 << 40) == -1
    assert b"pipelined" in lib.dvm_last_error()
    lib.dvm_destroy(h)


def test_velocity_axes_arguments(L):
    import numpy as np
    from paper_1810_00348_amd import cases
    lib = L.lib()
    case = cases.cavity((6, 5, 4), 10, kn=1.0)
    h = _ctx(L, case)
    P = C.POINTER(C.c_double)
    xi, w = cases.graded_velocity_axis(10, 5.0, 1.2)
    p = lambda a: np.ascontiguousarray(a).ctypes.data_as(P)
    keep = [xi, w, xi[::-1].copy(), xi + 0.01, -w]
    assert lib.dvm_set_velocity_axes(h, p(keep[0]), None, None, None, None, None) == -1
    assert lib.dvm_set_velocity_axes(h, p(keep[2]), p(keep[1]), None, None, None, None) == -1
    assert lib.dvm_set_velocity_axes(h, p(keep[3]), p(keep[1]), None, None, None, None) == -1
    assert b"symmetric" in lib.dvm_last_error()
    assert lib.dvm_set_velocity_axes(h, p(keep[0]), p(keep[4]), None, None, None, None) == -1
    assert lib.dvm_set_velocity_axes(h, p(keep[0]), p(keep[1]), None, None, p(keep[0]), p(keep[1])) == 0
    assert lib.dvm_set_velocity_axes(h, None, None, None, None, None, None) == 0
    lib.dvm_destroy(h)


def test_model_arguments(L):
    import numpy as np
    from paper_1810_00348_amd import cases
    lib = L.lib()
    case = cases.cavity((6, 5, 4), 10, kn=1.0)
    h = _ctx(L, case)
    assert lib.dvm_set_model(h, 2) == -1
    assert lib.dvm_set_model(h, 1) == 0
    info = L.Info()
    # the usual schedule: 5 nodes per x half in FP64 -> 1 per lane (2 would
    # leave a sixth of the slots empty), plain body
    assert lib.dvm_get_info(h, C.byref(info)) == 0 and (info.vel_per_lane, info.pipelined) == (1, 0)
    P = (C.c_double * (6 * case.ncells))()
    assert lib.dvm_get_stress(h, P) == -2          # no state yet
    hy = cases.stretched_axis(5, 1.0, 1.3)
    assert lib.dvm_set_spacing(h, None, hy.ctypes.data_as(C.POINTER(C.c_double)), None) == -1
    assert lib.dvm_set_model(h, 0) == 0
    assert lib.dvm_get_stress(h, P) == -2          # Shakhov keeps no stress
    assert lib.dvm_set_stress(h, P) == -2
    lib.dvm_destroy(h)
    low = cases.cavity((6, 5, 4), 10, kn=1.0, pr=0.5)
    g = L.Grid(*low.n, *low.L)
    vg = L.VGrid((C.c_int * 3)(*low.m), (C.c_double * 3)(*low.vmax))
    gas = L.Gas(low.kn, low.omega, low.pr, 1)
    h = C.c_void_p()
    assert lib.dvm_create(C.byref(g), C.byref(vg), C.byref(gas), 0, None, C.byref(h)) == 0
    assert lib.dvm_set_model(h, 1) == -1 and b"Pr" in lib.dvm_last_error()
    lib.dvm_destroy(h)


@pytest.mark.parametrize("name,prec,order,model,expect", [
    # (VL, BX, BY, BZ, pipelined) chosen by the library for the benchmark workloads
    ("c2", 0, 1, 0, (4, 4, 2, 16, 1)),    # FP64, 16 nodes per x half
    ("c2", 0, 1, 1, (4, 3, 2, 16, 1)),    # ES-BGK FP64: 3x2 bricks
    ("c2", 0, 2, 0, (2, 4, 2, 16, 1)),    # second order FP64: 2 per lane
    ("c3", 1, 2, 0, (4, 3, 2, 12, 1)),    # second order FP32: 3x2 bricks
    ("c3", 1, 1, 0, (4, 4, 2, 12, 1)),    # FP32, 14 nodes per half (empty slots)
    ("c3", 0, 1, 0, (4, 4, 2, 16, 1)),    # FP64, 14 nodes per half (empty slots)
    ("c4", 1, 1, 0, (4, 4, 2, 12, 1)),    # FP32, 24 nodes per half
    ("c1", 0, 1, 0, (2, 4, 2, 16, 1)),    # FP64, 6 nodes per half
])
def test_default_schedule_of_the_benchmark_workloads(L, name, prec, order, model, expect):
    """The sweep shape the library picks for each workload (host-only: no
    device work happens before a workspace is bound)."""
    from paper_1810_00348_amd import cases
    lib = L.lib()
    case = cases.config(name)
    h = _ctx(L, case, prec)
    if order == 2:
        assert lib.dvm_set_order(h, 2) == 0
    if model == 1:
        assert lib.dvm_set_model(h, 1) == 0
    info = L.Info()
    assert lib.dvm_get_info(h, C.byref(info)) == 0
    got = (info.vel_per_lane, info.brick[0], info.brick[1], info.brick[2], info.pipelined)
    assert got == expect, (name, prec, order, model, got)
    lib.dvm_destroy(h)


def test_esbgk_on_a_stretched_mesh_schedule(L):
    """ES-BGK on a stretched mesh takes the pipelined sweep with 2 or more
    velocities per lane; a velocity set that leaves 1 per lane is refused
    and the mesh left uniform (host-only: no device work)."""
    import numpy as np
    from paper_1810_00348_amd import cases
    lib = L.lib()
    case = cases.config("c2")
    h = _ctx(L, case, 0)
    assert lib.dvm_set_model(h, 1) == 0
    hx = cases.stretched_axis(case.n[0], case.L[0], 1.02)
    assert lib.dvm_set_spacing(h, hx.ctypes.data_as(C.POINTER(C.c_double)), None, None) == 0
    info = L.Info()
    assert lib.dvm_get_info(h, C.byref(info)) == 0
    got = (info.vel_per_lane, info.brick[0], info.brick[1], info.brick[2], info.pipelined)
    assert got == (4, 3, 2, 16, 1), got
    # the plain body has no ES-BGK kernel on a stretched mesh or on 3x2 bricks
    assert lib.dvm_set_schedule(h, 4, 3, 2, 0, 1) == 0
    assert lib.dvm_bind_workspace(h, C.c_void_p(1 << 20), 1 << 40) == -1
    assert b"pipelined" in lib.dvm_last_error()
    lib.dvm_destroy(h)
    # 5 nodes per x half in FP64: 1 per lane, no stretched ES-BGK kernel
    small = cases.cavity((6, 5, 4), 10, kn=1.0)
    h = _ctx(L, small)
    assert lib.dvm_set_model(h, 1) == 0
    hy = cases.stretched_axis(5, 1.0, 1.3)
    assert lib.dvm_set_spacing(h, None, hy.ctypes.data_as(C.POINTER(C.c_double)), None) == -1
    assert b"stretched" in lib.dvm_last_error()
    assert lib.dvm_get_info(h, C.byref(info)) == 0 and info.vel_per_lane == 1
    assert lib.dvm_set_model(h, 0) == 0
    assert lib.dvm_set_spacing(h, None, hy.ctypes.data_as(C.POINTER(C.c_double)), None) == 0
    assert lib.dvm_set_model(h, 1) == -1 and b"stretched" in lib.dvm_last_error()
    lib.dvm_destroy(h)


def test_brick_columns_shortened_for_32bit_face_offsets(L):
    """The sweep addresses a face cell of its brick by a 32-bit byte offset:
    on a wide grid with many velocities the library shortens the brick
    columns so that (BZ - 1) * max(nx, ny) + max(BX, BY) face cells stay
    below 4 GiB (host-only: no device work)."""
    from paper_1810_00348_amd import cases
    lib = L.lib()
    # 2000 x 2000 x 2 cells, 64^3 velocities, FP64: an octant has 32^3
    # velocities = 8192 lanes of 4 = 128 tiles, so one face cell holds
    # 128 x 64 x 4 x 8 bytes = 256 KiB and 4 GiB holds 16384 of them:
    # (BZ - 1) * 2000 + 4 < 16384 -> BZ <= 9; halving from 16 gives 8
    case = cases.cavity((2000, 2000, 2), 64, kn=1.0)
    h = _ctx(L, case, 0)
    info = L.Info()
    assert lib.dvm_get_info(h, C.byref(info)) == 0
    assert (info.vel_per_lane, info.brick[0], info.brick[1]) == (4, 4, 2)
    assert info.brick[2] == 8, tuple(info.brick)
    lib.dvm_destroy(h)
    # the benchmark grid keeps its 16-cell columns
    h = _ctx(L, cases.config("c2"), 0)
    assert lib.dvm_get_info(h, C.byref(info)) == 0 and info.brick[2] == 16
    lib.dvm_destroy(h)


def test_schedule_requests(L):
    """dvm_set_schedule picks a built kernel shape or refuses (host-only)."""
    from paper_1810_00348_amd import cases
    lib = L.lib()
    info = L.Info()
    h = _ctx(L, cases.config("c2"), 0)
    # a built shape: taken, the column length and body as given
    assert lib.dvm_set_schedule(h, 2, 4, 2, 7, 1) == 0
    assert lib.dvm_get_info(h, C.byref(info)) == 0
    assert (info.vel_per_lane, *info.brick, info.pipelined) == (2, 4, 2, 7, 0)
    # a shape that is not built: refused, the previous request stays
    assert lib.dvm_set_schedule(h, 4, 5, 2, 0, 0) == -1 and b"built" in lib.dvm_last_error()
    assert lib.dvm_get_info(h, C.byref(info)) == 0
    assert (info.vel_per_lane, *info.brick, info.pipelined) == (2, 4, 2, 7, 0)
    # out of range
    for args in ((9, 0, 0, 0, 0), (0, 0, 0, 0, 4), (0, -1, 0, 0, 0)):
        assert lib.dvm_set_schedule(h, *args) == -1
    # all zero: the library's choice again
    assert lib.dvm_set_schedule(h, 0, 0, 0, 0, 0) == 0
    assert lib.dvm_get_info(h, C.byref(info)) == 0
    assert (info.vel_per_lane, *info.brick, info.pipelined) == (4, 4, 2, 16, 1)
    # velocities per lane alone: the brick defaults of that width
    assert lib.dvm_set_schedule(h, 1, 0, 0, 0, 0) == 0
    assert lib.dvm_get_info(h, C.byref(info)) == 0
    assert (info.vel_per_lane, info.brick[0], info.brick[1]) == (1, 4, 4)
    # a shape built for the first order only, then the second order: the
    # request has no kernel any more and binding refuses it (before any
    # device work)
    assert lib.dvm_set_schedule(h, 4, 3, 2, 0, 2) == 0
    assert lib.dvm_set_order(h, 2) == 0
    assert lib.dvm_bind_workspace(h, C.c_void_p(4096), 1 << 40) == -1
    assert b"dvm_set_schedule" in lib.dvm_last_error()
    lib.dvm_destroy(h)
    # the solid-mask name is the same call
    h = _ctx(L, cases.cavity((3, 3, 3), 4), 0)
    mask = (C.c_ubyte * 27)(*([0] * 13 + [1] + [0] * 13))
    u = (C.c_double * 3)(0.0, 0.0, 0.0)
    assert lib.dvm_set_solid_mask(h, mask, u, 1.0) == 0
    assert lib.dvm_get_info(h, C.byref(info)) == 0 and info.nfluid == 26
    assert lib.dvm_set_solid_mask(h, mask, u, 0.0) == -1
    lib.dvm_destroy(h)


def test_z_face_offsets_bound_the_schedule(L):
    """The z face of a brick is addressed up to cell (BY - 1) * nx + BX - 1:
    on a grid so long in x that one face row of the velocity set overflows
    32-bit offsets even with one-cell columns, binding refuses the case
    (host-only: refused before any device work)."""
    from paper_1810_00348_amd import cases
    lib = L.lib()
    info = L.Info()
    # 64^3 velocities, FP64, 4 per lane: 256 KiB per face cell, 16384 face
    # cells in 4 GiB; a 20000-cell x extent puts the second z-face row of a
    # 4x2 brick beyond that
    case = cases.cavity((20000, 2, 2), 64, kn=1.0)
    h = _ctx(L, case, 0)
    assert lib.dvm_get_info(h, C.byref(info)) == 0
    assert (info.vel_per_lane, info.brick[0], info.brick[1], info.brick[2]) == (4, 4, 2, 1)
    assert lib.dvm_bind_workspace(h, C.c_void_p(4096), 1 << 40) == -1
    assert b"32-bit" in lib.dvm_last_error()
    # velocity groups shrink the face rows and let it through the check
    assert lib.dvm_set_velocity_groups(h, 4) == 0
    assert lib.dvm_get_info(h, C.byref(info)) == 0 and info.brick[2] >= 1
    lib.dvm_destroy(h)


def test_static_workspace_size_limit(L):
    """dvm_bind_static_workspace refuses a context larger than the static
    array before it touches a device, and leaves the context unbound."""
    from paper_1810_00348_amd import cases
    lib = L.lib()
    h = _ctx(L, cases.config("c2"))
    n = C.c_size_t()
    assert lib.dvm_required_workspace(h, C.byref(n)) == 0
    assert n.value > 64 << 20
    assert lib.dvm_bind_static_workspace(h) == -3
    msg = lib.dvm_last_error()
    assert b"static workspace" in msg and str(64 << 20).encode() in msg
    assert lib.dvm_init_uniform(h, 1.0, (C.c_double * 3)(0, 0, 0), 1.0) == -2  # still unbound
    lib.dvm_destroy(h)


def test_dependency_driven_schedule_and_parameter_precision(L):
    """Body 3 (one dependency-driven launch) exists for the first-order
    Shakhov sweep only; FP64 parameters beside FP32 storage for the 4-per-lane
    4x2 pipelined shape only (host-only checks)."""
    from paper_1810_00348_amd import cases
    lib = L.lib()
    info = L.Info()
    h = _ctx(L, cases.config("c2"), 0)
    assert lib.dvm_set_schedule(h, 0, 0, 0, 0, 3) == 0
    assert lib.dvm_get_info(h, C.byref(info)) == 0
    assert info.pipelined == 2 and info.sweep_launches == 1 and info.parameter_bits == 64
    assert lib.dvm_set_order(h, 2) == 0
    # the request has no second-order kernel: binding refuses
    assert lib.dvm_bind_workspace(h, C.c_void_p(1 << 20), 1 << 40) == -1
    assert lib.dvm_set_parameter_precision(h, 32) == -1          # FP64 context
    assert lib.dvm_set_parameter_precision(h, 64) == 0
    lib.dvm_destroy(h)
    h = _ctx(L, cases.config("c3"), 1)
    assert lib.dvm_set_parameter_precision(h, 48) == -1
    assert lib.dvm_set_parameter_precision(h, 64) == 0
    assert lib.dvm_get_info(h, C.byref(info)) == 0
    assert info.parameter_bits == 64 and info.vel_per_lane == 4 and tuple(info.brick[:2]) == (4, 2)
    n = C.c_size_t()
    assert lib.dvm_required_workspace(h, C.byref(n)) == 0
    assert lib.dvm_set_parameter_precision(h, 32) == 0
    m = C.c_size_t()
    assert lib.dvm_required_workspace(h, C.byref(m)) == 0
    assert n.value > m.value                                    # FP64 record and tables
    assert lib.dvm_set_parameter_precision(h, 64) == 0
    assert lib.dvm_set_schedule(h, 2, 4, 2, 0, 0) == 0
    assert lib.dvm_bind_workspace(h, C.c_void_p(1 << 20), 1 << 40) == -1
    assert b"FP64 parameters" in lib.dvm_last_error()
    lib.dvm_destroy(h)
