"""The dependency-driven sweep (one launch per velocity group and specular
phase; waves take bricks from a device-wide counter in diagonal order and
wait for their upwind bricks' ready flags) against the oracle, and bit for
bit against the per-diagonal launches of the same body: both sweep every
brick with the same arithmetic and write every moment record once, so the
iterates are identical."""
import numpy as np
import pytest

from paper_1810_00348_amd import cases

from test_gpu_parity import FP64_TOL, _group_cases, _ragged_cases, _solver, field_errors, run_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["ragged", "oddM", "cube", "nocorr", "bgk"])
def test_dependency_driven_sweep_matches_oracle(oracle_mod, name):
    case = _ragged_cases()[name]
    init = cases.random_fields(case, seed=7) if name in ("ragged", "bgk") else None
    s, o = run_pair(case, 3, oracle_mod, init=init, schedule=dict(pipelined="dyn"))
    info = s.info()
    assert info["sweep_kernel"] == "sweep_kernel_dyn", info
    err = field_errors(s.fields(), o.fields())
    print(name, err, info)
    for k in ("rho", "ux", "uy", "uz", "T"):
        assert err[k] <= FP64_TOL, (k, err)


@pytest.mark.parametrize("name,groups", [("cavity", 3), ("cube_half", 2)])
def test_dependency_driven_sweep_with_velocity_groups(oracle_mod, name, groups):
    case = _group_cases()[name]
    init = cases.random_fields(case, seed=33) if name == "cavity" else None
    s, o = run_pair(case, 3, oracle_mod, init=init, groups=groups, schedule=dict(pipelined="dyn"))
    info = s.info()
    assert info["sweep_kernel"] == "sweep_kernel_dyn" and info["velocity_groups"] == groups, info
    err = field_errors(s.fields(), o.fields())
    for k in ("rho", "ux", "uy", "uz", "T", "qx", "qy"):
        assert err[k] <= FP64_TOL, (k, err)


def _pair_bitwise(case, precision, iters, sched, init=None):
    Solver = _solver()
    out = []
    for body in (True, "dyn"):
        s = Solver(case, precision=precision, schedule=dict(sched, pipelined=body))
        if init is None:
            s.init_uniform()
        else:
            s.init_fields(*init)
        s.iterate(iters)
        out.append((s.state(), s.residual(per_field=True), s.info()))
        del s
    (a, ra, ia), (b, rb, ib) = out
    assert ia["sweep_kernel"] == "sweep_kernel_pf" and ib["sweep_kernel"] == "sweep_kernel_dyn"
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    assert np.array_equal(ra, rb)


@pytest.mark.parametrize("precision,vl,bx", [("f64", 4, 3), ("f64", 2, 4), ("f32", 4, 4)])
def test_dependency_driven_sweep_is_bitwise_the_diagonal_sweep(precision, vl, bx):
    case = cases.cavity((13, 10, 19), 16, kn=0.3, lid=0.4, vmax=4.5)
    _pair_bitwise(case, precision, 3, dict(vl=vl, bx=bx, by=2), init=cases.random_fields(case, seed=4))


def test_dependency_driven_sweep_cube_fp32_bitwise():
    case = cases.cube_half(nx=16, ny=12, nz=8, edge=4, x0=4, m=24, vmax=12.0, mach=5.0, kn=0.1)
    _pair_bitwise(case, "f32", 4, dict(vl=4, bx=4, by=2))


@pytest.mark.parametrize("name", ["ragged", "cube"])
def test_sweep_streams_give_the_same_iterate(oracle_mod, name):
    """The per-diagonal launches of disjoint octant sets on 1, 2, 4 (and,
    without a specular plane, 8) streams: every octant's sweep and moment
    records are the same, so the iterates agree bit for bit, and with the
    oracle to the FP64 bar."""
    Solver = _solver()
    case = _ragged_cases()[name]
    init = cases.random_fields(case, seed=7) if name == "ragged" else None
    counts = (1, 2, 4, 8) if name == "ragged" else (1, 2, 4)
    states = []
    for ns in counts:
        s = Solver(case, sweep_streams=ns)
        assert s.info()["sweep_streams"] == ns
        if init is None:
            s.init_uniform()
        else:
            s.init_fields(*init)
        s.iterate(3)
        states.append((s.state(), s.fields()))
        del s
    for st, _ in states[1:]:
        for x, y in zip(st[:3], states[0][0][:3]):
            assert np.array_equal(x, y)
    o = oracle_mod.Oracle(case)
    if init is None:
        o.init_uniform()
    else:
        o.init_fields(*init)
    o.iterate(3)
    err = field_errors(states[-1][1], o.fields())
    for k in ("rho", "ux", "uy", "uz", "T"):
        assert err[k] <= FP64_TOL, (k, err)
