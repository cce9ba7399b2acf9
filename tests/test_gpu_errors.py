"""Failure handling of the HIP path, forced from the host (no kernel is made
to fault): a non-physical state is detected by the parameter kernel, the
iteration reports it, and the context keeps the last good iterate."""
import numpy as np
import pytest

from paper_1810_00348_amd import cases

pytestmark = pytest.mark.gpu


def _solver():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_00348_amd import _lib
    from paper_1810_00348_amd.solver import Solver
    return Solver, _lib


def test_nonphysical_state_is_reported_and_last_good_iterate_kept():
    Solver, L = _solver()
    case = cases.cavity((8, 7, 6), 8, kn=1.0, lid=0.2)
    s = Solver(case)
    s.init_uniform()
    s.iterate(2)
    good = s.state()
    W, q, rw, M0 = [x.copy() if isinstance(x, np.ndarray) else x for x in good]
    W[4, 17] = -1.0          # negative energy: T < 0 in one cell
    s.set_state(W, q, rw, M0)
    with pytest.raises(L.DvmError) as err:
        s.iterate(3)
    assert err.value.status == L.DVM_ERR_NONPHYSICAL
    assert np.array_equal(s.state()[0], W)        # the state before the failed iteration
    # the context stays usable
    s.set_state(*good)
    n, r, _ = s.iterate(1)
    assert n == 1 and np.isfinite(r)


def test_invalid_initial_fields_are_rejected():
    Solver, L = _solver()
    case = cases.cavity((6, 6, 6), 8, kn=1.0, lid=0.2)
    s = Solver(case)
    rho, u, T = cases.random_fields(case, seed=3)
    T[5] = 0.0
    with pytest.raises(L.DvmError) as err:
        s.init_fields(rho, u, T)
    assert err.value.status == L.DVM_ERR_NONPHYSICAL
    with pytest.raises(L.DvmError) as err:
        s.iterate(1)                               # never initialised
    assert err.value.status == L.DVM_ERR_STATE


def test_not_converged_is_a_soft_status():
    Solver, L = _solver()
    case = cases.cavity((6, 6, 6), 8, kn=1.0, lid=0.2)
    s = Solver(case)
    s.init_uniform()
    n, r, ok = s.iterate(2, tol=1e-12)
    assert n == 2 and not ok and r > 1e-12
