"""dvm_bind_static_workspace: a context on the library's static device
workspace (no allocation) iterates exactly like the same context on a lent
workspace; two contexts in a row, the second smaller; the static array
passes from one context to the next."""
import ctypes as C

import numpy as np
import pytest

from paper_1810_00348_amd import cases

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


def _solver():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_00348_amd.solver import Solver
    return Solver


def _errors(a, b):
    out = {}
    for k in ("rho", "T"):
        out[k] = np.abs(a[k] - b[k]).max() / np.abs(b[k]).max()
    big = np.abs(b["u"]).max()
    for d in range(3):
        den = max(np.abs(b["u"][d]).max(), 1e-3 * big, 1e-4)
        out["u%d" % d] = np.abs(a["u"][d] - b["u"][d]).max() / den
    return out


def test_static_workspace_matches_lent_workspace():
    Solver = _solver()
    from paper_1810_00348_amd import _lib as L
    big = cases.config("c1")                                         # 16^3 x 12^3, 35 MiB
    small = cases.cavity((10, 9, 11), 10, kn=2.0, lid=0.3)           # 7.4 MiB
    first = None
    for case, init_seed, iters in ((big, None, 4), (small, 3, 3)):
        ref = Solver(case)
        s = Solver(case, static_workspace=True)
        assert s.workspace is None
        assert s.info()["workspace_bytes"] <= 64 << 20
        if init_seed is None:
            ref.init_uniform()
            s.init_uniform()
        else:
            init = cases.random_fields(case, seed=init_seed)
            ref.init_fields(*init)
            s.init_fields(*init)
        for _ in range(iters):
            ref.iterate(1)
            s.iterate(1)
        err = _errors(s.fields(), ref.fields())
        print(case.name, err)
        for k, v in err.items():
            assert v <= FP64_TOL, (case.name, k, err)
        assert abs(s.residual() - ref.residual()) <= 1e-8 * ref.residual()
        if first is None:
            first = s
        else:
            # the second context took the static array from the first
            with pytest.raises(L.DvmError) as e:
                first.iterate(1)
            assert e.value.status == L.DVM_ERR_STATE
            # the current owner keeps working
            s.iterate(1)
            ref.iterate(1)
            err = _errors(s.fields(), ref.fields())
            for k, v in err.items():
                assert v <= FP64_TOL, (k, err)
        del ref


def test_static_workspace_rejects_large_contexts():
    Solver = _solver()
    from paper_1810_00348_amd import _lib as L
    case = cases.cavity((24, 24, 24), 20, kn=1.0, lid=0.16)
    with pytest.raises(L.DvmError) as e:
        Solver(case, static_workspace=True)
    assert e.value.status == L.DVM_ERR_OOM
    assert "static workspace" in str(e.value)
