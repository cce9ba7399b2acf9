"""Host-side logic of the learned warm start (no GPU): network inputs and
targets on padded grids, channel scales, weight storage, case sampling."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1810_00348_amd import cases, warmstart as W  # noqa: E402
from oracle import unet_oracle as U  # noqa: E402


def test_features_pad_odd_grids_with_zeros():
    c = cases.cavity(25, 17, kn=0.3, lid=0.2)
    x = W.features(c)
    assert x.shape == (28, 28, 28, 6)
    assert np.all(x[25:] == 0) and np.all(x[:, 25:] == 0) and np.all(x[:, :, 25:] == 0)
    inner = x[:25, :25, :25]
    assert np.allclose(inner[..., 0], np.log10(0.3)) and np.allclose(inner[..., 1], 0.2)
    # wall mask: 1 next to the moving lid (y = 1), 0.5 next to the other walls, 0 inside
    assert np.all(inner[:, -1, :, 2] == 1.0)
    assert inner[12, 12, 12, 2] == 0.0 and inner[0, 12, 12, 2] == 0.5 and inner[12, 12, 0, 2] == 0.5
    # cell-centre positions as fractions of the side: x varies along W, z along D
    assert np.isclose(inner[3, 4, 0, 3], 0.5 / 25) and np.isclose(inner[3, 4, 24, 3], 24.5 / 25)
    assert np.isclose(inner[3, 7, 9, 4], 7.5 / 25) and np.isclose(inner[11, 7, 9, 5], 11.5 / 25)


def test_targets_and_mask():
    c = cases.cavity(8, 8, kn=1.0, lid=0.25)
    N = 8 ** 3
    rng = np.random.default_rng(0)
    f = {"rho": 1 + 0.01 * rng.standard_normal(N), "u": 0.05 * rng.standard_normal((3, N)),
         "T": 1 + 0.01 * rng.standard_normal(N)}
    scale = np.array([2.0, 3.0, 3.0, 3.0, 4.0], np.float32)
    t, m = W.targets(c, f, scale)
    assert t.shape == (8, 8, 8, 5) and m.sum() == N
    assert np.allclose(t[..., 0].ravel(), (f["rho"] - 1) / 0.25 / 2.0, atol=1e-6)
    assert np.allclose(t[..., 2].ravel(), f["u"][1] / 0.25 / 3.0, atol=1e-6)
    assert np.allclose(t[..., 4].ravel(), (f["T"] - 1) / 0.25 / 4.0, atol=1e-6)


def test_channel_scale_shares_the_velocity_scale():
    c = cases.cavity(8, 8, lid=0.5)
    N = 8 ** 3
    rng = np.random.default_rng(1)
    f = {"rho": 1 + 0.1 * rng.standard_normal(N), "u": np.stack([rng.standard_normal(N), 0.1 * rng.standard_normal(N),
                                                                   0.001 * rng.standard_normal(N)]),
         "T": 1 + rng.standard_normal(N)}
    s = W.channel_scale([(c, f)])
    assert s[1] == s[2] == s[3]
    rms = np.sqrt(np.mean(f["u"] ** 2)) / 0.5
    assert abs(s[1] - rms) < 1e-4 * rms


def test_stored_weights_are_bf16_and_biases_exact(tmp_path):
    theta = W.init_theta(3, base=8)
    specs = U.layer_specs(W.NET_IN, 5, 8)
    assert theta.size == U.param_count(specs)
    theta[-5:] = np.float32(0.123456789)
    s = W.store_params(theta, W.layer_table(8))
    P, Q = U.unpack(theta.astype(np.float64), specs), U.unpack(s.astype(np.float64), specs)
    for (w, b), (w2, b2) in zip(P, Q):
        assert np.array_equal(U.bf16_round(w), w2)
        assert np.array_equal(b, b2)
    path = str(tmp_path / "w.npz")
    W.save_weights(path, s, np.ones(5, np.float32), {"k": 1})
    t2, cs, meta = W.load_weights(path)
    assert np.array_equal(t2, s) and meta == {"k": 1}


def test_case_sampling_ranges():
    tr = W.training_cases(64)
    assert all(c.n[0] in range(24, 49, 4) and c.m[0] in (16, 18, 20, 22, 24) for c in tr)
    assert all(0.05 <= c.kn <= 10 and 0.05 <= c.faces[3].u[0] <= 0.5 for c in tr)
    ho = W.heldout_cases(32)
    assert all(c.n[0] % 2 == 1 and c.m[0] % 2 == 0 for c in ho)
    assert {c.name for c in tr}.isdisjoint({c.name for c in ho})
    # deterministic
    assert [c.kn for c in W.training_cases(8)] == [c.kn for c in W.training_cases(8)]


def test_field_difference_norms():
    a = {"rho": np.array([1.0, 1.1]), "u": np.zeros((3, 2)), "T": np.array([1.0, 1.0])}
    b = {"rho": np.array([1.0, 1.2]), "u": np.zeros((3, 2)), "T": np.array([1.0, 1.0])}
    d = W.field_difference(a, b)
    assert abs(d["rho"] - 0.1 / 1.2) < 1e-12 and d["T"] == 0.0
    dv = W.field_difference(a, b, "dev")
    assert abs(dv["rho"] - 0.1 / 0.2) < 1e-12


def test_divergence_detector():
    from paper_1810_00348_amd.solver import diverging
    down = [1.0, 0.5, 0.3, 0.2, 0.25, 0.15, 0.1]
    assert not any(diverging(down[:k], 3) for k in range(len(down) + 1))
    up = [1.0, 0.5, 0.6, 0.9, 1.3, 2.0]
    # three growths in a row and above the start from the fifth value on
    assert [diverging(up[:k], 3) for k in range(len(up) + 1)] == [False] * 5 + [True, True]
    assert not diverging(up, 0)
    # growing, but still below the start: not yet
    assert not diverging([1.0, 0.1, 0.2, 0.3, 0.4], 3)
