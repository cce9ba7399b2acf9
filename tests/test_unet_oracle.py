"""Pins of the FP64 U-Net reference (oracle/unet_oracle.py): brute-force
definitions, adjointness, finite differences, closed forms."""
import numpy as np
import pytest

from oracle import unet_oracle as U


def brute_conv(x, W, b):
    D, H, Wd, Ci = x.shape
    Co = W.shape[1]
    y = np.zeros((D, H, Wd, Co))
    taps = U.TAPS if W.shape[0] == 27 else [(0, 0, 0)]
    for d in range(D):
        for h in range(H):
            for w in range(Wd):
                for o in range(Co):
                    s = b[o]
                    for t, (dz, dy, dx) in enumerate(taps):
                        zz, yy, xx = d + dz, h + dy, w + dx
                        if 0 <= zz < D and 0 <= yy < H and 0 <= xx < Wd:
                            for i in range(Ci):
                                s += W[t, o, i] * x[zz, yy, xx, i]
                    y[d, h, w, o] = s
    return y


def test_conv3d_matches_definition():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 4, 2))
    W = rng.standard_normal((27, 3, 2))
    b = rng.standard_normal(3)
    assert np.abs(U.conv3d(x, W, b) - brute_conv(x, W, b)).max() < 1e-12
    W1 = rng.standard_normal((1, 3, 2))
    assert np.abs(U.conv3d(x, W1, b) - brute_conv(x, W1, b)).max() < 1e-12


def test_conv3d_backward_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 2, 3, 2))
    W = rng.standard_normal((27, 2, 2))
    b = rng.standard_normal(2)
    gy = rng.standard_normal((3, 2, 3, 2))
    gx, gW, gb = U.conv3d_backward(x, W, gy)
    f = lambda x_, W_, b_: (U.conv3d(x_, W_, b_) * gy).sum()
    eps = 1e-6
    for arr, g in ((x, gx), (W, gW), (b, gb)):
        for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]:
            old = arr[idx]
            arr[idx] = old + eps
            fp = f(x, W, b)
            arr[idx] = old - eps
            fm = f(x, W, b)
            arr[idx] = old
            assert abs((fp - fm) / (2 * eps) - g[idx]) < 1e-6


def test_pool_and_upsample_are_adjoint_to_their_backward():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4, 6, 2, 3))
    y = rng.standard_normal((2, 3, 1, 3))
    assert abs((U.avgpool2(x) * y).sum() - (x * U.avgpool2_backward(y)).sum()) < 1e-12
    z = rng.standard_normal((4, 6, 2, 3))
    assert abs((U.upsample2(y) * z).sum() - (y * U.upsample2_backward(z)).sum()) < 1e-12
    # average of a constant is the constant; upsampling repeats
    assert np.allclose(U.avgpool2(np.ones((4, 4, 4, 1))), 1.0)
    assert U.upsample2(np.arange(2.0).reshape(1, 1, 2, 1))[0, 0, :, 0].tolist() == [0, 0, 1, 1]


def test_network_gradient_finite_differences():
    specs = U.layer_specs(cin=3, cout=2, base=2)
    theta = U.init_params(specs, seed=3)
    theta += 0.05 * np.random.default_rng(4).standard_normal(theta.size)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((4, 4, 4, 3))
    t = rng.standard_normal((4, 4, 4, 2))
    mask = (rng.random((4, 4, 4)) > 0.2).astype(float)

    def loss(th):
        return U.mse(U.forward(th, x, specs), t, mask)[0]

    y, tape = U.forward(theta, x, specs, keep=True)
    L, gy = U.mse(y, t, mask)
    g = U.backward(theta, tape, gy, specs)
    assert g.shape == theta.shape
    eps = 1e-6
    for k in rng.choice(theta.size, 40, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += eps
        tm[k] -= eps
        fd = (loss(tp) - loss(tm)) / (2 * eps)
        assert abs(fd - g[k]) < 1e-6 + 1e-5 * abs(fd), (k, fd, g[k])


def test_param_count_of_the_warm_start_network():
    # 3 levels, 32 base channels, inputs (log Kn, lid speed, wall mask),
    # outputs (rho, u, T): about 1.4 M parameters
    assert U.param_count(U.layer_specs(3, 5, 32)) == 1413445


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3])
    th, m, v = U.adam(np.zeros(3), np.zeros(3), np.zeros(3), g, step=1, lr=0.01)
    assert np.allclose(th, -0.01 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-12)


def test_bf16_round_known_values():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.140625, 65504.0, 1e-3])
    r = U.bf16_round(v)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie -> even mantissa
    assert r[2] == 1.0 + 2 ** -7            # above half-way -> up
    assert r[3] == -3.140625                # exactly representable
    assert r[4] == 65536.0
    assert abs(r[5] - 1e-3) < 1e-3 * 2 ** -8
