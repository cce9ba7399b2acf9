"""Learned warm start of the iterative DVM solver.

A 3D U-Net (include/wsn.h, HIP/MFMA kernels in csrc/wsn.hip) maps the inputs
(log10 Kn, lid speed, wall mask) on the cell grid of a lid-driven cavity to
its converged macroscopic fields (rho, U, T).  The prediction seeds the
solver: the initial equilibrium is built from the predicted fields (the paper
builds it from the initial macroscopic fields, Sec. 2.2), rescaled to the
uniform start's total mass; the solver's own residual must still reach the
same tolerance, and the plain uniform start is the fallback.

Training data are converged fields that the solver itself produces over a
sweep of Kn and lid speed.  Everything here is data movement and driving;
the network arithmetic runs in the HIP kernels.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
import time
from typing import Dict, List, Optional

import numpy as np
import torch

from . import _lib as L
from . import cases

NET_IN, NET_OUT, NET_BASE = 3, 5, 32
_wsn = None


def _P(t):
    return C.c_void_p(t.data_ptr())


def wsn_lib():
    global _wsn
    if _wsn is None:
        lib = L.lib()
        sig = {
            "wsn_create": ([C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p,
                            C.POINTER(C.c_void_p)], C.c_int),
            "wsn_num_params": ([C.c_void_p], C.c_size_t),
            "wsn_set_params": ([C.c_void_p, C.c_void_p], C.c_int),
            "wsn_get_params": ([C.c_void_p, C.c_void_p], C.c_int),
            "wsn_get_grads": ([C.c_void_p, C.c_void_p], C.c_int),
            "wsn_forward": ([C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p], C.c_int),
            "wsn_backward_mse": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_float,
                                  C.POINTER(C.c_double)], C.c_int),
            "wsn_zero_grad": ([C.c_void_p], C.c_int),
            "wsn_adam_step": ([C.c_void_p, C.c_float, C.c_float, C.c_float, C.c_float], C.c_int),
            "wsn_test_conv": ([C.c_int] * 6 + [C.c_void_p] * 8, C.c_int),
            "wsn_selftest_mfma": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
            "wsn_last_error": ([], C.c_char_p),
            "wsn_destroy": ([C.c_void_p], None),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _wsn = lib
    return _wsn


def _chk(rc):
    if rc != 0:
        raise RuntimeError(f"wsn error {rc}: {wsn_lib().wsn_last_error().decode()}")


def _np(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


class WarmStartNet:
    """The U-Net on one GPU (weights, Adam state, activations for grids up to
    max_grid)."""

    def __init__(self, max_grid=(48, 48, 48), base: int = NET_BASE, cin: int = NET_IN,
                 cout: int = NET_OUT, device: str = "cuda:0"):
        self.device = torch.device(device)
        self.cin, self.cout, self.base = cin, cout, base
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        D, H, W = (pad4(n) for n in max_grid)
        with torch.cuda.device(self.device):
            _chk(wsn_lib().wsn_create(cin, cout, base, D, H, W, C.c_void_p(self.stream.cuda_stream),
                                      C.byref(h)))
        self._h = h
        self.max_grid = (D, H, W)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            wsn_lib().wsn_destroy(h)
            self._h = None

    @property
    def num_params(self) -> int:
        return int(wsn_lib().wsn_num_params(self._h))

    def set_params(self, theta: np.ndarray):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        assert theta.size == self.num_params
        _chk(wsn_lib().wsn_set_params(self._h, _np(theta)))

    def params(self) -> np.ndarray:
        out = np.empty(self.num_params, dtype=np.float32)
        _chk(wsn_lib().wsn_get_params(self._h, _np(out)))
        return out

    def grads(self) -> np.ndarray:
        out = np.empty(self.num_params, dtype=np.float32)
        _chk(wsn_lib().wsn_get_grads(self._h, _np(out)))
        return out

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        """x: [D, H, W, cin] float32 on the device -> [D, H, W, cout]."""
        D, H, W, c = x.shape
        assert c == self.cin and x.dtype == torch.float32 and x.is_contiguous()
        y = torch.empty((D, H, W, self.cout), dtype=torch.float32, device=self.device)
        _chk(wsn_lib().wsn_forward(self._h, _P(x), D, H, W, _P(y)))
        return y

    def backward_mse(self, target: torch.Tensor, mask: torch.Tensor, weight: float = 1.0) -> float:
        loss = C.c_double(0.0)
        _chk(wsn_lib().wsn_backward_mse(self._h, _P(target), _P(mask), weight, C.byref(loss)))
        return loss.value

    def zero_grad(self):
        _chk(wsn_lib().wsn_zero_grad(self._h))

    def adam_step(self, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
        _chk(wsn_lib().wsn_adam_step(self._h, lr, beta1, beta2, eps))


# ------------------------------------------------------------------ data

def pad4(n: int) -> int:
    return (n + 3) // 4 * 4


def features(case: cases.Case) -> np.ndarray:
    """[D, H, W, 3] network input on the grid padded to multiples of 4 (the
    padding cells are all zero): log10 Kn, lid speed, wall mask (1 next to the
    moving lid, 0.5 next to the other walls, 0 inside)."""
    nx, ny, nz = case.n
    D, H, W = pad4(nz), pad4(ny), pad4(nx)
    x = np.zeros((D, H, W, 3), dtype=np.float32)
    lid = case.faces[3].u[0]
    x[:nz, :ny, :nx, 0] = math.log10(case.kn)
    x[:nz, :ny, :nx, 1] = lid
    m = np.zeros((nz, ny, nx), dtype=np.float32)
    m[0, :, :] = m[-1, :, :] = 0.5
    m[:, 0, :] = m[:, :, 0] = m[:, :, -1] = 0.5
    m[:, -1, :] = 1.0
    x[:nz, :ny, :nx, 2] = m
    return x


def target_scale(case: cases.Case) -> float:
    """Deviations from the rest state scale with the lid speed."""
    return abs(case.faces[3].u[0])


def targets(case: cases.Case, fields: Dict[str, np.ndarray], chan_std: np.ndarray):
    """Network targets [D, H, W, 5] and cell mask [D, H, W] on the padded grid:
    ((rho - 1), u, (T - 1)) / lid speed / per-channel scale."""
    nx, ny, nz = case.n
    D, H, W = pad4(nz), pad4(ny), pad4(nx)
    t = np.zeros((D, H, W, 5), dtype=np.float32)
    s = target_scale(case)
    t[:nz, :ny, :nx, 0] = (fields["rho"].reshape(nz, ny, nx) - 1.0) / s
    for d in range(3):
        t[:nz, :ny, :nx, 1 + d] = fields["u"][d].reshape(nz, ny, nx) / s
    t[:nz, :ny, :nx, 4] = (fields["T"].reshape(nz, ny, nx) - 1.0) / s
    t /= chan_std[None, None, None, :]
    mask = np.zeros((D, H, W), dtype=np.float32)
    mask[:nz, :ny, :nx] = 1.0
    return t, mask


def sample_cases(n: int, seed: int, sizes, vsizes, name: str) -> List[cases.Case]:
    """Cavities with Kn log-uniform in [0.05, 10] and lid speed uniform in
    [0.05, 0.5] on the given spatial / velocity grid sizes."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        kn = float(10 ** rng.uniform(math.log10(0.05), 1.0))
        lid = float(rng.uniform(0.05, 0.5))
        N = int(rng.choice(sizes))
        M = int(rng.choice(vsizes))
        out.append(cases.cavity(N, M, kn=kn, lid=lid, name=f"{name}_{k}"))
    return out


def training_cases(n=256, seed=1810_00348):
    return sample_cases(n, seed, sizes=list(range(24, 49, 4)), vsizes=[16, 18, 20, 22, 24], name="train")


def heldout_cases(n=32, seed=1810_00348 + 1):
    return sample_cases(n, seed, sizes=[25, 27, 29, 31, 33, 37, 41, 45, 47], vsizes=[17, 19, 21, 23],
                        name="heldout")


def solve(case: cases.Case, tol: float = 1e-6, max_iters: int = 4000, init=None, precision="f64"):
    """Solve with the HIP solver from the uniform start (or init = (rho, u, T)
    with the uniform start's mass); returns iterations, wall seconds,
    converged flag and the fields."""
    from .solver import Solver
    s = Solver(case, precision=precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if init is None:
        s.init_uniform()
    else:
        rho, u, T = init
        s.init_fields(rho, u, T, target_mass=1.0)
    n, r, ok = s.iterate(max_iters, tol=tol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"iters": n, "seconds": dt, "converged": ok, "residual": r, "fields": s.fields()}


def predict(net: WarmStartNet, case: cases.Case, chan_std: np.ndarray):
    """Predicted (rho, u[3], T) on the case's grid (flat, cell order)."""
    nx, ny, nz = case.n
    x = torch.from_numpy(features(case)).to(net.device)
    y = net.forward(x.contiguous()).cpu().numpy()[:nz, :ny, :nx]
    y = y * chan_std[None, None, None, :] * target_scale(case)
    rho = 1.0 + y[..., 0].reshape(-1).astype(np.float64)
    u = np.stack([y[..., 1 + d].reshape(-1) for d in range(3)]).astype(np.float64)
    T = 1.0 + y[..., 4].reshape(-1).astype(np.float64)
    return rho, u, T


def warm_started_solve(net: WarmStartNet, case: cases.Case, chan_std: np.ndarray, tol=1e-6,
                       max_iters=4000):
    """Predict, seed, solve; falls back to the uniform start if the prediction
    is not a physical state or the seeded solve fails."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rho, u, T = predict(net, case, chan_std)
    t_pred = time.perf_counter() - t0
    ok = bool(np.all(np.isfinite(rho)) and np.all(np.isfinite(u)) and np.all(np.isfinite(T))
              and rho.min() > 0 and T.min() > 0)
    res = None
    if ok:
        try:
            res = solve(case, tol, max_iters, init=(rho, u, T))
        except (L.DvmError, FloatingPointError):
            res = None
    fallback = res is None or not res["converged"]
    if fallback:
        res = solve(case, tol, max_iters)
    res["seconds"] += t_pred
    res["predict_seconds"] = t_pred
    res["fallback"] = fallback
    return res


def train(net: WarmStartNet, data, chan_std, epochs: int, lr: float, batch: int = 4, seed: int = 0,
          log=None):
    """Adam on the masked MSE of normalised targets, minibatches of whole
    grids (gradients accumulated over the batch)."""
    rng = np.random.default_rng(seed)
    dev = net.device
    prepared = []
    for case, fields in data:
        x = torch.from_numpy(features(case)).to(dev).contiguous()
        t, m = targets(case, fields, chan_std)
        prepared.append((x, torch.from_numpy(t).to(dev).contiguous(), torch.from_numpy(m).to(dev).contiguous()))
    history = []
    for ep in range(epochs):
        order = rng.permutation(len(prepared))
        tot = 0.0
        for b0 in range(0, len(order), batch):
            idx = order[b0:b0 + batch]
            net.zero_grad()
            for k in idx:
                x, t, m = prepared[k]
                net.forward(x)
                tot += net.backward_mse(t, m, 1.0 / len(idx))
            net.adam_step(lr)
        history.append(tot / max(1, math.ceil(len(order) / batch)))
        if log:
            log(f"epoch {ep} loss {history[-1]:.5f}")
    return history
