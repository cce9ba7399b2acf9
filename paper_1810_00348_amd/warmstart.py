"""Learned warm start of the iterative DVM solver.

A 3D U-Net (include/wsn.h, HIP/MFMA kernels in csrc/wsn.hip) maps the inputs
(log10 Kn, lid speed, and the wall geometry: a wall mask and each cell's
position relative to the walls) on the cell grid of a lid-driven cavity to
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

NET_IN, NET_OUT, NET_BASE = 6, 5, 32
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
            "wsn_train_step": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_float,
                                C.POINTER(C.c_double)], C.c_int),
            "wsn_save": ([C.c_void_p, C.c_char_p], C.c_int),
            "wsn_load": ([C.c_void_p, C.c_char_p], C.c_int),
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
            try:
                wsn_lib().wsn_destroy(h)
            except Exception:  # interpreter shutdown: module state already torn down
                pass
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

    def train_step(self, batch, lr: float) -> float:
        """One step over ``batch`` = [(x, target, mask), ...] of device
        tensors (see wsn_train_step); returns the batch's mean loss."""
        n = len(batch)
        ins = (C.c_void_p * n)(*[_P(x) for x, _, _ in batch])
        tgs = (C.c_void_p * n)(*[_P(t) for _, t, _ in batch])
        mks = (C.c_void_p * n)(*[_P(m) for _, _, m in batch])
        dims = (C.c_int * (3 * n))(*[d for x, _, _ in batch for d in x.shape[:3]])
        loss = C.c_double(0.0)
        _chk(wsn_lib().wsn_train_step(self._h, n, ins, tgs, mks, dims, lr, C.byref(loss)))
        return loss.value

    def save(self, path: str):
        _chk(wsn_lib().wsn_save(self._h, path.encode()))

    def load(self, path: str):
        _chk(wsn_lib().wsn_load(self._h, path.encode()))


# ------------------------------------------------------------------ data

def pad4(n: int) -> int:
    return (n + 3) // 4 * 4


def features(case: cases.Case) -> np.ndarray:
    """[D, H, W, 6] network input on the grid padded to multiples of 4 (the
    padding cells are all zero): log10 Kn, lid speed, wall mask (1 next to the
    moving lid, 0.5 next to the other walls, 0 inside), and the cell centre's
    position (x, y, z) as a fraction of the cavity side -- the wall geometry
    seen from the cell, which the network's receptive field (about 40 cells)
    cannot always see itself."""
    nx, ny, nz = case.n
    D, H, W = pad4(nz), pad4(ny), pad4(nx)
    x = np.zeros((D, H, W, NET_IN), dtype=np.float32)
    lid = case.faces[3].u[0]
    x[:nz, :ny, :nx, 0] = math.log10(case.kn)
    x[:nz, :ny, :nx, 1] = lid
    m = np.zeros((nz, ny, nx), dtype=np.float32)
    m[0, :, :] = m[-1, :, :] = 0.5
    m[:, 0, :] = m[:, :, 0] = m[:, :, -1] = 0.5
    m[:, -1, :] = 1.0
    x[:nz, :ny, :nx, 2] = m
    x[:nz, :ny, :nx, 3] = ((np.arange(nx) + 0.5) / nx)[None, None, :]
    x[:nz, :ny, :nx, 4] = ((np.arange(ny) + 0.5) / ny)[None, :, None]
    x[:nz, :ny, :nx, 5] = ((np.arange(nz) + 0.5) / nz)[:, None, None]
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
    """Held-out cavities on uneven spatial grids.  The velocity grids are even:
    with an odd count a node sits at xi = 0, on the jump of the wall
    distribution in the wall-normal velocity, and the converged flow differs
    from the even-count one by tens of percent at these coarse grids (the two
    approach the limit from opposite sides) -- a property of the quadrature
    that the network's inputs do not carry."""
    return sample_cases(n, seed, sizes=[25, 27, 29, 31, 33, 37, 41, 45, 47], vsizes=[16, 18, 20, 22, 24],
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


def train(net: WarmStartNet, data, chan_std, epochs: int, lr, batch: int = 4, seed: int = 0,
          log=None, pad_jitter: int = 3, stop=None):
    """Adam on the masked MSE of normalised targets, minibatches of whole
    grids (gradients accumulated over the batch).  Each grid is placed at a
    random offset of 0..pad_jitter cells per axis inside a zero-padded grid
    with 0..pad_jitter more cells after it (then rounded up to a multiple of
    4), drawn afresh every epoch: odd-sized grids at inference put their walls
    at every alignment with the network's 2x2x2 pooling, and the network has
    to see those alignments in training.  lr: a number or a function of the
    epoch; stop(): optional early-stop test after an epoch."""
    rng = np.random.default_rng(seed)
    dev = net.device
    prepared = []
    for case, fields in data:
        nx, ny, nz = case.n
        x = torch.from_numpy(features(case)[:nz, :ny, :nx]).to(dev)
        t, _ = targets(case, fields, chan_std)
        prepared.append((case.n, x, torch.from_numpy(t[:nz, :ny, :nx]).to(dev)))
    history = []
    for ep in range(epochs):
        cur = lr(ep) if callable(lr) else lr
        order = rng.permutation(len(prepared))
        tot = 0.0
        for b0 in range(0, len(order), batch):
            idx = order[b0:b0 + batch]
            net.zero_grad()
            for k in idx:
                (nx, ny, nz), x0, t0 = prepared[k]
                oz, oy, ox = (int(rng.integers(0, pad_jitter + 1)) for _ in range(3))
                D, H, W = (pad4(n + o + int(rng.integers(0, pad_jitter + 1)))
                           for n, o in ((nz, oz), (ny, oy), (nx, ox)))
                x = torch.zeros((D, H, W, x0.shape[-1]), dtype=torch.float32, device=dev)
                t = torch.zeros((D, H, W, t0.shape[-1]), dtype=torch.float32, device=dev)
                m = torch.zeros((D, H, W), dtype=torch.float32, device=dev)
                x[oz:oz + nz, oy:oy + ny, ox:ox + nx] = x0
                t[oz:oz + nz, oy:oy + ny, ox:ox + nx] = t0
                m[oz:oz + nz, oy:oy + ny, ox:ox + nx] = 1.0
                net.forward(x)
                tot += net.backward_mse(t, m, 1.0 / len(idx))
            net.adam_step(cur)
        history.append(tot / max(1, math.ceil(len(order) / batch)))
        if log:
            log(f"epoch {ep} lr {cur:.2e} loss {history[-1]:.5f}")
        if stop is not None and stop():
            if log:
                log("stopping training early")
            break
    return history


# ------------------------------------------------------------------ pipeline

def generate(case_list, tol=1e-6, max_iters=4000, precision="f64", log=None):
    """Converged fields of every case from the plain uniform start."""
    out = []
    for k, c in enumerate(case_list):
        r = solve(c, tol, max_iters, precision=precision)
        out.append((c, r["fields"], {"iters": r["iters"], "seconds": r["seconds"], "converged": r["converged"]}))
        if log:
            log(f"gen {k} {c.name} n={c.n[0]} m={c.m[0]} kn={c.kn:.3f} lid={c.faces[3].u[0]:.3f} "
                f"iters={r['iters']} conv={r['converged']} {r['seconds']:.2f}s")
    return out


def channel_scale(data) -> np.ndarray:
    """RMS of the lid-normalised deviations over all training cells: one scale
    for rho, one shared by the three velocity components (so that the small
    spanwise component keeps its small weight in the loss), one for T."""
    acc = np.zeros(5)
    n = 0
    for case, fields in data:
        t, m = targets(case, fields, np.ones(5))
        sel = m > 0
        acc += (t[sel] ** 2).sum(axis=0)
        n += int(sel.sum())
    acc /= max(n, 1)
    acc[1:4] = acc[1:4].mean()
    return (np.sqrt(acc) + 1e-6).astype(np.float32)


def field_difference(a: Dict[str, np.ndarray], b: Dict[str, np.ndarray], norm: str = "max") -> Dict[str, float]:
    """Per macroscopic field: max_c |a - b| / max_c |b| (norm "max"), or for
    norm "dev" the L2 norm of a - b over the L2 norm of b's deviation from the
    rest state (rho - 1, u, T - 1): the error relative to what a solve has to
    build from the uniform start."""
    out = {}
    for key, x, y, ref in (("rho", a["rho"], b["rho"], 1.0), ("ux", a["u"][0], b["u"][0], 0.0),
                           ("uy", a["u"][1], b["u"][1], 0.0), ("uz", a["u"][2], b["u"][2], 0.0),
                           ("T", a["T"], b["T"], 1.0)):
        if norm == "max":
            out[key] = float(np.abs(x - y).max() / max(np.abs(y).max(), 1e-300))
        else:
            out[key] = float(np.linalg.norm(x - y) / max(np.linalg.norm(y - ref), 1e-300))
    return out


def evaluate(net, case_list, chan_std, tol=1e-6, max_iters=4000, log=None):
    """Plain and warm-started FP64 solves of every case, and (as the bound a
    perfect prediction could reach) a solve seeded with the plain solve's own
    converged rho, U, T."""
    rows = []
    for k, c in enumerate(case_list):
        plain = solve(c, tol, max_iters)
        warm = warm_started_solve(net, c, chan_std, tol, max_iters)
        exact = solve(c, tol, max_iters, init=(plain["fields"]["rho"], plain["fields"]["u"], plain["fields"]["T"]))
        rho, u, T = predict(net, c, chan_std)
        pred = {"rho": rho, "u": u, "T": T}
        row = {"case": c.name, "n": c.n[0], "m": c.m[0], "kn": c.kn, "lid": c.faces[3].u[0],
               "plain_iters": plain["iters"], "plain_s": plain["seconds"], "plain_converged": plain["converged"],
               "warm_iters": warm["iters"], "warm_s": warm["seconds"], "warm_converged": warm["converged"],
               "predict_s": warm["predict_seconds"], "fallback": warm["fallback"],
               "exact_seed_iters": exact["iters"],
               "final_diff": field_difference(warm["fields"], plain["fields"]),
               "prediction_error": field_difference(pred, plain["fields"]),
               "prediction_error_dev": field_difference(pred, plain["fields"], "dev")}
        rows.append(row)
        if log:
            log(f"eval {k} {c.name} kn={c.kn:.3f} lid={row['lid']:.3f} plain {plain['iters']} it "
                f"{plain['seconds']:.2f}s | warm {warm['iters']} it {warm['seconds']:.2f}s "
                f"fallback={warm['fallback']} | exact seed {exact['iters']} it | "
                f"pred err {max(row['prediction_error_dev'].values()):.2e} "
                f"diff={max(row['final_diff'].values()):.1e}")
    return rows


def store_params(theta: np.ndarray, specs) -> np.ndarray:
    """Weights rounded to BF16 (the precision the kernels use them in; biases
    stay FP32), so that the stored file compresses to the BF16 size."""
    out = np.array(theta, dtype=np.float32)
    off = 0
    for _, ci, co, taps, _ in specs:
        nw = taps * co * ci
        w = out[off:off + nw].view(np.uint32)
        w += np.uint32(0x7FFF) + ((w >> np.uint32(16)) & np.uint32(1))
        w &= np.uint32(0xFFFF0000)
        off += nw + co
    return out


def save_weights(path: str, theta: np.ndarray, chan_std: np.ndarray, meta: dict):
    import json
    np.savez_compressed(path, theta=theta, chan_std=chan_std.astype(np.float32),
                        meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))


def load_weights(path: str):
    import json
    with np.load(path, allow_pickle=False) as z:
        return z["theta"].astype(np.float32), z["chan_std"].astype(np.float32), json.loads(bytes(z["meta"]).decode())


def layer_table(base=NET_BASE, cin=NET_IN, cout=NET_OUT):
    """(name, c_in, c_out, taps, relu) per convolution, the order of the
    parameter vector of include/wsn.h."""
    b1, b2, b3 = base, 2 * base, 4 * base
    return [("e1a", cin, b1, 27, True), ("e1b", b1, b1, 27, True), ("e2a", b1, b2, 27, True),
            ("e2b", b2, b2, 27, True), ("b1", b2, b3, 27, True), ("b2", b3, b3, 27, True),
            ("d2a", b3 + b2, b2, 27, True), ("d2b", b2, b2, 27, True), ("d1a", b2 + b1, b1, 27, True),
            ("d1b", b1, b1, 27, True), ("out", b1, cout, 1, False)]


def init_theta(seed: int, base=NET_BASE, cin=NET_IN, cout=NET_OUT) -> np.ndarray:
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, ci, co, taps, relu in layer_table(base, cin, cout):
        std = math.sqrt((2.0 if relu else 1.0) / (taps * ci))
        parts.append((rng.standard_normal(taps * co * ci) * std).astype(np.float32))
        parts.append(np.zeros(co, np.float32))
    return np.concatenate(parts)


def pipeline(out_dir: str, n_train=256, n_eval=32, epochs=40, lr=1e-3, batch=4, tol=1e-6, max_iters=4000,
             time_budget_s=None, log=print):
    """Generate training solves, train the network on the GPU, evaluate the
    held-out cases; writes report.json and weights.npz into out_dir."""
    import json
    import os
    os.makedirs(out_dir, exist_ok=True)
    t_start = time.perf_counter()
    train_cases = training_cases(n_train)
    gen = generate(train_cases, tol, max_iters, log=log)
    t_gen = time.perf_counter() - t_start
    data = [(c, f) for c, f, s in gen if s["converged"]]
    chan_std = channel_scale(data)
    big = max(max(pad4(n + 6) for n in c.n) for c in train_cases + heldout_cases(n_eval))
    net = WarmStartNet(max_grid=(big, big, big))
    net.set_params(init_theta(seed=7))
    t0 = time.perf_counter()

    def lr_at(ep):
        # cosine decay of the learning rate
        return lr * 0.5 * (1 + math.cos(math.pi * ep / epochs))

    def over_budget():
        return bool(time_budget_s) and time.perf_counter() - t_start > time_budget_s

    history = train(net, data, chan_std, epochs, lr_at, batch, seed=1000,
                    log=lambda m: log(f"{m} ({time.perf_counter() - t0:.0f}s)"), stop=over_budget)
    t_train = time.perf_counter() - t0
    theta = store_params(net.params(), layer_table())
    net.set_params(theta)
    rows = evaluate(net, heldout_cases(n_eval), chan_std, tol, max_iters, log=log)
    meta = {"n_train": n_train, "converged_train": len(data), "epochs_run": len(history), "lr": lr,
            "batch": batch, "tol": tol, "seed_train": 1810_00348, "seed_eval": 1810_00348 + 1}
    save_weights(os.path.join(out_dir, "weights.npz"), theta, chan_std, meta)

    def tot(key):
        return float(sum(r[key] for r in rows))
    summary = {"plain_iters": tot("plain_iters"), "warm_iters": tot("warm_iters"),
               "exact_seed_iters": tot("exact_seed_iters"), "plain_s": tot("plain_s"),
               "warm_s": tot("warm_s"), "fallbacks": int(sum(r["fallback"] for r in rows)),
               "max_final_diff": max(max(r["final_diff"].values()) for r in rows),
               "median_iter_ratio": float(np.median([r["warm_iters"] / max(1, r["plain_iters"]) for r in rows]))}
    report = {"meta": meta, "gen": [{"case": c.name, "n": c.n[0], "m": c.m[0], "kn": c.kn,
                                     "lid": c.faces[3].u[0], **s} for c, f, s in gen],
              "gen_seconds": t_gen, "train_seconds": t_train, "loss_history": history,
              "chan_std": chan_std.tolist(), "eval": rows, "summary": summary}
    with open(os.path.join(out_dir, "report.json"), "w") as fh:
        json.dump(report, fh, indent=1)
    log(json.dumps(summary))
    return report


def main(argv=None):
    import argparse
    p = argparse.ArgumentParser(description="learned warm start: generate, train, evaluate")
    p.add_argument("--out", required=True)
    p.add_argument("--n-train", type=int, default=256)
    p.add_argument("--n-eval", type=int, default=32)
    p.add_argument("--epochs", type=int, default=40)
    p.add_argument("--lr", type=float, default=1e-3)
    p.add_argument("--batch", type=int, default=4)
    p.add_argument("--max-iters", type=int, default=4000)
    p.add_argument("--time-budget", type=float, default=None)
    a = p.parse_args(argv)

    def log(msg):
        print(msg, flush=True)
    pipeline(a.out, a.n_train, a.n_eval, a.epochs, a.lr, a.batch, 1e-6, a.max_iters, a.time_budget, log)


if __name__ == "__main__":
    main()
