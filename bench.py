"""Benchmark: phase-space point-updates per second of one outer iteration.

One step = one full outer iteration of the HIP path (per-cell parameters, the
upwind sweep of every discrete velocity with the on-the-fly equilibrium, the
moment reduction, finalisation, mass rescaling and the residual read-back) on
the 3D lid-driven cavity with 64^3 cells and 32^3 discrete velocities on
[-5,5]^3, Kn = 1, lid speed 0.16, FP64 -- synthetic input, resident in HBM.

Prints ONE JSON line (rank 0).  Besides the throughput it carries, for the
default workload, the metric's second half: iterations and wall time to
residual 1e-6 from the uniform start in FP64, in FP32 storage followed by
FP64, and both from the learned warm start (``time_to_residual``); the
roofline object adds the whole-iteration fraction and a plain device copy's
bandwidth as the practical ceiling; ``cpu_baseline`` names the host CPU and
the per-core rate.  Options:
  --gpus N      only N = 1 is supported (this build targets one GPU)
  --steps K     timed iterations (default 10)
  --warmup W    untimed iterations first (default 2)
  --workload    c2 (default), c3 (FP32 storage form) or c4 (cube, FP32)
  --precision   override f64/f32
  --no-cpu      skip the CPU oracle baseline
  --no-ttr      skip the time-to-residual runs
  --traffic F   JSON file with measured HBM bytes per sweep launch (from
                rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, calibrated)
  --time-to-residual
                instead of the throughput line: iterations and wall time to
                residual 1e-6 from the uniform start, FP64 storage, and FP32
                storage until its noise floor then FP64 from that state, with
                the per-field difference of the two converged solutions (one
                JSON line per workload)
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak figures of one MI355X (vendor): HBM3E 8 TB/s; FP64 vector 78.6 TFLOP/s
# (256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz).
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
# algorithmic work of one point-update of the sweep: one write of f^{n+1} and
# one read of the upwind operand (2 s bytes, s = bytes of the storage type),
# ~65 flops (equilibrium on the fly with separable Gaussian factors ~25,
# relaxation update ~14, 13 FP64 moment sums ~26)
FLOPS_PER_POINT = 65.0
KERNEL_SRC = os.path.join(ROOT, "paper_1810_00348_amd", "csrc", "dvm_kernels.hip")
TRAFFIC_DIR = os.path.join(ROOT, "profiles")


def kernel_sha() -> str:
    """Hash of the sweep kernel's code: the wave reduction, the sweep bodies
    and kernels (up to the list of instantiated variants) and the shared
    layout header, without comments and blank space; a measured traffic
    file is used only while this matches."""
    src = open(KERNEL_SRC).read()
    a = src.index("// Wave-level reduction of 13 FP64 values")
    b = src.index("#define DVM_SWEEP_VARIANTS")
    hdr = open(os.path.join(os.path.dirname(KERNEL_SRC), "dvm_internal.h")).read()
    code = re.sub(r"//[^\n]*", "", hdr + src[a:b])
    code = " ".join(code.split())
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def _pmc_sum(path: str, counter: str, kernel_substr: str):
    """Sum of a counter over the dispatches of one kernel, and their count."""
    tot, n = 0.0, 0
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter and kernel_substr in r["Kernel_Name"]:
                tot += float(r["Counter_Value"])
                n += 1
    return tot, n


def summarize_pmc(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, out, label):
    """Calibrated HBM bytes per sweep launch from rocprofv3 --pmc runs."""
    cf, _ = _pmc_sum(copy_fetch_csv, "FETCH_SIZE", "copyBuffer")
    cw, _ = _pmc_sum(copy_write_csv, "WRITE_SIZE", "copyBuffer")
    ffac = copy_bytes / (cf * 1024.0)
    wfac = copy_bytes / (cw * 1024.0)
    f, nf = _pmc_sum(fetch_csv, "FETCH_SIZE", "sweep_kernel")
    w, nw = _pmc_sum(write_csv, "WRITE_SIZE", "sweep_kernel")
    rec = {
        "kernel_source_sha256_16": kernel_sha(),
        "label": label,
        "launches": nf,
        "fetch_kib_total": f, "write_kib_total": w,
        "fetch_factor": round(ffac, 4), "write_factor": round(wfac, 4),
        "bytes_per_launch": (f * 1024.0 * ffac + w * 1024.0 * wfac) / max(1, nf),
        "read_bytes_per_launch": f * 1024.0 * ffac / max(1, nf),
        "write_bytes_per_launch": w * 1024.0 * wfac / max(1, nw),
        "commands": [
            "cd /tmp && export TMPDIR=/tmp",
            "timeout -s KILL 100 rocprofv3 --pmc FETCH_SIZE --output-format csv -d $R/gpurun_out/pmc/f -o f "
            "-- python3 $R/bench.py --workload W --steps 1 --warmup 0 --no-cpu",
            "timeout -s KILL 100 rocprofv3 --pmc WRITE_SIZE --output-format csv -d $R/gpurun_out/pmc/w -o w "
            "-- python3 $R/bench.py --workload W --steps 1 --warmup 0 --no-cpu",
            "timeout -s KILL 60 rocprofv3 --pmc FETCH_SIZE --output-format csv -d $R/gpurun_out/pmc/cf -o cf "
            "-- python3 $R/bench.py --copy-calib 4   (and WRITE_SIZE into .../cw)",
            "python bench.py --summarize-pmc <f csv> <w csv> <cf csv> <cw csv> 4294967296 LABEL",
        ],
        "note": "R = repository root; W = the workload of LABEL (one iteration = launches sweep launches); "
                "factors = bytes of a 4 GiB device copy / counter KiB x 1024",
    }
    with open(out, "w") as fo:
        json.dump(rec, fo, indent=1)
    print(json.dumps(rec))


def summarize_trace(db_path: str, out_md: str, title: str, command: str, bench_json: str = ""):
    """Kernel-trace summary (markdown) from a rocprofv3 --kernel-trace
    database: per kernel the calls, total, average, min and max duration,
    and for the sweep kernels the wall time their launches cover (the union
    of the launch intervals: launches on several streams overlap, so the
    sum of their durations exceeds the sweep phase's wall time)."""
    import sqlite3
    con = sqlite3.connect(db_path)
    rows = con.execute("select name, start, end from kernels").fetchall()
    con.close()
    by = {}
    for name, t0, t1 in rows:
        by.setdefault(name, []).append((t0, t1))
    total = sum(t1 - t0 for v in by.values() for t0, t1 in v)
    lines = [f"# Kernel stats: {title}", "", "Command (run from the repository root on one MI355X; output directory "
             "under gpurun_out/):", "", "```", command, "```", "",
             "| kernel | calls | total ms | avg us | % | min us | max us |", "|---|---|---|---|---|---|---|"]
    for name, v in sorted(by.items(), key=lambda kv: -sum(t1 - t0 for t0, t1 in kv[1])):
        d = [(t1 - t0) / 1e3 for t0, t1 in v]
        short = name if len(name) <= 80 else name[:77] + "..."
        lines.append(f"| `{short}` | {len(d)} | {sum(d) / 1e3:.3f} | {sum(d) / len(d):.1f} | "
                     f"{100.0 * sum(d) * 1e3 / total:.2f} | {min(d):.1f} | {max(d):.1f} |")
    sw = sorted(iv for name, v in by.items() if "sweep_kernel" in name for iv in v)
    if sw:
        busy, cur0, cur1 = 0, None, None
        for t0, t1 in sw:
            if cur1 is None or t0 > cur1:
                if cur1 is not None:
                    busy += cur1 - cur0
                cur0, cur1 = t0, t1
            else:
                cur1 = max(cur1, t1)
        busy += cur1 - cur0
        summed = sum(t1 - t0 for t0, t1 in sw)
        lines += ["", f"Sweep launches: {len(sw)}; summed duration {summed / 1e6:.3f} ms; wall time covered by "
                  f"them (union of the launch intervals) {busy / 1e6:.3f} ms; launches in flight on average "
                  f"{summed / busy:.2f}."]
    if bench_json:
        with open(bench_json) as f:
            d = json.loads(f.read().strip().splitlines()[-1])
        iters = d["steps"]
        lines += ["", f"The bench line printed by the same profiled command: {d['value']} GPt/s, "
                  f"{d['ms_per_step']} ms per iteration, sweep phase {d['config']['phase_ms']['sweep']} ms per "
                  f"iteration by HIP events over the {iters} timed iterations (the trace above also holds the "
                  f"{d['warmup']} warm-up iterations and the 3 iterations of the per-launch timing pass)."]
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def measured_traffic(label: str):
    """Bytes per sweep launch from the committed counter summary, if it was
    taken on the current kernel source and the same workload/schedule."""
    path = os.path.join(TRAFFIC_DIR, f"sweep_traffic_{label}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256_16") != kernel_sha():
        return None
    return rec.get("bytes_per_launch")


def workload(name: str, kn: float):
    from paper_1810_00348_amd import cases
    if name == "c2":
        return cases.config("c2", kn=kn), "f64"
    if name == "c3":
        return cases.config("c3"), "f32"
    if name == "c4":
        return cases.config("c4"), "f32"
    if name == "c6":
        return cases.config("c6"), "f32"
    raise SystemExit(f"unknown workload {name}")


def describe(name: str, case) -> str:
    grid = f"{case.n[0]}x{case.n[1]}x{case.n[2]}"
    vel = f"{case.m[0]}^3 velocities on [-{case.vmax[0]:g},{case.vmax[0]:g}]^3"
    if name == "c4":
        return f"{case.name}: cube half-domain {grid} cells x {vel}, Ma 5, Kn 0.1"
    if name == "c6":
        return (f"{case.name}: full-domain cube of the paper's Sec. 4.2, {grid} stretched cells x {vel}, "
                f"Ma 2, Kn 1 ({case.points:.3g} points)")
    return f"{case.name}: lid-driven cavity {grid} cells x {vel}, Kn={case.kn:g}, lid {case.faces[3].u[0]:g}"


def cpu_baseline(case, budget_s: float = 25.0):
    """The FP64 oracle, as it stands, for one outer iteration on a bounded
    sample of the workload: the same spatial grid with a reduced velocity grid
    (the oracle's cost is linear in the number of phase-space points)."""
    from oracle import oracle as O
    from paper_1810_00348_amd import cases
    import dataclasses
    O.build(force=False)
    m = 16
    sample = dataclasses.replace(case, m=(m, m, m), name=case.name + f"_sample_v{m}")
    o = O.Oracle(sample)
    o.init_uniform()
    t0 = time.perf_counter()
    o.iterate(1)
    dt = time.perf_counter() - t0
    pts = sample.points
    model, nproc, avail = host_cpu()
    return {
        "value": pts / dt / 1e9,
        "unit": "GPt/s",
        "cores": o.threads,
        "kind": "oracle",
        "per_core_value": pts / dt / 1e9 / max(1, o.threads),
        "cpu_model": model,
        "nproc": nproc,
        "cpus_available": avail,
        "sample": f"one FP64 oracle iteration on {sample.n[0]}x{sample.n[1]}x{sample.n[2]} cells x "
                  f"{m}^3 velocities ({pts:.3g} points, {dt:.1f} s)",
    }


def solve(case, prec, max_iters, tol, desc):
    """Iterate from the uniform start, printing the residual of every
    iteration; one JSON line with the totals and a few field values."""
    import numpy as np
    import torch
    from paper_1810_00348_amd.solver import Solver
    t0 = time.perf_counter()
    s = Solver(case, precision=prec)
    s.init_uniform()
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    hist = []
    t1 = time.perf_counter()
    for it in range(1, max_iters + 1):
        _, r, _ = s.iterate(1)
        hist.append(r)
        print(f"iter {it} residual {r:.4e} elapsed {time.perf_counter() - t1:.2f} s", file=sys.stderr, flush=True)
        if tol > 0 and r <= tol:
            break
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    f = s.fields()
    nx, ny, nz = case.n
    rho = f["rho"].reshape(nz, ny, nx)
    T = f["T"].reshape(nz, ny, nx)
    fluid = ~case.solid.astype(bool) if case.solid is not None else np.ones_like(rho, bool)
    out = {"workload": desc, "precision": prec, "velocity_groups": s.info()["velocity_groups"],
           "workspace_GiB": round(s.info()["workspace_bytes"] / 2 ** 30, 1),
           "setup_seconds": round(t_setup, 2), "iterations": len(hist), "seconds": round(dt, 2),
           "s_per_iter": round(dt / len(hist), 4), "GPt_per_s": round(case.points * len(hist) / dt / 1e9, 1),
           "residual_history": [float(f"{x:.4e}") for x in hist],
           "fields": {"rho_max": float(rho[fluid].max()), "T_max": float(T[fluid].max()),
                      "rho_min": float(rho[fluid].min())}}
    print(json.dumps(out), flush=True)


def warmstart_kernels(n, steps, warmup):
    """The warm-start U-Net's BF16 MFMA convolutions against the dense BF16
    peak: algorithmic FLOPs 2 * voxels * taps * c_in * c_out per convolution
    (levels n^3, (n/2)^3, (n/4)^3), forward alone and one training step
    (forward, input and weight gradients: three times the forward FLOPs)."""
    import numpy as np
    import torch
    from paper_1810_00348_amd import warmstart as W
    net = W.WarmStartNet(max_grid=(n, n, n))
    net.set_params(W.init_theta(7))
    level = {"e1a": 0, "e1b": 0, "e2a": 1, "e2b": 1, "b1": 2, "b2": 2, "d2a": 1, "d2b": 1, "d1a": 0,
             "d1b": 0, "out": 0}
    fl = sum(2.0 * (n ** 3 / 8 ** level[name]) * taps * ci * co for name, ci, co, taps, _ in W.layer_table())
    rng = np.random.default_rng(0)
    x = torch.from_numpy(rng.standard_normal((n, n, n, W.NET_IN)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.standard_normal((n, n, n, W.NET_OUT)).astype(np.float32)).cuda()
    m = torch.ones((n, n, n), dtype=torch.float32, device="cuda")

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    def train():
        net.zero_grad()
        net.forward(x)
        net.backward_mse(t, m)
        net.adam_step(1e-4)

    tf = timed(lambda: net.forward(x))
    tt = timed(train)
    out = {"metric": "warm-start U-Net BF16 MFMA throughput", "grid": n, "steps": steps,
           "forward_ms": round(tf * 1e3, 3), "train_step_ms": round(tt * 1e3, 3),
           "forward_gflop": round(fl / 1e9, 2),
           "roofline": {"bound": "mfma", "unit": "TFLOP/s", "peak": 2500.0,
                        "achieved_forward": round(fl / tf / 1e12, 2), "achieved_train": round(3 * fl / tt / 1e12, 2),
                        "frac_forward": round(fl / tf / 1e12 / 2500.0, 4),
                        "frac_train": round(3 * fl / tt / 1e12 / 2500.0, 4)}}
    print(json.dumps(out), flush=True)


def time_to_residual_row(name, case, net, chan_std, tol=1e-6, max_iters=3000):
    """Wall time to the residual tolerance from the uniform start (the full
    dvm_iterate loop including its per-iteration residual read-back): FP64
    storage, and FP32 storage until its noise floor followed by FP64 from the
    same state; per-field max |x - x64| / max |x64| of the two solutions.
    Then both again from the learned warm start (the committed network's
    prediction, its time included)."""
    import numpy as np
    import torch
    from paper_1810_00348_amd import warmstart as W
    from paper_1810_00348_amd.solver import Solver, solve_fp32_then_fp64

    def field_diff(a, b):
        return {key: float(f"{np.abs(x - y).max() / max(np.abs(y).max(), 1e-300):.3e}")
                for key, x, y in (("rho", a["rho"], b["rho"]), ("ux", a["u"][0], b["u"][0]),
                                  ("uy", a["u"][1], b["u"][1]), ("uz", a["u"][2], b["u"][2]),
                                  ("T", a["T"], b["T"]))}

    row = {"workload": name, "case": case.name, "points_per_iteration": case.points, "tol": tol}
    s = Solver(case, precision="f64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.init_uniform()
    it, r, ok = s.iterate(max_iters, tol=tol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    f64 = s.fields()
    row["f64"] = {"iters": it, "seconds": round(dt, 3), "converged": ok, "residual": r,
                  "ms_per_iter": round(dt * 1e3 / max(it, 1), 3)}
    del s
    torch.cuda.empty_cache()
    m = solve_fp32_then_fp64(case, tol, max_iters)
    row["f32_then_f64"] = {k: (round(v, 3) if isinstance(v, float) and k.endswith("seconds") else v)
                           for k, v in m.items() if k != "fields"}
    row["mixed_vs_f64_converged"] = field_diff(m["fields"], f64)
    row["speedup_time_to_residual"] = round(row["f64"]["seconds"] / m["seconds"], 3)
    torch.cuda.empty_cache()
    # learned warm start: FP64, and FP32 then FP64
    w = W.warm_started_solve(net, case, chan_std, tol=tol, max_iters=max_iters)
    row["warm_f64"] = {"iters": w["iters"], "seconds": round(w["seconds"], 3), "converged": w["converged"],
                       "fallback": w["fallback"]}
    row["warm_f64_vs_f64_converged"] = field_diff(w["fields"], f64)
    row["speedup_warm_f64"] = round(row["f64"]["seconds"] / w["seconds"], 3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred = W.predict(net, case, chan_std)
    t_pred = time.perf_counter() - t0
    mw = solve_fp32_then_fp64(case, tol, max_iters, init=pred, target_mass=1.0)
    row["warm_f32_then_f64"] = {"iters": mw["iters"], "f32_iters": mw["f32_iters"], "f64_iters": mw["f64_iters"],
                                "seconds": round(mw["seconds"] + t_pred, 3), "converged": mw["converged"]}
    row["warm_mixed_vs_f64_converged"] = field_diff(mw["fields"], f64)
    row["speedup_warm_mixed"] = round(row["f64"]["seconds"] / row["warm_f32_then_f64"]["seconds"], 3)
    torch.cuda.empty_cache()
    return row


def load_warmstart_net(big):
    from paper_1810_00348_amd import warmstart as W
    theta, chan_std, _ = W.load_weights(os.path.join(os.path.dirname(W.__file__), "data", "warmstart_unet.npz"))
    net = W.WarmStartNet(max_grid=(big, big, big))
    net.set_params(theta)
    return net, chan_std


def time_to_residual(workloads, tol=1e-6, max_iters=3000):
    """One JSON line per workload (see time_to_residual_row)."""
    big = max(max(case.n) for _, case in workloads)
    net, chan_std = load_warmstart_net(big)
    for name, case in workloads:
        print(json.dumps(time_to_residual_row(name, case, net, chan_std, tol, max_iters)), flush=True)


def precision_error(name, case, checkpoints=(1, 5, 20), floor_iters=60, tol=1e-6, parameter_bits=0):
    """The FP32 storage form against the FP64 path on the same inputs: both
    from the uniform start, per-field max |x32 - x64| / max |x64| (rho, U_x,
    U_y, U_z, T, q_x, q_y, q_z) after each checkpoint iteration count; then
    FP64 to the tolerance and FP32 for floor_iters iterations (its residual
    stalls at its floor), and the same errors between those two states."""
    import numpy as np
    import torch
    from paper_1810_00348_amd.solver import Solver

    def errors(a, b):
        out = {}
        for key in ("rho", "T"):
            out[key] = float(f"{np.abs(a[key] - b[key]).max() / np.abs(b[key]).max():.3e}")
        for vec, names in (("u", ("ux", "uy", "uz")), ("q", ("qx", "qy", "qz"))):
            big = np.abs(b[vec]).max()
            for d, k in enumerate(names):
                den = max(np.abs(b[vec][d]).max(), 1e-3 * big, 1e-300)
                out[k] = float(f"{np.abs(a[vec][d] - b[vec][d]).max() / den:.3e}")
        return out

    row = {"workload": name, "case": case.name, "checkpoints": {}, "parameter_bits": parameter_bits or 32}
    s64 = Solver(case, precision="f64")
    s32 = Solver(case, precision="f32", parameter_bits=parameter_bits)
    s64.init_uniform()
    s32.init_uniform()
    done = 0
    for k in checkpoints:
        s64.iterate(k - done)
        s32.iterate(k - done)
        done = k
        row["checkpoints"][str(k)] = errors(s32.fields(), s64.fields())
    it64, r64, ok64 = s64.iterate(3000, tol=tol)
    hist = []
    for _ in range(max(0, floor_iters - done)):
        _, r, _ = s32.iterate(1)
        hist.append(r)
    row["f64_converged"] = {"iters": done + it64, "residual": r64, "converged": ok64}
    row["f32_floor"] = {"iters": floor_iters, "residual_last": hist[-1] if hist else None,
                        "residual_min": min(hist) if hist else None,
                        "residual_last10_max": max(hist[-10:]) if hist else None}
    row["f32_floor_vs_f64_converged"] = errors(s32.fields(), s64.fields())
    del s64, s32
    torch.cuda.empty_cache()
    return row


def copy_bandwidth(gib: float = 4.0, reps: int = 5):
    """Achievable HBM bandwidth on this device: a plain device-to-device copy
    of gib GiB (read + write counted), best of reps, timed with HIP events."""
    import torch
    n = int(gib * 2 ** 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * n * 8 / (best / 1e3) / 1e9


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--kn", type=float, default=1.0)
    ap.add_argument("--precision", default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--body", default=None, choices=("plain", "pf", "dyn"),
                    help="sweep body in place of the library's choice: plain, software-pipelined (pf) "
                         "or pipelined in one dependency-driven launch (dyn)")
    ap.add_argument("--brick", default=None, metavar="VL,BX,BY,BZ",
                    help="sweep schedule in place of the library's choice: velocities per lane and brick cells "
                         "(0 keeps that value)")
    ap.add_argument("--streams", type=int, default=0, choices=(0, 1, 2, 4, 8),
                    help="streams for the per-diagonal sweep launches (0: the library's default)")
    ap.add_argument("--param-bits", type=int, default=0, choices=(0, 32, 64),
                    help="FP32 storage: per-cell parameters and equilibrium evaluation in FP64 (64)")
    ap.add_argument("--precision-error", action="store_true",
                    help="instead of the throughput line: per-field error of the FP32 storage form against "
                         "FP64 on the same inputs (after 1, 5, 20 iterations and at the FP32 floor)")
    ap.add_argument("--floor-iters", type=int, default=60,
                    help="--precision-error: FP32 iterations run to reach its residual floor")
    ap.add_argument("--no-ttr", action="store_true",
                    help="skip the time-to-residual runs of the default line (64^3 x 32^3 cavity, Kn 1)")
    ap.add_argument("--traffic", default=None)
    ap.add_argument("--time-to-residual", action="store_true")
    ap.add_argument("--solve", type=int, default=0, metavar="ITERS",
                    help="solve the workload from the uniform start for up to ITERS iterations "
                         "(or to --tol), one progress line per iteration")
    ap.add_argument("--tol", type=float, default=0.0)
    ap.add_argument("--warmstart", type=int, default=0, metavar="GRID",
                    help="time the warm-start U-Net (forward, and one training step) on a GRID^3 grid")
    ap.add_argument("--model", default="shakhov", choices=("shakhov", "esbgk"),
                    help="collision model (esbgk: the ellipsoidal statistical BGK model)")
    ap.add_argument("--order", type=int, default=1, choices=(1, 2),
                    help="spatial order of the upwind sweep (2: the second-order extension)")
    ap.add_argument("--stretch", type=float, default=0.0,
                    help="run the workload on a mesh stretched geometrically by this ratio per cell")
    ap.add_argument("--copy-calib", type=float, default=0.0,
                    help="only run a plain device copy of this many GiB (counter calibration)")
    ap.add_argument("--summarize-trace", nargs=4, default=None, metavar=("DB", "NAME", "TITLE", "BENCH_JSON"),
                    help="write profiles/NAME.md from a rocprofv3 --kernel-trace database")
    ap.add_argument("--summarize-pmc", nargs=6, default=None,
                    metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV", "COPY_BYTES", "LABEL"),
                    help="write profiles/sweep_traffic_LABEL.json from rocprofv3 --pmc CSVs")
    args = ap.parse_args()
    if args.summarize_trace:
        db, name, title, bj = args.summarize_trace
        cmd = ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats -d $REPO/gpurun_out/prof/W -o W "
               "-- python3 $REPO/bench.py --workload W --steps 10 --warmup 2 --no-cpu --no-ttr")
        summarize_trace(db, os.path.join(TRAFFIC_DIR, name + ".md"), title, cmd, bj)
        return
    if args.summarize_pmc:
        a = args.summarize_pmc
        summarize_pmc(a[0], a[1], a[2], a[3], float(a[4]),
                      os.path.join(TRAFFIC_DIR, f"sweep_traffic_{a[5]}.json"), a[5])
        return
    if args.copy_calib > 0:
        import torch
        n = int(args.copy_calib * 2 ** 30) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 8}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (the sweep shards by velocity across "
              "GPUs by design, but no multi-GPU path is built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.warmstart > 0:
        warmstart_kernels(args.warmstart, args.steps, args.warmup)
        return

    if args.precision_error:
        case, _ = workload(args.workload, args.kn)
        print(json.dumps(precision_error(args.workload, case, floor_iters=args.floor_iters,
                                         parameter_bits=args.param_bits)), flush=True)
        return

    if args.time_to_residual:
        from paper_1810_00348_amd import cases
        wl = [(f"c2_kn{kn:g}", cases.config("c2", kn=kn)) for kn in (10.0, 1.0, 0.1)]
        wl.append(("c3", cases.config("c3")))
        time_to_residual(wl)
        return

    import torch
    from paper_1810_00348_amd.solver import Solver

    case, prec = workload(args.workload, args.kn)
    if args.precision:
        prec = args.precision
    if args.stretch > 0:
        from paper_1810_00348_amd import cases as _cases
        centres = (None, None, None) if args.workload != "c4" else (2.5, 3.0, None)
        case = _cases.stretched(case, args.stretch, centres)
    if args.order != 1 or args.model != "shakhov":
        import dataclasses as _dc
        tag = (f"_order{args.order}" if args.order != 1 else "") + ("_esbgk" if args.model != "shakhov" else "")
        case = _dc.replace(case, order=args.order, model=args.model, name=case.name + tag)
    if args.solve > 0:
        solve(case, prec, args.solve, args.tol, describe(args.workload, case))
        return
    sched = None if args.body is None else {"pipelined": {"plain": False, "pf": True, "dyn": "dyn"}[args.body]}
    if args.brick:
        vl, bx, by, bz = (int(x) for x in args.brick.split(","))
        sched = dict(sched or {}, vl=vl, bx=bx, by=by, bz=bz)
    s = Solver(case, precision=prec, schedule=sched, parameter_bits=args.param_bits, sweep_streams=args.streams)
    s.init_uniform()
    info = s.info()
    if args.warmup:
        s.iterate(args.warmup)
    s.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tm = s.timings()
    # per-launch durations, in a pass of their own after the timed steps
    # (an event pair around every sweep launch on its stream): the launches
    # of the sweep's streams overlap, so their average duration is longer
    # than the sweep phase's wall time divided by the launches
    s.set_timing(2)
    s.iterate(3)
    lt = s.launch_timings()
    lt_phase = s.timings()
    s.set_timing(0)

    ms = dt * 1e3 / args.steps
    pts = case.points
    value = pts / (ms / 1e3) / 1e9
    iters = max(1, tm["iterations"])
    sweep_ms = tm["sweep_ms"] / iters
    launches = info["sweep_launches"]
    sbytes = 8 if prec == "f64" else 4
    # dominant kernel: the sweep.  Algorithmic bytes per launch = points per
    # launch x 2 s; averaged over the launches of an iteration this is
    # (points x 2 s) / (sweep time of one iteration).
    achieved_gbs = pts * 2 * sbytes / (sweep_ms / 1e3) / 1e9
    label = f"{args.workload}_{prec}_vl{info['vel_per_lane']}_b{info['brick'][0]}x{info['brick'][1]}x{info['brick'][2]}"
    if args.stretch > 0:
        label += f"_stretch{args.stretch:g}"
    if args.order != 1:
        label += f"_order{args.order}"
    if args.model != "shakhov":
        label += f"_{args.model}"
    if info["sweep_kernel"] == "sweep_kernel_dyn":
        label += "_dyn"
    elif info["sweep_streams"] != 1:
        label += f"_s{info['sweep_streams']}"
    if prec == "f32" and info["parameter_bits"] == 64:
        label += "_p64"
    line = {
        "metric": "phase-space GPoint-updates/s per iteration",
        "value": round(value, 3),
        "unit": "GPt/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {
            "workload": describe(args.workload, case),
            "velocity_groups": info["velocity_groups"],
            "upwind_order": case.order,
            "model": case.model,
            "points_per_iteration": pts,
            "brick": info["brick"],
            "vel_per_lane": info["vel_per_lane"],
            "sweep_kernel": info["sweep_kernel"],
            "sweep_streams": info["sweep_streams"],
            "parameter_bits": info["parameter_bits"],
            "sweep_launches_per_iteration": launches,
            "phase_ms": {"params": round(tm["params_ms"] / iters, 4),
                         "sweep": round(sweep_ms, 4),
                         "finalize": round(tm["finalize_ms"] / iters, 4)},
            "residual_after": s.residual(),
            "paper_context": "K40, FP32, 64^3 x 32^3 cavity: 4.33 s/iteration = 1.98 GPt/s "
                             "(Table iteration_time); 190x over one Xeon core",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved_gbs, 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(achieved_gbs / PEAK_HBM_GBS, 4),
            "traffic": measured_traffic(label),
            "kernel": info["sweep_kernel"],
            "bytes_per_point": 2 * sbytes,
            "launches_per_step": launches,
            # HIP events around every launch (agrees with the kernel
            # trace's average), the algorithmic rate of one launch over
            # its own duration, and how many launches run at once
            "avg_launch_ms": round(lt["launch_ms_total"] / max(1, lt["launches"]), 5),
            "achieved_per_launch": round(pts * 2 * sbytes / launches
                                         / (lt["launch_ms_total"] / max(1, lt["launches"]) / 1e3) / 1e9, 1),
            "launches_in_flight": round(lt["launch_ms_total"] / max(1e-9, lt_phase["sweep_ms"]), 3),
            "alu_view": {"flops_per_point": FLOPS_PER_POINT,
                         "achieved_tflops": round(pts * FLOPS_PER_POINT / (sweep_ms / 1e3) / 1e12, 3),
                         "peak_tflops_fp64": PEAK_FP64_TFLOPS},
            "traffic_label": label,
        },
    }
    # the whole iteration (parameters, sweep, finalisation, residual
    # read-back) at the same algorithmic bytes, and a plain copy's rate on
    # this device as the practical ceiling beside the vendor peak
    step_gbs = pts * 2 * sbytes / (ms / 1e3) / 1e9
    line["roofline"]["achieved_step"] = round(step_gbs, 1)
    line["roofline"]["frac_step"] = round(step_gbs / PEAK_HBM_GBS, 4)
    del s
    torch.cuda.empty_cache()
    cgbs = copy_bandwidth()
    line["roofline"]["copy_gbs"] = round(cgbs, 1)
    line["roofline"]["frac_of_copy"] = round(achieved_gbs / cgbs, 4)
    # the measured HBM bytes per launch over the live launch time, against
    # the same peak (the third figure of the roofline: what the memory
    # system actually moved, beside the algorithmic rate above)
    tr = line["roofline"]["traffic"]
    if tr is not None and sweep_ms > 0:
        gbs = tr * launches / (sweep_ms / 1e3) / 1e9
        line["roofline"]["traffic_gbs"] = round(gbs, 1)
        line["roofline"]["traffic_frac"] = round(gbs / PEAK_HBM_GBS, 4)
    plain = args.stretch == 0 and args.order == 1 and args.model == "shakhov" and args.precision is None
    if args.workload == "c2" and args.kn == 1.0 and plain and not args.no_ttr:
        # the metric's second half: time to residual 1e-6 from the uniform
        # start, FP64 against FP32-then-FP64 and the learned warm start
        net, chan_std = load_warmstart_net(max(case.n))
        line["time_to_residual"] = time_to_residual_row("c2_kn1", case, net, chan_std)
        del net
        torch.cuda.empty_cache()
    if not args.no_cpu and args.workload != "c6":
        line["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
