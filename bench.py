"""Throughput of the backward sweep of the multistep BSDE scheme on one MI355X.

A "step" of this benchmark is one full backward solve (every time layer of
the sweep, every kernel of the hot path) of the workload below, with the
initial layers already resident in HBM.  The metric is
grid-point x time-step updates per second: n_x * N / (seconds per solve).

Default workload: the call under different lending and borrowing rates
(r = 0.01, R = 0.06, sigma = 0.2, mu = 0.05, K = S0 = 100, T = 0.5) on a
262144-point log-price grid, N = 1024 steps, k = 4, L = 16, Picard to 1e-14,
FP64.  The log-price interval is ln S0 +- 52, which keeps the Gauss-Hermite
spread at about 16 cells per unit (stability ratio 15.8).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_VALU_PEAK_TFLOPS = 78.6  # 256 CU x 64 FP64 FMA lanes x 2 flop x 2.4 GHz
HBM_PEAK_GBS = 8000.0


def workload(name: str):
    import workloads as W

    if name == "bidask1d":
        return W.bidask_call_1d(n_x=262144, n_t=1024, k=4, L=16, half_width=52.0,
                                picard_tol=1e-14, picard_max=30)
    if name == "bidask1d_literal":
        return W.bidask_call_1d(n_x=262144, n_t=1024, k=4, L=16, half_width=None,
                                picard_tol=1e-14, picard_max=30)
    if name == "sine1d":
        return W.sine_1d()
    if name in ("bs1d_exact", "bs1d_literal_exact"):
        # Black-Scholes call, 16384 points, N = 256, k = 4, exact Gaussian
        # expectations (the Toeplitz sweep on matrix cores); the stable twin
        # interval (stability ratio 16) or the literal ln S0 +- 6 sigma sqrt(T)
        nx, nt = 16384, 256
        hw = 0.2 * math.sqrt(2 * 0.33 / nt) / 16.0 * (nx - 1) / 2 if name == "bs1d_exact" else None
        wl = W.bs_call_1d(n_x=nx, n_t=nt, k=4, L=32, half_width=hw)
        wl.problem["quad"] = "exact"
        wl.name += "_exact"
        return wl
    raise SystemExit(f"unknown workload {name}")


def flops_per_point_step(pb: dict, picard_mean: float) -> float:
    """Algorithmic FP64 operations of one grid point and one time step.

    Per Gauss-Hermite node (j, l): two spline evaluations (4 mul + 3 add
    each), the driver, and three weighted accumulations (f, f dW, z: 2 each).
    Per layer j = K_y one more accumulation of y.  Then the z combination
    (3K + 1), the y constant (2K) and each Picard iteration (driver + 2).
    Driver cost: linear 4, bid-ask 8, cubic 5, exp 14 (exp counted as 1).
    """
    drv = {"linear": 4, "bidask": 8, "cubic": 5, "exp": 14}[pb["driver"]]
    K, L = max(pb["k_y"], pb["k_z"]), pb["L"]
    per_node = 7 + 7 + drv + 6
    return K * L * per_node + 2 * L + (3 * K + 1) + 2 * K + picard_mean * (drv + 2)


def bytes_per_point_step(pb: dict) -> float:
    """Algorithmic HBM bytes of the sweep kernel per point-step (FP64): read
    layers n+2..n+K whole (y, z and M_y, M_z: 32 B each) and the values of
    layer n+1 (16 B), write the values of layer n and the second derivatives
    of layer n+1 (16 B each)."""
    K = max(pb["k_y"], pb["k_z"])
    return 32.0 * (K - 1) + 16.0 + 32.0


# the sources of the 1-D sweep kernel, its launch and its workspace layout
KERNEL_SOURCES = ["capi.hip", "sweep.hip", "device_common.h", "kernels.h", "plan_math.cpp", "plan_math.h"]


def sources_sha1() -> str:
    """Hash of the library sources, to tie stored counter readings to a kernel version."""
    import hashlib

    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1909_13560_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload_name: str):
    """HBM bytes per sweep launch from the committed counter readings, or None
    when they were taken on other kernel sources or another workload."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("sources_sha1") != sources_sha1() or t.get("workload") != workload_name:
        return None
    return 1024.0 * (t["fetch_kib"] * t["read_factor"] + t["write_kib"] * t["write_factor"])


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def omp_threads() -> int:
    """Threads the OpenMP oracle uses: OMP_NUM_THREADS if set, else the cores
    this process may run on."""
    v = os.environ.get("OMP_NUM_THREADS", "")
    if v.isdigit() and int(v) > 0:
        return int(v)
    return len(os.sched_getaffinity(0))


def cpu_baseline(wl, budget_s: float = 15.0):
    """Serial oracle on the first steps of the same workload (bounded sample),
    and the same sample on all cores (the OpenMP build of the same source).
    Returns the report and the oracle's layer at the sample's last step
    (n_stop, y, z) for the full-size parity check."""
    import oracle

    oracle.build(force=False)
    pb = dict(wl.problem)
    K = wl.K
    iy, iz = wl.init_layers()
    # probe one step, then size the sample to the budget
    t0 = time.perf_counter()
    oracle.solve(pb, iy, iz, n_stop=pb["n_t"] - K)
    one = time.perf_counter() - t0
    steps = max(1, min(pb["n_t"] - K + 1, int(budget_s / max(one, 1e-3))))
    n_stop = pb["n_t"] - K + 1 - steps
    t0 = time.perf_counter()
    yo, zo, _ = oracle.solve(pb, iy, iz, n_stop=n_stop)
    el = time.perf_counter() - t0
    t0 = time.perf_counter()
    yp, zp, _ = oracle.solve(pb, iy, iz, n_stop=n_stop, threads=True)
    el_all = time.perf_counter() - t0
    same = bool(np.array_equal(yp, yo) and np.array_equal(zp, zo))
    nx = pb["n_x"]
    model = cpu_model()
    return ({"value": nx * steps / el, "unit": "grid-point*time-step/s", "cores": 1,
             "kind": "oracle", "cpu": model,
             "sample": f"first {steps} of {pb['n_t'] - K + 1} backward steps at full grid "
                       f"({nx} points), serial FP64 C oracle, {el:.1f} s",
             "all_cores": {"value": nx * steps / el_all, "cores": omp_threads(),
                           "seconds": el_all, "identical_to_serial": same,
                           "kind": "oracle, OpenMP over the points of a layer"}},
            (n_stop, yo, zo[0]))


def run_batch(args, B, torch, np, ms_fp64_single):
    """Seeded batch of independent calls of uneven sizes, FP32 form, one
    launch per time step per instance group, autotuned; checked against the
    same batch in the FP64 form."""
    import workloads as W

    dev = "cuda:0"
    t0 = time.perf_counter()
    wls = W.option_batch(count=args.batch, prec="fp32_comp")
    ios = []
    for w in wls:
        iy, iz = w.init_layers()
        n = iy.shape[1]
        ios.append((torch.as_tensor(iy, device=dev), torch.as_tensor(iz.reshape(iy.shape), device=dev),
                    torch.empty(n, dtype=torch.float64, device=dev),
                    torch.empty(n, dtype=torch.float64, device=dev)))
    point_steps = sum(w.problem["n_x"] * w.problem["n_t"] for w in wls)
    print(f"[bench] batch of {len(wls)}: {point_steps:.3e} point-steps, inputs built in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()

    def timed(plan, ws, reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            B.bsde_solve_batched(plan, ws, ios, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    plan = B.bsde_plan([w.problem for w in wls])
    ws = B.workspace(plan, dev)
    tune = B.bsde_autotune(plan, ws, ios, stream=stream, reps=3)
    rc, st = B.bsde_solve_batched(plan, ws, ios, stream=stream, stats=True)
    print(f"[bench] batch fp32 status {B.bsde_status_string(rc)} stats {st} tune {tune}",
          file=sys.stderr, flush=True)
    ms = timed(plan, ws, max(1, min(args.steps, 3)))
    y32 = [io[2].cpu().numpy() for io in ios]
    del plan, ws
    # the same batch in FP64 (reference for the FP32 error; also timed)
    for w in wls:
        w.problem["prec"] = "fp64"
    plan = B.bsde_plan([w.problem for w in wls])
    ws = B.workspace(plan, dev)
    B.bsde_solve_batched(plan, ws, ios, stream=stream)
    ms64 = timed(plan, ws, 1)
    err_x0, err_grid = 0.0, 0.0
    for w, io, y in zip(wls, ios, y32):
        y64 = io[2].cpu().numpy()
        i = w.node_index()
        err_x0 = max(err_x0, abs(y[i] - y64[i]) / max(abs(y64[i]), 1.0))
        err_grid = max(err_grid, float(np.max(np.abs(y - y64) / np.maximum(np.abs(y64), 1.0))))
    del plan, ws
    return {"instances": len(wls), "point_steps": point_steps, "prec": "fp32_comp",
            "value": point_steps / (ms * 1e-3), "unit": "grid-point*time-step/s",
            "ms_per_solve": ms, "fp64_ms_per_solve": ms64,
            "speedup_vs_fp64_batch": ms64 / ms,
            "speedup_vs_fp64_single_headline": (point_steps / (ms * 1e-3)) /
            (262144 * 1024 / (ms_fp64_single * 1e-3)),
            "autotune": tune, "max_rel_err_y0_vs_fp64": err_x0,
            "max_rel_err_grid_vs_fp64": err_grid,
            "stability_ratio_max": st["stability_ratio"],
            "recipe": "numpy PCG64 seed 1909: K~U[80,120], sigma~U[.1,.5], r~U[0,.06], "
                      "T~U[.1,2], n_x=round(2^U[10,16]), N in {64,128,256,512}, k=4, L=16; "
                      "even: Black-Scholes, odd: bid-ask R=r+.05"}


def flops_per_point_step_2d(pb: dict, picard_mean: float) -> float:
    """FP64 operations of one point and step of the 2-D sweep if each tensor
    node's three bicubic tensor-spline values were evaluated directly: per
    tensor node (K L^2 of them) three 16-term sums (32 flops each), the linear
    driver (6) and the weighted accumulations (y: 2, z1: 4, z2: 4); per layer
    j = K_y the y expectation (2 per node); the z combination and each Picard
    iteration (8).  The kernel does not evaluate this form (see the next
    function); the count is kept as a reference."""
    K, L = max(pb["k_y"], pb["k_z"]), pb["L"]
    per_node = 3 * 32 + 6 + 10
    return K * L * L * per_node + 2 * L * L + 2 * (3 * K + 1) + 2 * K + picard_mean * 8


def window_columns_2d(pb: dict, tile_cols: int = 512) -> float:
    """Mean over the node rows (j, l0) of the axis-1 window width per tile
    column of the 2-D sweep: the tile's columns plus the row's node spread
    along axis 1, plus 2 (as the plan sizes it)."""
    import numpy as np

    K, L = max(pb["k_y"], pb["k_z"]), pb["L"]
    a, _ = np.polynomial.hermite.hermgauss(L)
    dt = pb["T"] / pb["n_t"]
    dx1 = (pb["x_max"][1] - pb["x_min"][1]) / (pb["n_x"][1] - 1)
    vol = pb["vol"]
    widths = []
    for j in range(1, K + 1):
        sq = math.sqrt(2 * j * dt)
        for l0 in range(L):
            s1 = (pb["drift"][1] * j * dt + vol[1][0] * sq * a[l0] + vol[1][1] * sq * a) / dx1
            m1 = np.floor(s1)
            widths.append(tile_cols + (m1.max() - m1.min()) + 2)
    return float(np.mean(widths)) / tile_cols


def flops_per_point_step_2d_executed(pb: dict, picard_mean: float) -> float:
    """FP64 operations the 2-D sweep executes per point and step (axis-split
    evaluation).  Per node row (j, l0) and window column, the axis-0 terms
    U = A0 v(p) + B0 v(p+1) + C0 Mxx(p) + D0 Mxx(p+1) and the same V with
    Myy, Mxxyy for y, z1, z2 (6 sums of 7 flops), over window_columns_2d
    columns per point; per tensor node the axis-1 combination
    A1 U(q) + B1 U(q+1) + C1 V(q) + D1 V(q+1) for y, z1, z2 (3 x 7), the
    driver (6) and the accumulations (10); per layer j = K_y the y expectation
    (2 per node); the z combination and each Picard iteration (8)."""
    K, L = max(pb["k_y"], pb["k_z"]), pb["L"]
    per_row = 6 * 7 * window_columns_2d(pb)
    per_node = 3 * 7 + 6 + 10
    return (K * L * (per_row + L * per_node) + 2 * L * L + 2 * (3 * K + 1) + 2 * K
            + picard_mean * 8)


def run_2d(args, B, torch, np):
    """A few backward steps of the basket call on the 1024 x 1024 tensor grid
    (N = 128, k = 3, 16 x 16 Gauss-Hermite nodes, FP64)."""
    import workloads as W

    dev = "cuda:0"
    wl = W.basket_2d(n_x=1024, n_t=128, k=3, L=16)
    pb = wl.problem
    steps = args.steps_2d
    pb["n_stop"] = pb["n_t"] - wl.K + 1 - steps
    iy, iz = wl.init_layers()
    npts = iy.shape[1]
    t_iy = torch.as_tensor(iy, device=dev)
    t_iz = torch.as_tensor(iz.reshape(wl.K, -1), device=dev)
    y0 = torch.empty(npts, dtype=torch.float64, device=dev)
    z0 = torch.empty(2 * npts, dtype=torch.float64, device=dev)
    plan = B.bsde_plan(pb)
    ws = B.workspace(plan, dev)
    stream = torch.cuda.current_stream()
    rc, st = B.bsde_solve(plan, ws, t_iy, t_iz, y0, z0, stream=stream, stats=True)
    kt = B.bsde_profile_kernels(plan, ws, [(t_iy, t_iz, y0, z0)], stream=stream)
    sweep_ms = kt["sweep_ms"] / kt["sweep_launches"]
    spline_ms = kt["spline_ms"] / max(kt["spline_launches"], 1)
    fl_direct = flops_per_point_step_2d(pb, st["picard_iter_mean"]) * npts
    fl = flops_per_point_step_2d_executed(pb, st["picard_iter_mean"]) * npts
    print(f"[bench] 2-D basket: status {B.bsde_status_string(rc)} {st} kernels {kt}",
          file=sys.stderr, flush=True)
    # whole solves (all N - K + 1 steps), replayed between events on the stream
    pf = dict(pb)
    pf["n_stop"] = 0
    plan_f = B.bsde_plan(pf)
    ws_f = B.workspace(plan_f, dev)
    rc_f, _ = B.bsde_solve(plan_f, ws_f, t_iy, t_iz, y0, z0, stream=stream, stats=False)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        B.bsde_solve(plan_f, ws_f, t_iy, t_iz, y0, z0, stream=stream, stats=False)
    e1.record(stream)
    torch.cuda.synchronize()
    full_s = e0.elapsed_time(e1) / reps * 1e-3
    steps_full = pb["n_t"] - wl.K + 1
    print(f"[bench] 2-D basket full solve: {full_s * 1e3:.1f} ms, status "
          f"{B.bsde_status_string(rc_f)}", file=sys.stderr, flush=True)
    # the FP32 form (float ring with error feedback): kernel times of the same
    # steps, whole solves, and the whole grid against the FP64 solve
    y64, z64 = y0.cpu().numpy(), z0.cpu().numpy()
    p32 = dict(pb, prec="fp32_comp")
    plan32 = B.bsde_plan(p32)
    ws32 = B.workspace(plan32, dev)
    kt32 = B.bsde_profile_kernels(plan32, ws32, [(t_iy, t_iz, y0, z0)], stream=stream)
    plan32f = B.bsde_plan(dict(p32, n_stop=0))
    ws32f = B.workspace(plan32f, dev)
    rc32, _ = B.bsde_solve(plan32f, ws32f, t_iy, t_iz, y0, z0, stream=stream, stats=False)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        B.bsde_solve(plan32f, ws32f, t_iy, t_iz, y0, z0, stream=stream, stats=False)
    e1.record(stream)
    torch.cuda.synchronize()
    full32 = e0.elapsed_time(e1) / reps * 1e-3
    y32, z32 = y0.cpu().numpy(), z0.cpu().numpy()
    err32 = float(max(np.max(np.abs(y32 - y64) / np.maximum(np.abs(y64), 1.0)),
                      np.max(np.abs(z32 - z64) / np.maximum(np.abs(z64), 1.0))))
    fp32 = {"sweep_kernel_us": 1e3 * kt32["sweep_ms"] / kt32["sweep_launches"],
            "spline_us_per_layer": 1e3 * kt32["spline_ms"] / max(kt32["spline_launches"], 1),
            "full_solve_s": full32, "speedup_vs_fp64": full_s / full32,
            "max_rel_err_vs_fp64": err32, "status": B.bsde_status_string(rc32)}
    print(f"[bench] 2-D basket FP32: {fp32}", file=sys.stderr, flush=True)
    return {"workload": wl.name, "points": npts, "steps_timed": steps, "dtype": "f64",
            "sweep_kernel_us": sweep_ms * 1e3, "spline_us_per_layer": spline_ms * 1e3,
            "value": npts / ((sweep_ms + spline_ms) * 1e-3), "unit": "grid-point*time-step/s",
            "roofline": {"bound": "alu", "achieved": fl / (sweep_ms * 1e-3) / 1e12,
                         "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": fl / (sweep_ms * 1e-3) / 1e12 / FP64_VALU_PEAK_TFLOPS,
                         "flops_per_launch": fl,
                         "flops_counted": "executed (axis-split evaluation)",
                         "flops_per_launch_direct_form": fl_direct,
                         "frac_direct_form": fl_direct / (sweep_ms * 1e-3) / 1e12
                         / FP64_VALU_PEAK_TFLOPS},
            "full_solve_s": full_s, "full_solve_steps": steps_full,
            "full_solve_value": npts * steps_full / full_s,
            "stability_ratio": st["stability_ratio"], "fp32_comp": fp32}


def time_solves(B, torch, wl, prec="fp64", reps=5, autotune=True, extra=None):
    """Whole solves of one workload, replayed between events after a checked
    solve; returns (ms per solve, stats, kernel times, y0 at x0, z0 at x0, y, z)."""
    dev = "cuda:0"
    pb = dict(wl.problem, prec=prec, **(extra or {}))
    iy, iz = wl.init_layers()
    K, n = iy.shape
    t_iy = torch.as_tensor(iy, device=dev).contiguous()
    t_iz = torch.as_tensor(iz.reshape(K, -1), device=dev).contiguous()
    y0 = torch.empty(n, dtype=torch.float64, device=dev)
    z0 = torch.empty(iz.shape[1] * n, dtype=torch.float64, device=dev)
    plan = B.bsde_plan(pb)
    ws = B.workspace(plan, dev)
    stream = torch.cuda.current_stream()
    io = [(t_iy, t_iz, y0, z0)]
    if autotune:
        B.bsde_autotune(plan, ws, io, stream=stream, reps=5)
    rc, st = B.bsde_solve(plan, ws, t_iy, t_iz, y0, z0, stream=stream, stats=True)
    B.bsde_solve(plan, ws, t_iy, t_iz, y0, z0, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        B.bsde_solve(plan, ws, t_iy, t_iz, y0, z0, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    kt = B.bsde_profile_kernels(plan, ws, io, stream=stream)
    y, z = y0.cpu().numpy(), z0.cpu().numpy()
    return ms, st, kt, y, z, B.bsde_status_string(rc)


def toeplitz_flops_per_point_step(pb: dict) -> tuple:
    """Algorithmic and executed FP64 operations of the Toeplitz sweep per point
    and step: per layer j, 8 products per band entry (expectation and
    dW-weighted, of y and z, from the values and the second derivatives:
    16 flops), over the band's nb_j entries (executed: nb_j + 15, the 16 x 16
    tiles' corners); the combination and Picard are left out (under 1%)."""
    K = max(pb["k_y"], pb["k_z"])
    dt = pb["T"] / pb["n_t"]
    dx = (pb["x_max"] - pb["x_min"]) / (pb["n_x"] - 1)
    alg = exe = 0.0
    for j in range(1, K + 1):
        m0 = pb["drift"] * j * dt / dx
        rho = pb["vol"] * math.sqrt(j * dt) / dx
        reach = 9.0 * rho + 1.0
        nb = math.ceil(m0 + reach) - math.floor(m0 - reach) + 2
        alg += 16.0 * nb
        exe += 16.0 * (nb + 15)
    return alg, exe


def smoothing_study(B, torch, twin, substeps: int = 8):
    """The Black-Scholes call of ``twin`` (16384 points, N = 256, k = 4) from
    its payoff at T: raw, Kreiss-smoothed (orders 2 and 4) and time-shifted
    terminal layers, the K - 1 initial layers by the method's 1-step scheme on
    the device (``substeps`` per dt), Gauss-Hermite and exact expectations;
    the errors at the money against the closed form, and the time of a solve."""
    import workloads as W

    dev = "cuda:0"
    p0, nx = twin.problem, twin.problem["n_x"]
    out = {}
    for term in ("raw", "kreiss2", "kreiss4", "shift"):
        wl = W.bs_call_1d(n_x=nx, n_t=p0["n_t"], k=p0["k_y"], L=p0["L"],
                          half_width=(p0["x_max"] - p0["x_min"]) / 2, terminal=term)
        ty, tz = W.terminal_layer(wl)
        ye, ze = wl.exact_at_t0()
        i = wl.node_index()
        for q in ("gh", "exact"):
            pb = dict(wl.problem, quad=q)
            plan = B.bsde_plan(pb)
            ws = B.workspace(plan, dev)
            K = wl.K
            t_iy = torch.zeros((K, nx), dtype=torch.float64, device=dev)
            t_iz = torch.zeros((K, nx), dtype=torch.float64, device=dev)
            t_iy[K - 1] = torch.as_tensor(ty, device=dev)
            t_iz[K - 1] = torch.as_tensor(tz.reshape(-1), device=dev)
            stream = torch.cuda.current_stream()
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(stream)
            B.bsde_initial_layers(pb, substeps, ws, t_iy, t_iz, stream=stream)
            e[1].record(stream)
            y0 = torch.empty(nx, dtype=torch.float64, device=dev)
            z0 = torch.empty(nx, dtype=torch.float64, device=dev)
            rc, _ = B.bsde_solve(plan, ws, t_iy, t_iz, y0, z0, stream=stream)  # captures
            e[2].record(stream)
            B.bsde_solve(plan, ws, t_iy, t_iz, y0, z0, stream=stream)
            e.append(torch.cuda.Event(enable_timing=True))
            e[3].record(stream)
            torch.cuda.synchronize()
            out[f"{term}_{q}"] = {"abs_err_y0": abs(float(y0[i]) - float(ye[i])),
                                  "abs_err_z0": abs(float(z0[i]) - float(ze[i])),
                                  "initial_layers_ms": e[0].elapsed_time(e[1]),
                                  "solve_ms": e[2].elapsed_time(e[3]),
                                  "status": B.bsde_status_string(rc)}
    print(f"[bench] configs: smoothing study {out}", file=sys.stderr, flush=True)
    return out


def shared_grid_batch(B, torch, np, count: int = 256):
    """The batched workload's shared-grid subset (Black-Scholes calls on one
    16384-point interval, N = 256, k = 4, K and r varying), FP64: Gauss-Hermite
    (L = 16) on the vector ALUs against exact expectations on the matrix cores
    (Toeplitz sweep), whole batched solves timed, errors at the money against
    the closed form."""
    import workloads as W

    dev = "cuda:0"
    stream = torch.cuda.current_stream()
    out = {"instances": count}
    for quad in ("gh", "exact"):
        wls = W.option_batch(count=count, shared_grid=count, prec="fp64")
        ios = []
        for w in wls:
            w.problem["quad"] = quad
            iy, iz = w.init_layers()
            n = iy.shape[1]
            ios.append((torch.as_tensor(iy, device=dev), torch.as_tensor(iz.reshape(iy.shape), device=dev),
                        torch.empty(n, dtype=torch.float64, device=dev),
                        torch.empty(n, dtype=torch.float64, device=dev)))
        plan = B.bsde_plan([w.problem for w in wls])
        ws = B.workspace(plan, dev)
        if quad == "gh":
            B.bsde_autotune(plan, ws, ios, stream=stream, reps=2)
        rc, st = B.bsde_solve_batched(plan, ws, ios, stream=stream, stats=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        reps = 2
        for _ in range(reps):
            B.bsde_solve_batched(plan, ws, ios, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        err = 0.0
        for w, io in zip(wls, ios):
            ye, _ = w.exact_at_t0()
            i = w.node_index()
            err = max(err, abs(float(io[2][i]) - ye[i]) / max(abs(ye[i]), 1.0))
        point_steps = sum(w.problem["n_x"] * w.problem["n_t"] for w in wls)
        rec = {"ms_per_solve": ms, "value": point_steps / (ms * 1e-3), "status": B.bsde_status_string(rc),
               "max_rel_err_y0_vs_closed_form": err}
        if quad == "exact":
            steps = wls[0].problem["n_t"] - wls[0].K + 1
            fl = toeplitz_flops_per_point_step(wls[0].problem)[0] * sum(w.problem["n_x"] for w in wls)
            rec["matrix_core_tflops"] = fl * steps / (ms * 1e-3) / 1e12
        out[quad] = rec
        del plan, ws, ios
    print(f"[bench] configs: shared-grid batch {out}", file=sys.stderr, flush=True)
    return out


def run_configs(args, B, torch, np):
    """The other configurations: the sine problem (1025 points, N = 64, k = 2),
    Black-Scholes (16384 points, N = 256, L = 32, k = 4) on its stable twin and
    on the literal interval (Gauss-Hermite, and the exact Gaussian expectation
    on matrix cores), and the bid-ask call on its literal interval (R = 965)."""
    import workloads as W

    out = {}
    wl = W.sine_1d()
    ms, st, kt, y, z, rc = time_solves(B, torch, wl)
    ye, ze = wl.exact_at_t0()
    i = wl.node_index()
    out["sine_1025_nt64_k2"] = {"ms_per_solve": ms, "value": wl.problem["n_x"] * wl.problem["n_t"] / (ms * 1e-3),
                                "abs_err_y0": float(abs(y[i] - ye[i])), "abs_err_z0": float(abs(z[i] - ze[i])),
                                "status": rc, "path": kt["path"]}
    print(f"[bench] configs: sine {out['sine_1025_nt64_k2']}", file=sys.stderr, flush=True)
    nx, nt = 16384, 256
    twin = W.bs_call_1d(n_x=nx, n_t=nt, k=4, L=32, half_width=0.2 * math.sqrt(2 * 0.33 / nt) / 16.0 * (nx - 1) / 2)
    lit = W.bs_call_1d(n_x=nx, n_t=nt, k=4, L=32, half_width=None)
    for name, wl, extra in (("bs_16384_nt256_k4_L32_twin_gh", twin, None),
                            ("bs_16384_nt256_k4_L32_literal_gh", lit, None),
                            ("bs_16384_nt256_k4_literal_exact", lit, {"quad": "exact"}),
                            ("bs_16384_nt256_k4_twin_exact", twin, {"quad": "exact"})):
        ms, st, kt, y, z, rc = time_solves(B, torch, wl, extra=extra)
        ye, ze = wl.exact_at_t0()
        i = wl.node_index()
        rec = {"ms_per_solve": ms, "value": nx * nt / (ms * 1e-3), "status": rc,
               "abs_err_y0": float(abs(y[i] - ye[i])), "abs_err_z0": float(abs(z[i] - ze[i])),
               "stability_ratio": st["stability_ratio"], "path": kt["path"],
               "sweep_kernel_us": 1e3 * kt["sweep_ms"] / max(kt["sweep_launches"], 1)}
        if extra:
            alg, exe = toeplitz_flops_per_point_step(wl.problem)
            us = rec["sweep_kernel_us"]
            rec["roofline"] = {"bound": "mfma", "unit": "TFLOP/s", "peak": FP64_VALU_PEAK_TFLOPS,
                               "achieved": alg * nx / (us * 1e-6) / 1e12,
                               "frac": alg * nx / (us * 1e-6) / 1e12 / FP64_VALU_PEAK_TFLOPS,
                               "executed_tflops": exe * nx / (us * 1e-6) / 1e12,
                               "flops_per_point_step": alg}
        out[name] = rec
        print(f"[bench] configs: {name} {rec}", file=sys.stderr, flush=True)
    out["smoothing_study"] = smoothing_study(B, torch, twin)
    out["shared_grid_batch"] = shared_grid_batch(B, torch, np)
    wl = W.bidask_call_1d(half_width=None)
    ms, st, kt, y, z, rc = time_solves(B, torch, wl, reps=3)
    out["bidask_262144_nt1024_literal_gh"] = {
        "ms_per_solve": ms, "value": wl.problem["n_x"] * wl.problem["n_t"] / (ms * 1e-3),
        "stability_ratio": st["stability_ratio"], "path": kt["path"], "status": rc,
        "note": "timing only: at this stability ratio Gauss-Hermite aliasing makes the "
                "scheme unstable, so the values are not an approximation of the price"}
    print(f"[bench] configs: bidask literal {out['bidask_262144_nt1024_literal_gh']}",
          file=sys.stderr, flush=True)
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="bidask1d",
                    help="bidask1d (the headline), bidask1d_literal, sine1d, bs1d_exact, "
                         "bs1d_literal_exact, or basket2d (the 2-D basket alone)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp64-only", action="store_true", help="skip the FP32-form run")
    ap.add_argument("--batch", type=int, default=4096,
                    help="instances of the batched workload (0 skips it)")
    ap.add_argument("--steps-2d", type=int, default=6,
                    help="backward steps of the 2-D basket workload to time (0 skips it)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="skip the directly launched, event-timed solve (profiler runs that "
                         "should see the graph replays only)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other configurations (sine, Black-Scholes, literal bid-ask)")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="profiling runs: stop each solve after this many backward steps "
                         "(same per-step kernel shape; throughput then counts those steps)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run only a plain device-to-device copy of this many MiB (for "
                         "scaling the hardware byte counters) and exit")
    args = ap.parse_args()
    if args.calibrate_copy_mib:
        import torch

        n = args.calibrate_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "copies": 3}))
        return 0
    if args.gpus != 1:
        print("bench.py measures one GPU: the method has no cross-GPU communication and this "
              "build runs on a single MI355X; --gpus must be 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1909_13560_amd as B

    if args.workload == "basket2d":
        # the 2-D basket alone (profiling runs of its kernels)
        import torch

        import paper_1909_13560_amd as B

        torch.cuda.set_device(0)
        print(json.dumps({"two_d": run_2d(args, B, torch, np)}), flush=True)
        return 0
    wl = workload(args.workload)
    pb = wl.problem
    steps_run = pb["n_t"] - wl.K + 1
    if args.profile_steps:
        args.batch = 0
        args.steps_2d = 0
        steps_run = min(args.profile_steps, steps_run)
        pb["n_stop"] = pb["n_t"] - wl.K + 1 - steps_run
        args.no_cpu_baseline = True
    dev = "cuda:0"
    torch.cuda.set_device(0)
    iy, iz = wl.init_layers()
    K, nx = wl.K, pb["n_x"]
    t_iy = torch.as_tensor(iy, device=dev).contiguous()
    t_iz = torch.as_tensor(iz.reshape(K, nx), device=dev).contiguous()
    stream = torch.cuda.current_stream()
    ye, ze = wl.exact_at_t0()
    i = wl.node_index()

    def run(prec: str):
        """Time full solves of the workload in one precision form."""
        p = dict(pb, prec=prec)
        plan = B.bsde_plan(p)
        ws = B.workspace(plan, dev)
        y0 = torch.empty(nx, dtype=torch.float64, device=dev)
        z0 = torch.empty(nx, dtype=torch.float64, device=dev)
        # the library's own kernel-shape choice for this plan, made once (like
        # the plan itself) before anything is timed; profiling runs keep the
        # plan's default shape, since a profiler distorts the candidates' times
        if not args.profile_steps:
            tune = B.bsde_autotune(plan, ws, [(t_iy, t_iz, y0, z0)], stream=stream, reps=20)
            print(f"[bench] {prec}: autotune {tune}", file=sys.stderr, flush=True)
        # one checked solve: status and Picard statistics
        rc, st = B.bsde_solve(plan, ws, t_iy, t_iz, y0, z0, stream=stream, stats=True)
        print(f"[bench] workload {wl.name} {prec} status {B.bsde_status_string(rc)} stats {st}",
              file=sys.stderr, flush=True)
        for _ in range(args.warmup):
            B.bsde_solve(plan, ws, t_iy, t_iz, y0, z0, stream=stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            B.bsde_solve(plan, ws, t_iy, t_iz, y0, z0, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        print(f"[bench] {prec}: {args.steps} solves, {ms:.3f} ms per solve", file=sys.stderr,
              flush=True)
        # per-kernel durations from hipEvents around every launch of one solve
        # launched directly (skipped when a profiler should see graph
        # replays only)
        kt = None
        if not args.no_kernel_events:
            kt = B.bsde_profile_kernels(plan, ws, [(t_iy, t_iz, y0, z0)], stream=stream)
            print(f"[bench] {prec}: kernels {kt}", file=sys.stderr, flush=True)
        return ms, st, kt, y0.cpu().numpy(), z0.cpu().numpy()

    ms, st, kt, y_h, z_h = run("fp64")
    value = nx * (pb["n_t"] if not args.profile_steps else steps_run) / (ms * 1e-3)
    # the sweep kernel's average launch duration in the timed region: the
    # solve is the replayed graph of steps_run sweep launches (plus the
    # initial-layer scatter and splines and the final gather, together well
    # under 1% of it), timed by the events around the replays; counting the
    # whole solve against the launches makes this an upper bound
    sweep_ms = ms / steps_run
    sweep_ms_direct = kt["sweep_ms"] / kt["sweep_launches"] if kt else None
    spline_ms = kt["spline_ms"] / kt["spline_launches"] if kt and kt["spline_launches"] else 0.0
    exact = pb.get("quad") == "exact"
    if exact:  # the Toeplitz sweep: matrix-core products of the bands
        fl = toeplitz_flops_per_point_step(pb)[0] * nx
    else:
        fl = flops_per_point_step(pb, st["picard_iter_mean"]) * nx
    achieved = fl / (sweep_ms * 1e-3) / 1e12
    # error of the headline value against the closed form
    err = {"y0": float(y_h[i]), "z0": float(z_h[i]),
           "abs_err_y0": float(abs(y_h[i] - ye[i])), "abs_err_z0": float(abs(z_h[i] - ze[i]))}

    fp32 = None
    if not args.fp64_only:
        ms32, st32, kt32, y32, z32 = run("fp32_comp")
        sw32 = ms32 / steps_run
        scale = np.maximum(np.abs(y_h), 1.0)
        x = wl.grid(0)
        sg = wl.extra.get("sigma", 0.2)
        core = np.abs(x - wl.x0) <= 6 * sg * math.sqrt(pb["T"])  # where the price matters
        fp32 = {
            "max_rel_err_vs_fp64_y_core": float(np.max((np.abs(y32 - y_h) / scale)[core])),
            "max_rel_err_vs_fp64_z_core": float(np.max(
                (np.abs(z32 - z_h) / np.maximum(np.abs(z_h), 1.0))[core])),
            "value": nx * (pb["n_t"] if not args.profile_steps else steps_run) / (ms32 * 1e-3),
            "ms_per_step": ms32, "speedup_vs_fp64": ms / ms32, "kernel_us": sw32 * 1e3,
            "vector_alu_tflops": flops_per_point_step(pb, st32["picard_iter_mean"]) * nx
            / (sw32 * 1e-3) / 1e12,
            "max_rel_err_vs_fp64_y": float(np.max(np.abs(y32 - y_h) / scale)),
            # where the largest differences sit (grid index and x, final layer)
            "argmax_y": {"i": int(np.argmax(np.abs(y32 - y_h) / scale)),
                         "x": float(x[int(np.argmax(np.abs(y32 - y_h) / scale))])},
            "argmax_z": {"i": int(np.argmax(np.abs(z32 - z_h) / np.maximum(np.abs(z_h), 1.0))),
                         "x": float(x[int(np.argmax(np.abs(z32 - z_h) /
                                                    np.maximum(np.abs(z_h), 1.0)))])},
            "max_rel_err_vs_fp64_z": float(np.max(np.abs(z32 - z_h) / np.maximum(np.abs(z_h), 1.0))),
            "rel_err_y0_vs_closed_form": float(abs(y32[i] - ye[i]) / max(abs(ye[i]), 1.0)),
            "rel_err_z0_vs_closed_form": float(abs(z32[i] - ze[i]) / max(abs(ze[i]), 1.0)),
            "config": ({"points_per_lane": kt32["points_per_lane"],
                        "node_groups": kt32["node_groups"], "path": kt32["path"]} if kt32 else None),
        }

    batched = None
    if args.batch:
        batched = run_batch(args, B, torch, np, ms)
    two_d = run_2d(args, B, torch, np) if args.steps_2d else None
    configs = None if (args.no_configs or args.profile_steps) else run_configs(args, B, torch, np)

    out = {
        "metric": "grid-point*time-step updates/sec (k=4, L=16)",
        "value": value,
        # the same rate counting only the layers the sweep computes, N - K + 1
        "value_computed_steps": nx * steps_run / (ms * 1e-3),
        "unit": "grid-point*time-step/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_x": nx, "n_t": pb["n_t"], "k": pb["k_y"],
                   "L": pb["L"], "driver": pb["driver"], "x_min": pb["x_min"],
                   "x_max": pb["x_max"], "picard_tol": pb["picard_tol"],
                   "stability_ratio": st["stability_ratio"]},
        "roofline": {"bound": "mfma" if exact else "alu", "achieved": achieved,
                     "peak": FP64_VALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK_TFLOPS,
                     "traffic": None if exact else measured_traffic(wl.name),
                     "kernel": "sweep_toeplitz" if exact else "sweep_fused",
                     "kernel_us": sweep_ms * 1e3,
                     "kernel_us_measured_as": "graph-replayed solves between hipEvents on "
                                              "the launch stream, per sweep launch",
                     "kernel_us_direct_launch": (sweep_ms_direct * 1e3 if kt else None),
                     "flops_per_launch": fl,
                     "hbm_bytes_per_launch_algorithmic": bytes_per_point_step(pb) * nx},
        "spline_kernel_us": spline_ms * 1e3,
        "sweep_config": ({"points_per_lane": kt["points_per_lane"],
                          "node_groups": kt["node_groups"], "path": kt["path"],
                          "blocks": kt["blocks"], "lds_bytes": kt["lds_bytes"]} if kt else None),
        "accuracy": err,
        "fp32_comp": fp32,
        "batched": batched,
        "two_d": two_d,
        "configs": configs,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"], (n_stop, yo, zo) = cpu_baseline(wl, args.cpu_budget)
        # the library against the oracle at full size, over the same steps
        par = {"n_stop": n_stop, "steps": pb["n_t"] - wl.K + 1 - n_stop}
        for prec in (["fp64"] if args.fp64_only else ["fp64", "fp32_comp"]):
            y_g, z_g, _, _ = B.solve(dict(pb, n_stop=n_stop, prec=prec), iy, iz)
            par[f"max_rel_err_{prec}"] = float(max(
                np.max(np.abs(y_g - yo) / np.maximum(np.abs(yo), 1.0)),
                np.max(np.abs(z_g[0] - zo) / np.maximum(np.abs(zo), 1.0))))
        out["oracle_parity_full_grid"] = par
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
