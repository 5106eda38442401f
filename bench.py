#!/usr/bin/env python3
"""Throughput of the RK4 time stepper on one MI355X.

Workload: the driven-dissipative GP + reservoir equation (Eqs. PULSE_psi /
PULSE_res, one component: Laplacian, g|psi|^2 psi, pump, reservoir rate equation;
V = 0) on a 4096^2 periodic grid, complex64 psi and float32 n, RK4 dt 0.02, ring
pump 2 P_th, seeded noise start.  Inputs are generated on the host and resident in
HBM before the timed region starts.

Metric: grid-point RK4 updates per second, U = Nx Ny steps / seconds (Sec. 4 of
the paper).  The timed steps are replays of one captured hipGraph (the solver's
default way of stepping; the graph is captured after the warmup, outside the timed
region).  Printed as one JSON line together with
  roofline      the dominant kernel's algorithmic bytes per launch over its mean
                launch time, from a separate pass of direct launches bracketed by
                HIP events on the solver's stream, against 8 TB/s; traffic = HBM
                bytes per launch from rocprofv3 counters when a measurement for the
                current kernel source is on file;
  copy_kernel_GBps  the library's streaming copy kernel on a 1 GiB buffer (read +
                write bytes over HIP-event time): the attainable-bandwidth reference;
  walk_pattern  (complex64 with the reservoir) the step kernel's bytes moved in the
                wide walk's access pattern with none of its arithmetic (phx_walk_pattern,
                HIP events): the floor that pattern sets, and the step kernel's launch
                time over it;
  cpu_baseline  the CPU oracle (complex128, OpenMP) timed on a bounded sample of
                the same workload on all its threads and on one thread, with the
                host's CPU model.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point RK4 updates/s + HBM GB/s at 4096² c64; surrogate vs plain at L2 1e-3"
HBM_PEAK_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rk4_traffic.json")
COPY_BYTES = 1 << 30


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the counter summary, if it was taken
    on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    from paper_2411_18341_amd.profiling import kernel_source_hash
    if t.get("source_hash") != kernel_source_hash() or t.get("workload") != workload:
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def copy_bandwidth_gbps(torch, nbytes=COPY_BYTES, reps=20):
    """Read+write bandwidth of the library's streaming copy kernel (phx_stream_copy)
    over a 1 GiB buffer, timed with HIP events on the stream it runs on."""
    from paper_2411_18341_amd import phx
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1.0)
    for _ in range(3):
        phx.stream_copy(dst, src)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        phx.stream_copy(dst, src)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    ok = bool(torch.equal(dst[:1 << 20], src[:1 << 20]))
    del src, dst
    if not ok:
        raise RuntimeError("streaming copy kernel produced wrong data")
    return 2.0 * nbytes * reps / (ms * 1e-3) / 1e9


def walk_pattern_us(torch, psi, n, P, reps=20):
    """Mean time of the walk-pattern kernel (the wide step kernel's loads and stores
    without its arithmetic) from HIP events on torch's current stream.  As the solver
    does between steps, the timed launches alternate between two sets of arrays (each
    launch reads what the previous one wrote; only P is read every time), so that no
    launch finds its inputs in the caches because they were read unchanged the time
    before.  The first launch is checked: psi copied, n + P written."""
    from paper_2411_18341_amd import phx
    psi_a, n_a = psi.clone(), n.clone()
    psi_b, n_b = torch.empty_like(psi), torch.empty_like(n)
    phx.walk_pattern(psi_b, n_b, psi_a, n_a, P)
    torch.cuda.synchronize()
    ok = bool(torch.equal(psi_b, psi_a)) and bool(torch.equal(n_b, n_a + P))
    if not ok:
        raise RuntimeError("walk-pattern kernel produced wrong data")
    for _ in range(3):
        phx.walk_pattern(psi_a, n_a, psi_b, n_b, P)
        phx.walk_pattern(psi_b, n_b, psi_a, n_a, P)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for k in range(reps):
        if k % 2 == 0:
            phx.walk_pattern(psi_a, n_a, psi_b, n_b, P)
        else:
            phx.walk_pattern(psi_b, n_b, psi_a, n_a, P)
    stop.record()
    torch.cuda.synchronize()
    us = start.elapsed_time(stop) * 1e3 / reps
    del psi_a, n_a, psi_b, n_b
    return us


def cpu_model() -> str:
    """Host CPU model name (the 'model name' field lscpu reports)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(ph, psi, n0, P, steps: int, noise: float = 0.0, imag: bool = False, V=None,
                 steps_1t: int = 0) -> dict:
    """The oracle timed on this host: `steps` steps with all its OpenMP threads, then
    `steps_1t` steps on one thread (same workload and grid)."""
    import oracle
    op = oracle.Physics(**{k: getattr(ph, k) for k in (
        "nx", "ny", "dx", "dy", "bc_x", "bc_y", "components", "reservoir", "hbar", "mass", "g",
        "g_x", "g_r", "R", "gamma_c", "gamma_r", "delta_lt")})

    def run(k):
        t0 = time.perf_counter()
        if imag:
            oracle.rk4_imag(op, psi, V=V, dt=ph.dt, steps=k)
        elif noise > 0:
            oracle.rk4_noise(op, psi, n0, None, P, dt=ph.dt, steps=k, nu=noise, seed=1)
        else:
            oracle.rk4(op, psi, n0, None, P, dt=ph.dt, steps=k)
        return time.perf_counter() - t0

    threads = oracle.num_threads()
    dt = run(steps)
    out = {"value": ph.nx * ph.ny * steps / dt, "unit": "UP/s", "cores": threads, "kind": "oracle",
           "sample": f"full {ph.nx}x{ph.ny} grid of the same workload, {steps} RK4 steps, "
                     f"complex128 plain C oracle on {threads} OpenMP threads, {dt:.1f} s",
           "cpu_model": cpu_model(), "host_threads": os.cpu_count()}
    if steps_1t > 0:
        oracle.set_num_threads(1)
        try:
            d1 = run(steps_1t)
        finally:
            oracle.set_num_threads(threads)
        out["one_thread"] = {"value": ph.nx * ph.ny * steps_1t / d1, "unit": "UP/s",
                             "sample": f"{steps_1t} RK4 steps of the same grid on 1 thread, {d1:.1f} s"}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=4096, help="grid side (default 4096)")
    ap.add_argument("--precision", choices=["c64", "c128"], default="c64")
    ap.add_argument("--cpu-steps", type=int, default=50, help="oracle steps for the CPU baseline (about 10-30 s)")
    ap.add_argument("--cpu-steps-1t", type=int, default=3,
                    help="oracle steps for the one-thread CPU figure (0: skip)")
    ap.add_argument("--event-steps", type=int, default=100,
                    help="steps of the separate pass that times each kernel launch with HIP events")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel", choices=["auto", "stage", "step"], default="auto",
                    help="RK4 kernel family (auto: whole-step kernel)")
    ap.add_argument("--no-tune", action="store_true", help="skip the tile-shape search before timing")
    ap.add_argument("--noise", type=float, default=0.0,
                    help="intensity nu of the truncated-Wigner Wiener noise (0 = the deterministic workload)")
    ap.add_argument("--drive", type=float, default=None, metavar="OMEGA",
                    help="add a coherent drive of frequency OMEGA (a Gaussian spot, amplitude 0.8, width 30)")
    ap.add_argument("--imag", action="store_true",
                    help="imaginary-time propagation of the trapped scalar GP (dx 0.01, dtau 5e-5) instead of "
                         "the driven workload")
    ap.add_argument("--tile", type=int, nargs=2, metavar=("WX", "ROWS"), default=None,
                    help="force this tile shape (no search)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures a single GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2411_18341_amd import bytemodel, inputs, phx

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    precision = phx.PHX_C64 if args.precision == "c64" else phx.PHX_C128
    real_bytes = 4 if precision == phx.PHX_C64 else 8

    V0 = None
    if args.imag:
        ph, psi0, V0 = inputs.conservative(args.n, dx=0.01)
        ph.dt = 5e-5
        n0 = P = None
        workload = (f"imaginary-time ground state of the scalar GP (g 1) in a harmonic trap, {args.n}x{args.n}, "
                    f"periodic, {'complex64' if real_bytes == 4 else 'complex128'}, dx 0.01, RK4 dtau {ph.dt}")
    else:
        ph, psi0, n0, P = inputs.driven(args.n)
        workload = (f"driven-dissipative GP + reservoir, {args.n}x{args.n}, periodic, "
                    f"{'complex64 psi + float32 n' if real_bytes == 4 else 'complex128 psi + float64 n'}, "
                    f"ring pump 2 P_th (radius 20, width 3), RK4 dt {ph.dt}")
    # the step kernel's counter record is the deterministic workload's: the noise is a separate pass
    step_workload = workload
    if args.noise > 0:
        workload += f", Wiener noise nu {args.noise}"
    E = None
    if args.drive is not None:
        workload += f", coherent drive omega {args.drive} (Gaussian spot 0.8, width 30)"
        X, Y = inputs.coords(args.n, args.n, ph.dx, ph.dy)
        E = torch.from_numpy((0.8 * np.exp(-(X * X + Y * Y) / (2 * 30.0 ** 2)))[None]).to(
            dtype=phx.torch_dtypes(precision)[0], device="cuda:0").contiguous()
    cdt, rdt = phx.torch_dtypes(precision)
    dev = torch.device("cuda:0")
    psi = torch.from_numpy(psi0).to(dtype=cdt, device=dev).contiguous()
    n = None if n0 is None else torch.from_numpy(n0).to(dtype=rdt, device=dev).contiguous()
    Pd = None if P is None else torch.from_numpy(P).to(dtype=rdt, device=dev).contiguous()
    Vd = None if V0 is None else torch.from_numpy(V0).to(dtype=rdt, device=dev).contiguous()
    family = {"auto": phx.PHX_KERNEL_AUTO, "stage": phx.PHX_KERNEL_STAGE, "step": phx.PHX_KERNEL_STEP}[args.kernel]
    # the timed steps are replays of one captured graph of G steps (G even, dividing K)
    G = next((g for g in range(min(64, args.steps), 1, -1) if g % 2 == 0 and args.steps % g == 0), 0)
    cfg = phx.config_from_physics(ph, precision=precision, kernel=family, noise=args.noise, seed=1,
                                  drive=E is not None, drive_omega=args.drive or 0.0, imag_time=args.imag,
                                  graph_steps=G if G else -1)
    if args.tile:
        cfg.tile_wx, cfg.tile_rows = args.tile
    solver = phx.Solver(cfg, psi, n, Vd, Pd, E=E)
    if args.tile:
        tune = {"tile_wx": args.tile[0], "tile_rows": args.tile[1]}
    else:
        tune = solver.autotune(reps=30, use_cache=False) if not args.no_tune else None

    copy_gbps = copy_bandwidth_gbps(torch)

    solver.step(args.warmup)
    if G:  # capture the graph before the timed region
        solver.step(G)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-kernel launch times: a separate pass of direct launches bracketed by HIP events
    solver.set_timing(True)
    solver.step(args.event_steps)
    times = solver.kernel_times()
    solver.set_timing(False)
    obs = solver.observables()
    solver.close()

    cells = args.n * args.n
    value = cells * args.steps / wall
    res = not args.imag
    stage_model = bytemodel.rk4_stage_fused(real_bytes, reservoir=res, has_v=args.imag, drive=E is not None)
    step_model = bytemodel.rk4_whole_step(real_bytes, reservoir=res, has_v=args.imag)
    if E is not None:  # the whole-step kernel reads the drive profile once per step
        step_model = {"step": step_model["step"] + 2 * real_bytes}
    per_launch = {f"rk4_stage{s}": stage_model[f"stage{s}"] for s in range(1, 5)}
    per_launch["rk4_step"] = step_model["step"]
    per_launch["wiener_noise"] = bytemodel.wiener_noise(real_bytes, reservoir=True)
    per_launch["imag_norm"] = bytemodel.imag_norm(real_bytes)["norm"]
    per_launch["imag_scale"] = bytemodel.imag_norm(real_bytes)["scale"]
    kernels = {}
    for name, t in times.items():
        if name not in per_launch:
            continue
        avg_ms = t["ms_total"] / t["launches"]
        nbytes = per_launch[name] * cells
        kernels[name] = {"launches": t["launches"], "avg_us": avg_ms * 1e3, "bytes_per_launch": nbytes,
                         "GBps": nbytes / (avg_ms * 1e-3) / 1e9}
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
    d = kernels[dom]
    # counter measurements of the whole-step kernel are kept per region shape
    shape_key = dom
    if dom == "rk4_step" and tune is not None:
        wx, rows = tune["tile_wx"], tune["tile_rows"]
        shape_key = f"rk4_step_wide{8 if wx == 2 else 12}" if wx in (2, 3) else f"rk4_step_{wx}x{rows}"
    # the drive and imaginary time change what the stage kernels read: their counter records
    # are separate files
    traffic = measured_traffic(shape_key, step_workload) if args.drive is None and not args.imag else None
    roofline = {"bound": "hbm", "achieved": round(d["GBps"], 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(d["GBps"] / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": shape_key, "bytes_per_launch": d["bytes_per_launch"],
                "avg_launch_us": round(d["avg_us"], 2)}
    family_name = "whole-step (1 launch per step)" if dom == "rk4_step" else "stage-fused (4 launches per step)"
    step_bytes = step_model["step"] if dom == "rk4_step" else stage_model["step"]
    if args.noise > 0:
        step_bytes += per_launch["wiener_noise"]
    if args.imag:
        step_bytes += per_launch["imag_norm"] + per_launch["imag_scale"]
    step_gbps = step_bytes * cells * args.steps / wall / 1e9

    walk = None
    if real_bytes == 4 and res and E is None and args.n % 2 == 0:
        wus = walk_pattern_us(torch, psi, n, Pd)
        walk = {"us": round(wus, 2), "GBps": round(step_model["step"] * cells / (wus * 1e-6) / 1e9, 1),
                "band_rows": "the 8-row ring's device-filling height",
                "step_kernel_over_pattern": round(d["avg_us"] / wus, 3) if dom == "rk4_step" else None}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(ph, psi0, n0, P, args.cpu_steps, args.noise, args.imag, V0, args.cpu_steps_1t)

    line = {
        "metric": METRIC, "value": value, "unit": "UP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "graph_capture_steps": G, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if real_bytes == 4 else "f64",
        "data": "synthetic",
        "config": {"workload": workload, "grid": [args.n, args.n], "integrator": "rk4", "noise": args.noise,
                   "drive_omega": args.drive, "imag_time": args.imag,
                   "kernel_family": family_name,
                   "tile": None if tune is None else [tune["tile_wx"], tune["tile_rows"]]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "step_model_bytes_per_point": step_bytes,
        "step_algorithmic_GBps": round(step_gbps, 1),
        "copy_kernel_GBps": round(copy_gbps, 1),
        "walk_pattern": walk,
        "event_pass_steps": args.event_steps,
        "kernels": {k: {kk: round(vv, 2) if isinstance(vv, float) else vv for kk, vv in v.items()}
                    for k, v in kernels.items()},
        "final_norm": obs["norm"][0], "nonfinite": obs["nonfinite"],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
