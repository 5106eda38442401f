"""Throughput against grid size, the analogue of the paper's Fig. 4 (Sec. 4.2), and
the per-kernel time split, the analogue of its Fig. 5 (Sec. 4.4).

For each side N the driven-dissipative workload (complex64 psi, float32 n, ring
pump, RK4 dt 0.02, periodic) runs on one GPU with each RK4 kernel family:
  stage  four stage-fused launches per step (220 B/pt of algorithmic traffic)
  step   one whole-step launch per step (28 B/pt)
after a tile-shape search for that size (--precisions c64 c128 adds complex128 psi
with float64 n).  Reported per (N, family): grid-point updates per second from the
wall clock with kernel timing off, the algorithmic GB/s of the step, and the mean
time of every kernel launched (HIP events on the solver's stream, in a separate
pass).  Small grids fit the 256 MB Infinity Cache and launch overhead dominates the
smallest; large ones stream from HBM.

    python -m paper_2411_18341_amd.sweep --sizes 128 256 512 1024 2048 4096 8192 --out sweep.md

With --batch it first measures the batched workload of 256 driven instances on
grids of 128..1024 (one persistent launch per step) against stepping the same
instances with one solver each; with --spinor the 4096^2 two-component workload
with RK4 and with Dormand-Prince; with --noise the 4096^2 driven workload with the
truncated-Wigner noise on and off; with --drive the stage-fused kernels with and without
the coherent drive; with --ensemble a batched noisy Monte Carlo ensemble.
"""
from __future__ import annotations

import argparse
import json
import time

from . import bytemodel, inputs, phx


def steps_for(n: int) -> int:
    """Timed step count: about 4e9 point updates per measurement, within [50, 5000]."""
    return max(50, min(5000, int(4e9 / (n * n))))


def measure(n: int, family: str, precision=phx.PHX_C64, warmup: int = 20, tune_reps: int = 5):
    import torch
    ph, psi0, n0, P = inputs.driven(n)
    cdt, rdt = phx.torch_dtypes(precision)
    dev = torch.device("cuda:0")
    psi = torch.from_numpy(psi0).to(dtype=cdt, device=dev).contiguous()
    nn = torch.from_numpy(n0).to(dtype=rdt, device=dev).contiguous()
    Pd = torch.from_numpy(P).to(dtype=rdt, device=dev).contiguous()
    del psi0, n0, P
    kernel = {"stage": phx.PHX_KERNEL_STAGE, "step": phx.PHX_KERNEL_STEP}[family]
    cfg = phx.config_from_physics(ph, precision=precision, kernel=kernel)
    solver = phx.Solver(cfg, psi, nn, None, Pd)
    try:
        tune = solver.autotune(reps=tune_reps, use_cache=False)
        steps = steps_for(n)
        # the warm-up runs as many steps as the timed call, so that the replayed graph
        # is captured and instantiated before the clock starts
        solver.step(max(warmup, steps))
        torch.cuda.synchronize()
        # wall clock with kernel timing off (graph replays as in production), then a
        # separate pass with HIP events around every launch for the per-kernel times
        t0 = time.perf_counter()
        solver.step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        solver.set_timing(True)
        solver.step(min(steps, 200))
        torch.cuda.synchronize()
        times = solver.kernel_times()
    finally:
        solver.close()
    real_bytes = 4 if precision == phx.PHX_C64 else 8
    model = (bytemodel.rk4_whole_step if family == "step" else bytemodel.rk4_stage_fused)(
        real_bytes, reservoir=True, has_v=False)
    cells = n * n
    return {
        "n": n, "family": family, "precision": "c64" if precision == phx.PHX_C64 else "c128",
        "steps": steps, "tile": [tune["tile_wx"], tune["tile_rows"]],
        "UPs": cells * steps / wall, "us_per_step": wall / steps * 1e6,
        "algorithmic_GBps": model["step"] * cells * steps / wall / 1e9,
        "kernels_us": {k: v["ms_total"] / v["launches"] * 1e3 for k, v in times.items()},
    }


def measure_batch(steps: int = 500, warmup: int = 20, count: int = 256, seed: int = 4, loop_steps: int = 50):
    """The batched sweep workload (inputs.batch_sizes / batch_pumps / batch_instance:
    `count` driven instances on square grids drawn log-uniformly in [128, 1024],
    complex64) stepped by one persistent launch per step, against the same instances
    stepped one solver at a time (each with its own whole-step launches, graph
    chunks and default region shape)."""
    import torch
    sizes = inputs.batch_sizes(count, seed)
    pumps = inputs.batch_pumps(count, seed)
    ph0, _, _, _ = inputs.batch_instance(int(sizes[0]), 1.0, 0)
    cfg = phx.config_from_physics(ph0, precision=phx.PHX_C64)
    b = phx.Batch([(int(n), int(n)) for n in sizes], [cfg], [0] * count, precision=phx.PHX_C64)
    solvers = []
    for k, (n, p) in enumerate(zip(sizes, pumps)):
        ph, psi, n0, P = inputs.batch_instance(int(n), float(p), 1000 + k)
        b.view(b.psi, k).copy_(torch.from_numpy(psi[0]).to(torch.complex64))
        b.view(b.n, k).copy_(torch.from_numpy(n0[0]).to(torch.float32))
        b.view(b.P, k).copy_(torch.from_numpy(P[0]).to(torch.float32))
    cells = int(sum(int(n) * int(n) for n in sizes))
    b.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the same instances as separate solvers (copies of the batch's current states)
    for k, n in enumerate(sizes):
        n = int(n)
        ph, _, _, P = inputs.batch_instance(n, float(pumps[k]), 1000 + k)
        psi = b.view(b.psi, k).clone().view(1, n, n)
        nn = b.view(b.n, k).clone().view(1, n, n)
        Pd = b.view(b.P, k).clone().view(1, n, n)
        c = phx.config_from_physics(ph, precision=phx.PHX_C64, kernel=phx.PHX_KERNEL_STEP)
        solvers.append(phx.Solver(c, psi, nn, None, Pd))
    for s in solvers:
        s.step(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in solvers:
        s.step(loop_steps)
    torch.cuda.synchronize()
    wall_loop = time.perf_counter() - t0
    for s in solvers:
        s.close()
    return {"instances": count, "cells": cells, "steps": steps, "UPs": cells * steps / wall,
            "us_per_step": wall / steps * 1e6, "one_solver_per_instance_UPs": cells * loop_steps / wall_loop,
            "one_solver_per_instance_steps": loop_steps}


def measure_spinor(n: int = 4096, accepted: int = 20, rk4_steps: int = 50, reservoir: bool = False):
    """The spinor workload (inputs.spinor: two components, TE-TM coupling, cross
    interaction, disorder potential, zero boundaries, complex64) on an n x n grid, or
    with `reservoir` its driven form (inputs.spinor_driven: a reservoir and a ring
    pump per component): RK4 with the tuned kernel family (the two-component
    streaming whole-step kernel), and Dormand-Prince with rtol = atol = 1e-6 from
    dt 1e-3 for `accepted` accepted steps.  Reports point updates per second
    (accepted steps for RK45), attempts, and per-kernel launch times with their
    algorithmic bandwidth."""
    import torch
    if reservoir:
        ph, psi0, n0, V, P = inputs.spinor_driven(n)
    else:
        ph, psi0, V = inputs.spinor(n)
        n0 = P = None
    dev = torch.device("cuda:0")
    out = {"n": n, "reservoir": reservoir}
    real = lambda a: None if a is None else torch.from_numpy(a).to(dtype=torch.float32, device=dev).contiguous()
    for integ in ("rk4", "rk45"):
        psi = torch.from_numpy(psi0).to(dtype=torch.complex64, device=dev).contiguous()
        kw = dict(precision=phx.PHX_C64)
        if integ == "rk45":
            kw.update(integrator=phx.PHX_RK45, rtol=1e-6, atol=1e-6, dt=1e-3)
        cfg = phx.config_from_physics(ph, **kw)
        solver = phx.Solver(cfg, psi, real(n0), real(V), real(P))
        try:
            if integ == "rk4":
                solver.autotune(reps=3, use_cache=False)
            solver.step(2)
            torch.cuda.synchronize()
            info0 = solver.info()
            solver.set_timing(True)
            count = rk4_steps if integ == "rk4" else accepted
            t0 = time.perf_counter()
            solver.step(count)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            info1 = solver.info()
            times = solver.kernel_times()
        finally:
            solver.close()
        if integ == "rk4":
            model = bytemodel.rk4_stage_fused(4, reservoir=reservoir, has_v=True, components=2)
            names = {f"rk4_stage{k}": model[f"stage{k}"] for k in range(1, 5)}
            names["rk4_step"] = bytemodel.rk4_whole_step(4, reservoir=reservoir, has_v=True, components=2)["step"]
        else:
            model = bytemodel.dopri5_attempt(4, reservoir=reservoir, has_v=True, components=2)
            names = {f"dp_stage{k}": model[f"stage{k}"] for k in range(2, 8)}
            names["dp_stage1"] = model["restart"]  # after the first step every attempt restarts from K1
        ks = {}
        for k, v in times.items():
            us = v["ms_total"] / v["launches"] * 1e3
            ks[k] = {"launches": v["launches"], "avg_us": us}
            if k in names:
                ks[k]["algorithmic_GBps"] = names[k] * n * n / (us * 1e-6) / 1e9
        r = {"UPs": n * n * count / wall, "wall_s": wall, "kernels": ks}
        if integ == "rk45":
            acc = info1["steps_accepted"] - info0["steps_accepted"]
            rej = info1["steps_rejected"] - info0["steps_rejected"]
            r.update({"accepted": acc, "rejected": rej, "dt_final": info1["dt"],
                      "attempts_per_s": (acc + rej) / wall, "bytes_per_point_attempt": model["attempt"]})
        out[integ] = r
    return out


def measure_spinor_imag(n: int = 4096, steps: int = 50, drive: bool = False, omega: float = 1.3):
    """The spinor workload (inputs.spinor, complex64, n x n) in imaginary time, or with
    `drive` in real time with a coherent drive (a Gaussian spot of amplitude 0.8 per
    component, the two with opposite phase gradients): RK4 steps on each kernel family
    (the two-component streaming whole-step kernel, which in imaginary time writes one
    norm partial per wave, and the stage-fused family, with its separate norm pass in
    imaginary time), point updates per second of whole steps and per-kernel launch
    times."""
    import numpy as np
    import torch
    ph, psi0, V = inputs.spinor(n)
    dev = torch.device("cuda:0")
    out = {"n": n, "drive": drive}
    model = bytemodel.rk4_whole_step(4, reservoir=False, has_v=True, components=2)["step"] + (16 if drive else 0)
    X, Y = inputs.coords(n, n, ph.dx, ph.dy)
    spot = 0.8 * np.exp(-(X * X + Y * Y) / (2 * 30.0 ** 2))
    E0 = np.stack([spot * np.exp(0.5j * X), spot * np.exp(-0.5j * X)]).astype(np.complex64)
    for family, kernel in (("step", phx.PHX_KERNEL_STEP), ("stage", phx.PHX_KERNEL_STAGE)):
        psi = torch.from_numpy(psi0).to(dtype=torch.complex64, device=dev).contiguous()
        Vd = torch.from_numpy(V).to(dtype=torch.float32, device=dev).contiguous()
        if drive:
            cfg = phx.config_from_physics(ph, precision=phx.PHX_C64, drive=True, drive_omega=omega, kernel=kernel)
            Ed = torch.from_numpy(E0).to(device=dev).contiguous()
            solver = phx.Solver(cfg, psi, None, Vd, None, E=Ed)
        else:
            cfg = phx.config_from_physics(ph, precision=phx.PHX_C64, imag_time=True, kernel=kernel)
            solver = phx.Solver(cfg, psi, None, Vd, None)
        try:
            solver.step(4)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            solver.step(steps)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            solver.set_timing(True)
            solver.step(10)
            torch.cuda.synchronize()
            times = solver.kernel_times()
        finally:
            solver.close()
        ks = {}
        for k, v in times.items():
            us = v["ms_total"] / v["launches"] * 1e3
            ks[k] = {"launches": v["launches"], "avg_us": us}
            if k == "rk4_step":
                ks[k]["algorithmic_GBps"] = model * n * n / (us * 1e-6) / 1e9
        out[family] = {"UPs": n * n * steps / wall, "us_per_step": wall / steps * 1e6, "kernels": ks}
    return out


def measure_noise(n: int = 4096, nu: float = 1.0, steps: int = 300, warmup: int = 20, timed_steps: int = 40):
    """The driven workload (complex64, n x n) with the complex Wiener noise of the
    truncated-Wigner form switched on: point updates per second of whole noisy RK4
    steps (graph replays, as phx_step runs them), the same without noise, and the
    mean launch time of the step kernel and of the noise pass with the pass's
    algorithmic bandwidth (complex read + write, reservoir read)."""
    import torch
    ph, psi0, n0, P = inputs.driven(n)
    dev = torch.device("cuda:0")
    out = {"n": n, "nu": nu}
    for label, noise in (("deterministic", 0.0), ("noisy", nu)):
        psi = torch.from_numpy(psi0).to(dtype=torch.complex64, device=dev).contiguous()
        nn = torch.from_numpy(n0).to(dtype=torch.float32, device=dev).contiguous()
        Pd = torch.from_numpy(P).to(dtype=torch.float32, device=dev).contiguous()
        cfg = phx.config_from_physics(ph, precision=phx.PHX_C64, noise=noise, seed=1234)
        solver = phx.Solver(cfg, psi, nn, None, Pd)
        try:
            tune = solver.autotune(reps=10, use_cache=False)
            solver.step(max(warmup, steps))  # the replayed graph is captured before the clock starts
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            solver.step(steps)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            solver.set_timing(True)
            solver.step(timed_steps)
            torch.cuda.synchronize()
            times = solver.kernel_times()
        finally:
            solver.close()
        ks = {k: v["ms_total"] / v["launches"] * 1e3 for k, v in times.items()}
        r = {"tile": [tune["tile_wx"], tune["tile_rows"]], "UPs": n * n * steps / wall,
             "us_per_step": wall / steps * 1e6, "kernels_us": ks}
        if "wiener_noise" in ks:
            r["noise_algorithmic_GBps"] = bytemodel.wiener_noise(4, True) * n * n / (ks["wiener_noise"] * 1e-6) / 1e9
        out[label] = r
    return out


def measure_drive(n: int = 4096, omega: float = 1.3, steps: int = 100, warmup: int = 10, timed_steps: int = 20):
    """The driven workload (complex64, n x n) with and without a coherent drive (a
    Gaussian spot of amplitude 0.8), on the streaming whole-step kernel and on the
    stage-fused kernels: point updates per second of whole steps (graph replays), and
    per kernel the mean launch time with its algorithmic bandwidth (the drive adds one
    complex read per stage launch, or per step in the whole-step kernel)."""
    import numpy as np
    import torch
    ph, psi0, n0, P = inputs.driven(n)
    X, Y = inputs.coords(n, n, ph.dx, ph.dy)
    E0 = (0.8 * np.exp(-(X * X + Y * Y) / (2 * 30.0 ** 2)))[None].astype(np.complex64)
    dev = torch.device("cuda:0")
    out = {"n": n, "omega": omega}
    runs = (("undriven", False, phx.PHX_KERNEL_STAGE), ("driven", True, phx.PHX_KERNEL_STAGE),
            ("undriven_step", False, phx.PHX_KERNEL_STEP), ("driven_step", True, phx.PHX_KERNEL_STEP))
    for label, drive, family in runs:
        psi = torch.from_numpy(psi0).to(dtype=torch.complex64, device=dev).contiguous()
        nn = torch.from_numpy(n0).to(dtype=torch.float32, device=dev).contiguous()
        Pd = torch.from_numpy(P).to(dtype=torch.float32, device=dev).contiguous()
        Ed = torch.from_numpy(E0).to(device=dev).contiguous() if drive else None
        cfg = phx.config_from_physics(ph, precision=phx.PHX_C64, kernel=family, drive=drive, drive_omega=omega)
        solver = phx.Solver(cfg, psi, nn, None, Pd, E=Ed)
        try:
            tune = solver.autotune(reps=5, use_cache=False)
            solver.step(max(warmup, steps))  # the replayed graph is captured before the clock starts
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            solver.step(steps)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            solver.set_timing(True)
            solver.step(timed_steps)
            torch.cuda.synchronize()
            times = solver.kernel_times()
        finally:
            solver.close()
        if family == phx.PHX_KERNEL_STAGE:
            model = bytemodel.rk4_stage_fused(4, reservoir=True, has_v=False, drive=drive)
        else:
            model = {"step": bytemodel.rk4_whole_step(4, reservoir=True, has_v=False)["step"] + (8 if drive else 0)}
        ks = {}
        for k, v in times.items():
            us = v["ms_total"] / v["launches"] * 1e3
            ks[k] = {"avg_us": us}
            if k.startswith("rk4_stage"):
                ks[k]["algorithmic_GBps"] = model["stage" + k[-1]] * n * n / (us * 1e-6) / 1e9
            if k == "rk4_step":
                ks[k]["algorithmic_GBps"] = model["step"] * n * n / (us * 1e-6) / 1e9
        out[label] = {"tile": [tune["tile_wx"], tune["tile_rows"]], "UPs": n * n * steps / wall,
                      "us_per_step": wall / steps * 1e6, "step_bytes_per_point": model["step"], "kernels": ks}
    return out


def measure_ensemble(count: int = 128, n: int = 256, nu: float = 1.0, steps: int = 400, warmup: int = 20):
    """A Monte Carlo ensemble of the truncated-Wigner form: `count` copies of the
    driven workload on n x n grids (complex64), each with its own noise seed, stepped
    by one batched launch per step plus one noise pass over all instances; against the
    same batch without noise.  Reports point updates per second of the ensemble."""
    import torch
    ph, psi0, n0, P = inputs.driven(n)
    out = {"count": count, "n": n, "nu": nu}
    for label, noise in (("deterministic", 0.0), ("noisy", nu)):
        cfg = phx.config_from_physics(ph, precision=phx.PHX_C64, noise=noise)
        b = phx.Batch([(n, n)] * count, [cfg], precision=phx.PHX_C64, seeds=list(range(1000, 1000 + count)))
        for k in range(count):
            b.view(b.psi, k).copy_(torch.from_numpy(psi0[0]).to(torch.complex64))
            b.view(b.n, k).copy_(torch.from_numpy(n0[0]).to(torch.float32))
            b.view(b.P, k).copy_(torch.from_numpy(P[0]).to(torch.float32))
        b.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[label] = {"UPs": count * n * n * steps / wall, "us_per_step": wall / steps * 1e6}
    return out


def table(rows) -> str:
    out = ["| N | precision | family | tile | steps | µs/step | G UP/s | algorithmic GB/s | mean launch µs per kernel |",
           "|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        ks = ", ".join(f"{k} {v:.2f}" for k, v in sorted(r["kernels_us"].items()))
        out.append(f"| {r['n']} | {r['precision']} | {r['family']} | {r['tile'][0]}x{r['tile'][1]} | {r['steps']} | "
                   f"{r['us_per_step']:.2f} | {r['UPs'] / 1e9:.2f} | {r['algorithmic_GBps']:.0f} | {ks} |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--sizes", type=int, nargs="*", default=[128, 256, 512, 1024, 2048, 4096, 8192])
    ap.add_argument("--families", nargs="+", default=["stage", "step"], choices=["stage", "step"])
    ap.add_argument("--precisions", nargs="+", default=["c64"], choices=["c64", "c128"])
    ap.add_argument("--out", default=None, help="write the markdown table here")
    ap.add_argument("--batch", action="store_true", help="also measure the 256-instance batched workload")
    ap.add_argument("--spinor", action="store_true", help="also measure the 4096^2 spinor workload (RK4, RK45)")
    ap.add_argument("--spinor-reservoir", action="store_true",
                    help="also measure the 4096^2 spinor workload with a reservoir per component")
    ap.add_argument("--spinor-imag", action="store_true",
                    help="also measure the 4096^2 spinor workload in imaginary time on both kernel families")
    ap.add_argument("--spinor-drive", action="store_true",
                    help="also measure the 4096^2 spinor workload with a coherent drive on both kernel families")
    ap.add_argument("--noise", action="store_true", help="also measure the 4096^2 driven workload with Wiener noise")
    ap.add_argument("--drive", action="store_true", help="also measure the stage-fused kernels with a coherent drive")
    ap.add_argument("--ensemble", action="store_true", help="also measure a batched noisy ensemble (128 x 256^2)")
    args = ap.parse_args()
    if args.ensemble:
        r = measure_ensemble()
        print(json.dumps({"ensemble": r}), flush=True)
        if args.out:
            with open(args.out + ".ensemble.json", "w") as f:
                json.dump(r, f, indent=1)
    if args.drive:
        r = measure_drive()
        print(json.dumps({"drive": r}), flush=True)
        if args.out:
            with open(args.out + ".drive.json", "w") as f:
                json.dump(r, f, indent=1)
    if args.noise:
        r = measure_noise()
        print(json.dumps({"noise": r}), flush=True)
        if args.out:
            with open(args.out + ".noise.json", "w") as f:
                json.dump(r, f, indent=1)
    if args.spinor:
        r = measure_spinor()
        print(json.dumps({"spinor": r}), flush=True)
        if args.out:
            with open(args.out + ".spinor.json", "w") as f:
                json.dump(r, f, indent=1)
    if args.spinor_imag:
        r = measure_spinor_imag()
        print(json.dumps({"spinor_imag": r}), flush=True)
        if args.out:
            with open(args.out + ".spinor_imag.json", "w") as f:
                json.dump(r, f, indent=1)
    if args.spinor_drive:
        r = measure_spinor_imag(drive=True)
        print(json.dumps({"spinor_drive": r}), flush=True)
        if args.out:
            with open(args.out + ".spinor_drive.json", "w") as f:
                json.dump(r, f, indent=1)
    if args.spinor_reservoir:
        r = measure_spinor(reservoir=True)
        print(json.dumps({"spinor_reservoir": r}), flush=True)
        if args.out:
            with open(args.out + ".spinor_reservoir.json", "w") as f:
                json.dump(r, f, indent=1)
    if args.batch:
        r = measure_batch()
        print(json.dumps({"batch": r}), flush=True)
        if args.out:
            with open(args.out + ".batch.json", "w") as f:
                json.dump(r, f, indent=1)
    rows = []
    precs = {"c64": phx.PHX_C64, "c128": phx.PHX_C128}
    for prec in args.precisions:
        for n in args.sizes:
            for fam in args.families:
                r = measure(n, fam, precision=precs[prec])
                rows.append(r)
                print(json.dumps(r), flush=True)
    md = table(rows)
    print(md, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(md + "\n")


if __name__ == "__main__":
    main()
