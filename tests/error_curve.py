"""Error against the oracle as a function of the step count: the driven-dissipative
workload at 1024^2 (ring pump 2 P_th, noise start; Eqs. PULSE_psi / PULSE_res,
integrated by the RK4 of Eqs. rk4_K1-rk4_final) run by the GPU in complex64 + float32
n and in complex128 + float64 n, every cell compared with the complex128 oracle on the
same (single-precision-rounded) inputs after 10 .. 10^4 steps.

Writes a markdown table (argument 1, default profiles/error_vs_steps_driven1024.md).

    python tests/error_curve.py [out.md] [--steps 10000] [--shape WX ROWS]

Prints one line per checkpoint as it goes (the oracle takes about a minute per 5000
steps on 16 cores).  Test infrastructure: it runs the oracle, so it lives beside the
tests.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

from gpu_helpers import C64, C128, GpuRun, oracle_physics, quantize, rel_l2  # noqa: E402
import oracle  # noqa: E402
from paper_2411_18341_amd import inputs  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("out", nargs="?", default=os.path.join(ROOT, "profiles", "error_vs_steps_driven1024.md"))
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--shape", type=int, nargs=2, default=None, help="whole-step tile shape of the GPU runs")
    args = ap.parse_args()

    ph, psi, n0, P = inputs.driven(args.n)
    q = quantize(C64, psi, n0, None, P)  # exact in double too: both runs start from the same values
    kw = {} if args.shape is None else dict(tile_wx=args.shape[0], tile_rows=args.shape[1])
    runs = {C64: GpuRun(ph, *q, precision=C64, **kw), C128: GpuRun(ph, *q, precision=C128)}
    op = oracle_physics(ph)
    o_psi, o_n = q[0].copy(), q[1].copy()
    marks = [m for m in (10, 30, 100, 300, 1000, 2000, 3000, 5000, 10000, 20000, 50000) if m <= args.steps]
    if marks[-1] != args.steps:
        marks.append(args.steps)
    rows = []
    done = 0
    t0 = time.time()
    for m in marks:
        k = m - done
        o_psi, o_n = oracle.rk4(op, o_psi, o_n, None, q[3], dt=ph.dt, steps=k)
        row = {"steps": m, "t": m * ph.dt}
        for prec, run in runs.items():
            run.step(k)
            g_psi, g_n = run.state()
            row[prec] = (rel_l2(g_psi, o_psi), rel_l2(g_n, o_n))
        row["norm"] = float(np.sum(np.abs(o_psi) ** 2) * ph.dx * ph.dy)
        row["max_rho"] = float(np.max(np.abs(o_psi) ** 2))
        rows.append(row)
        done = m
        print(f"steps {m:6d} t {m * ph.dt:7.1f}: c64 psi {row[C64][0]:.3e} n {row[C64][1]:.3e} | "
              f"c128 psi {row[C128][0]:.3e} n {row[C128][1]:.3e} | oracle norm {row['norm']:.4e} "
              f"max rho {row['max_rho']:.3e} ({time.time() - t0:.0f} s)", flush=True)
    for run in runs.values():
        run.close()

    def last_within(prec, tol):
        # the last checkpoint such that it and every earlier one meet the tolerance
        last = None
        for r in rows:
            if max(r[prec]) > tol:
                break
            last = r["steps"]
        return last

    shape = "automatic tile plan" if args.shape is None else f"whole-step shape {args.shape[0]} x {args.shape[1]}"
    lines = [
        f"# Error against the oracle vs step count, driven workload {args.n}^2 (MI355X)",
        "",
        f"Workload: driven-dissipative GP + reservoir, {args.n}x{args.n}, periodic, dx 0.2, RK4 dt {ph.dt}, "
        "ring pump 2 P_th (radius 20, width 3), noise start of amplitude 1e-3 (seed 2), n0 = 0; inputs "
        "rounded to single precision and given to all three runs.  GPU: complex64 + float32 n and "
        f"complex128 + float64 n ({shape} for complex64); oracle: the plain C complex128 RK4.  Relative L2 "
        "over every cell: |gpu - oracle| / |oracle|.",
        "",
        f"command: python tests/error_curve.py <out.md> --steps {args.steps}" +
        ("" if args.shape is None else f" --shape {args.shape[0]} {args.shape[1]}"),
        "",
        "| steps | t | c64 psi | c64 n | c128 psi | c128 n | oracle norm | oracle max rho |",
        "|---|---|---|---|---|---|---|---|",
    ]
    for r in rows:
        lines.append(f"| {r['steps']} | {r['t']:.1f} | {r[C64][0]:.3e} | {r[C64][1]:.3e} | {r[C128][0]:.3e} | "
                     f"{r[C128][1]:.3e} | {r['norm']:.4e} | {r['max_rho']:.3e} |")
    lines += ["",
              f"Last checkpoint up to which complex64 stays within 1e-5: {last_within(C64, 1e-5)} steps; "
              f"complex128 within 1e-12: {last_within(C128, 1e-12)} steps.", ""]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


if __name__ == "__main__":
    main()
