"""Coarse grid + learned corrector standing in for the fine grid (driven workload).

Fine grid: the driven-dissipative workload at 1024^2 (dx 0.2, RK4 dt 0.02), every
trajectory started from a condensate seeded on the ring pump (the pump alone does
not condense within the run from noise), snapshots every 250 steps.
Coarse grid: 256^2 over the same domain (dx 0.8) with RK4 dt 0.08 = 4 fine steps.
D is the 4x4 block mean.  Network input: features of a coarse state (Re psi,
Im psi scaled by sqrt(rho_s), n by n_s, P by P_th, rho_s = 22.5 and n_s = 15 the
homogeneous steady state at P = 2 P_th).  Target: the residual
    r = D(fine state after 4 fine steps) - coarse RK4 step of D(fine state)
scaled the same way, so the corrected coarse step is
    coarse_step(D u) + correction(features(D u)).
Everything runs in libphx kernels: the fine and coarse trajectories (batched
whole-step RK4), coarse-graining, features, residuals, the network's forward and
backward passes and Adam; this module only sequences the calls.

    python -m paper_2411_18341_amd.surrogate --train-traj 500 --eval-traj 50 --out report.json
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import inputs, phx

RHO_S = 22.5   # (P - P_th)/gamma_c at P = 2 P_th
N_S = 15.0     # gamma_c / R


def fine_physics(n=1024):
    ph, _, _, P = inputs.driven(n, seed=0)
    return ph, P


def coarse_config(ph, n_coarse, dt):
    c = phx.config_from_physics(ph, precision=phx.PHX_C64, dt=dt)
    c.nx = c.ny = n_coarse
    c.dx = c.dy = ph.dx * ph.nx / n_coarse
    return c


class Pipeline:
    def __init__(self, n_fine=1024, factor=4, device="cuda:0"):
        import torch
        self.torch = torch
        self.dev = device
        self.nf = n_fine
        self.f = factor
        self.nc = n_fine // factor
        self.ph, self.P = fine_physics(n_fine)
        self.pth = inputs.pump_threshold(self.ph.gamma_c, self.ph.gamma_r, self.ph.R)
        self.cfg_f = phx.config_from_physics(self.ph, precision=phx.PHX_C64)
        self.cfg_c = coarse_config(self.ph, self.nc, self.ph.dt * factor)

    # -------------------------------------------------------------- batches
    def fine_batch(self, seeds):
        """Fine trajectories started from seeded ring condensates (inputs.ring_condensate)."""
        torch = self.torch
        b = phx.Batch([(self.nf, self.nf)] * len(seeds), [self.cfg_f], precision=phx.PHX_C64, device=self.dev)
        P = torch.from_numpy(self.P[0]).to(self.dev, torch.float32)
        for k, s in enumerate(seeds):
            _, psi, n0, _ = inputs.ring_condensate(self.nf, int(s), self.ph.dx)
            b.view(b.psi, k).copy_(torch.from_numpy(psi[0]).to(torch.complex64))
            b.view(b.n, k).copy_(torch.from_numpy(n0[0]).to(torch.float32))
            b.view(b.P, k).copy_(P)
        return b

    def coarse_batch(self, count, cfg=None):
        return phx.Batch([(self.nc, self.nc)] * count, [cfg or self.cfg_c], precision=phx.PHX_C64, device=self.dev)

    # Whole batches go through one launch each: equal instances are contiguous in the
    # packed buffers, so they form one grid of count*n rows for the pointwise kernels
    # and the 4x4 block mean (a block never straddles two instances).
    def coarsen_all(self, fine, coarse, factor=None, n_src=None):
        f = self.f if factor is None else factor
        nsrc = self.nf if n_src is None else n_src
        count = len(fine.grids)
        phx.phx_coarsen(phx.PHX_C64, fine.stacked(fine.psi), fine.stacked(fine.n), fine.stacked(fine.P),
                        nsrc, nsrc * count, f, coarse.stacked(coarse.psi), coarse.stacked(coarse.n),
                        coarse.stacked(coarse.P))

    def features_all(self, coarse, out):
        count = len(coarse.grids)
        phx.phx_corrector_features(phx.PHX_C64, coarse.stacked(coarse.psi), coarse.stacked(coarse.n),
                                   coarse.stacked(coarse.P), self.nc, self.nc * count, math.sqrt(RHO_S), N_S,
                                   self.pth, out)

    # -------------------------------------------------------------- data
    def generate(self, seeds, snapshots=20, every=250, log=print):
        """Training pairs from fine trajectories: (features, residual) tensors of
        shape [len(seeds)*snapshots, nc, nc, 4] and [..., 3]."""
        torch = self.torch
        n = len(seeds)
        fine = self.fine_batch(seeds)
        coarse = self.coarse_batch(n)
        ref = self.coarse_batch(n)
        X = torch.empty((n * snapshots, self.nc, self.nc, 4), dtype=torch.float32, device=self.dev)
        R = torch.empty((n * snapshots, self.nc, self.nc, 3), dtype=torch.float32, device=self.dev)
        t0 = time.time()
        for s in range(snapshots):
            fine.step(every - self.f)
            self.coarsen_all(fine, coarse)
            self.features_all(coarse, X[s * n:(s + 1) * n])
            coarse.step(1)
            fine.step(self.f)
            self.coarsen_all(fine, ref)
            phx.phx_corrector_residual(phx.PHX_C64, ref.stacked(ref.psi), ref.stacked(ref.n),
                                       coarse.stacked(coarse.psi), coarse.stacked(coarse.n), self.nc,
                                       self.nc * n, math.sqrt(RHO_S), N_S, R[s * n:(s + 1) * n])
            torch.cuda.synchronize()
            log(f"snapshot {s + 1}/{snapshots} t={(s + 1) * every * self.ph.dt:.1f} ({time.time() - t0:.1f}s)")
        return X, R

    # -------------------------------------------------------------- training
    def target_scales(self, R):
        """RMS of the psi channels (together) and of the n channel of the residuals;
        the network is trained on the residual divided by these."""
        sp = float(R[..., :2].double().pow(2).mean().sqrt())
        sn = float(R[..., 2].double().pow(2).mean().sqrt())
        return max(sp, 1e-12), max(sn, 1e-12)

    def train(self, X, R, epochs=10, batch=16, lr=1e-3, seed=0, log=print):
        torch = self.torch
        sp, sn = self.target_scales(R)
        self.r_scale = (sp, sn)
        R[..., :2] /= sp
        R[..., 2] /= sn
        log(f"residual rms: psi {sp:.3e}, n {sn:.3e} (targets normalized)")
        net = phx.Corrector(self.nc, self.nc, batch, device=self.dev)
        net.init_random(seed)
        rng = np.random.default_rng(seed)
        n = X.shape[0]
        steps = 0
        history = []
        t0 = time.time()
        total = epochs * (n // batch)
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(n)).to(self.dev)
            run = 0.0
            for b in range(n // batch):
                idx = perm[b * batch:(b + 1) * batch]
                xb = X.index_select(0, idx).contiguous()
                rb = R.index_select(0, idx).contiguous()
                frac = steps / max(1, total)
                cur_lr = lr * 0.5 * (1 + math.cos(math.pi * frac))  # cosine decay
                net.train_step(xb, rb, cur_lr)
                steps += 1
                if b % 50 == 0:
                    run = net.loss.item()
            history.append(run)
            log(f"epoch {ep + 1}/{epochs} loss {run:.4e} ({time.time() - t0:.1f}s)")
        torch.cuda.synchronize()
        return net, history, time.time() - t0

    # -------------------------------------------------------------- evaluation
    def box_weights(self, m):
        """[m, nf] matrix of the area-weighted average from the fine grid's cells onto
        the m cells of the same interval (m not a divisor of nf): coarse cell k covers
        fine coordinates [k nf/m, (k+1) nf/m) and takes each fine cell with its overlap
        (the generalization of the block mean: a constant field stays constant, local
        means are kept)."""
        nf = self.nf
        w = np.zeros((m, nf))
        r = nf / m
        for k in range(m):
            lo, hi = k * r, (k + 1) * r
            for i in range(int(math.floor(lo)), min(nf, int(math.ceil(hi)))):
                w[k, i] = max(0.0, min(hi, i + 1) - max(lo, i)) / r
        return self.torch.from_numpy(w).to(self.dev)

    def resampled_batch(self, fine, m, dt):
        """Plain runs on an m^2 grid over the same domain (m not a divisor of the fine
        size): the fine states averaged onto the m^2 cells by area weights
        (box_weights, along x and along y), the pump evaluated on the m^2 grid."""
        torch = self.torch
        n = len(fine.grids)
        b = phx.Batch([(m, m)] * n, [coarse_config(self.ph, m, dt)], precision=phx.PHX_C64, device=self.dev)
        ph_m, _, _, P_m = inputs.driven(m, seed=0, dx=self.ph.dx * self.nf / m)
        P_m = torch.from_numpy(P_m[0]).to(self.dev, torch.float32)
        W = self.box_weights(m)

        def resample(a):
            a = a.to(torch.complex128) if a.is_complex() else a.to(torch.float64)
            Wc = W.to(a.dtype)
            return Wc @ a @ Wc.T

        for k in range(n):
            b.view(b.psi, k).copy_(resample(fine.view(fine.psi, k)).to(torch.complex64))
            b.view(b.n, k).copy_(resample(fine.view(fine.n, k)).to(torch.float32))
            b.view(b.P, k).copy_(P_m)
        return b

    def evaluate(self, net, seeds, t_start=2500, horizons=(8, 64, 512), log=print):
        """Relative L2 errors (density |psi|^2 and reservoir n) of coarse+corrector
        and of plain runs at 256^2, 384^2, 512^2 and 768^2 against the fine 1024^2
        reference, from shared starts at t_start (D(fine state) for 256^2 and 512^2,
        the area-weighted average of the fine state for 384^2 and 768^2), plus the GPU
        time of each run.  Errors on the 256^2 grid (the runs whose size is a multiple of 256)
        and on the 128^2 grid (every run), each state block-averaged onto it."""
        torch = self.torch
        n = len(seeds)
        fine0 = self.fine_batch(seeds)
        fine0.step(t_start)
        nm = self.nf // 2
        cfg_m = coarse_config(self.ph, nm, self.ph.dt * 2)
        # other plain resolutions: 768^2 at the fine step, 384^2 at 4 fine steps
        extra = {"plain_768": (3 * self.nf // 4, self.ph.dt, 1), "plain_384": (3 * self.nf // 8, self.ph.dt * 4, 4)}
        results = {}
        for H in horizons:
            assert H % self.f == 0
            fine = self.fine_batch(seeds)
            fine.psi.copy_(fine0.psi)
            fine.n.copy_(fine0.n)
            plain = self.coarse_batch(n)
            corr = self.coarse_batch(n)
            mid = phx.Batch([(nm, nm)] * n, [cfg_m], precision=phx.PHX_C64, device=self.dev)
            self.coarsen_all(fine, plain)
            self.coarsen_all(fine, corr)
            self.coarsen_all(fine, mid, factor=2)
            torch.cuda.synchronize()
            timings = {}

            def timed(name, fn):
                torch.cuda.synchronize()
                t = time.perf_counter()
                fn()
                torch.cuda.synchronize()
                timings[name] = time.perf_counter() - t

            others = {name: self.resampled_batch(fine, m, dt) for name, (m, dt, _) in extra.items()}
            torch.cuda.synchronize()
            timed("fine_1024", lambda: fine.step(H))
            timed("plain_256", lambda: plain.step(H // self.f))
            timed("plain_512", lambda: mid.step(H // 2))
            for name, (m, dt, per) in extra.items():
                timed(name, lambda b=others[name], k=H // per: b.step(k))
            x = torch.empty((n, self.nc, self.nc, 4), dtype=torch.float32, device=self.dev)
            y = torch.empty((n, self.nc, self.nc, 3), dtype=torch.float32, device=self.dev)
            big = phx.Corrector(self.nc, self.nc, n, device=self.dev)
            big.params.copy_(net.params)

            def corrected():
                for _ in range(H // self.f):
                    self.features_all(corr, x)
                    big.forward(x, y)
                    corr.step(1)
                    phx.phx_corrector_apply(phx.PHX_C64, corr.stacked(corr.psi), corr.stacked(corr.n), y,
                                            self.nc, self.nc * n, math.sqrt(RHO_S) * self.r_scale[0],
                                            N_S * self.r_scale[1])

            timed("corrected_256", corrected)
            big.close()
            ref = self.coarse_batch(n)
            mid_c = self.coarse_batch(n)
            self.coarsen_all(fine, ref)
            self.coarsen_all(mid, mid_c, factor=2, n_src=nm)
            torch.cuda.synchronize()

            def err(b, r):
                rho = (b.psi.abs() ** 2).double()
                rho_r = (r.psi.abs() ** 2).double()
                e_rho = float(torch.linalg.norm(rho - rho_r) / torch.linalg.norm(rho_r))
                e_n = float(torch.linalg.norm(b.n.double() - r.n.double()) / torch.linalg.norm(r.n.double()))
                return e_rho, e_n

            # every run block-averaged onto 128^2
            n128 = self.nf // 8
            to128 = {}
            for name, (src, size) in {"fine_1024": (fine, self.nf), "plain_256": (plain, self.nc),
                                      "plain_512": (mid, nm), "corrected_256": (corr, self.nc),
                                      **{k: (others[k], extra[k][0]) for k in extra}}.items():
                dst = phx.Batch([(n128, n128)] * n, [coarse_config(self.ph, n128, self.ph.dt)],
                                precision=phx.PHX_C64, device=self.dev)
                self.coarsen_all(src, dst, factor=size // n128, n_src=size)
                to128[name] = dst
            m768_c = self.coarse_batch(n)
            self.coarsen_all(others["plain_768"], m768_c, factor=3, n_src=extra["plain_768"][0])
            torch.cuda.synchronize()

            res = {"fine_steps": H, "gpu_seconds": timings}
            for name, b in (("plain_256", plain), ("plain_512", mid_c), ("plain_768", m768_c),
                            ("corrected_256", corr)):
                e = err(b, ref)
                res[name] = {"rel_l2_density": e[0], "rel_l2_reservoir": e[1]}
            for name, b in to128.items():
                if name == "fine_1024":
                    continue
                e = err(b, to128["fine_1024"])
                res.setdefault(name, {})
                res[name]["rel_l2_density_128"] = e[0]
                res[name]["rel_l2_reservoir_128"] = e[1]
            results[str(H)] = res
            log(json.dumps({str(H): res}))
        return results


PLAIN_RUNS = ("plain_256", "plain_384", "plain_512", "plain_768")


def plain_cost_at(r, err, key):
    """GPU seconds a plain run needs for relative error `err`, interpolated
    log-linearly between the plain runs that bracket it on the (error, cost) curve
    (errors on the 128^2 grid, which every run reaches by block averages); the fine
    run is the end point of error 0.  None if no plain run is as inaccurate."""
    t = r["gpu_seconds"]
    pts = sorted((r[name][key], t[name]) for name in PLAIN_RUNS)  # rising error
    if err <= 0:
        return t["fine_1024"]
    better = [(e, c) for e, c in pts if e <= err]
    worse = [(e, c) for e, c in pts if e > err]
    if not better:
        # between the fine run (error 0) and the most accurate plain run: the fine
        # run's cost bounds it from above
        return t["fine_1024"]
    if not worse:
        return None
    (e0, c0), (e1, c1) = better[-1], worse[0]
    if e0 <= 0:
        return c0
    w = (math.log(err) - math.log(e0)) / (math.log(e1) - math.log(e0))
    return math.exp(math.log(c0) + w * (math.log(c1) - math.log(c0)))


def speedup_at(results, target=1e-3, key="rel_l2_density_128"):
    """The protocol's comparison at each horizon: if the corrected coarse run's error
    is within `target`, its speedup over the plain cost interpolated at `target`;
    else its error, its cost and the plain cost interpolated at that same error
    (the speedup at equal error), and whether some plain run is both cheaper and
    more accurate (the corrected run is then dominated)."""
    out = {}
    for H, r in results.items():
        t = r["gpu_seconds"]
        e_c = r["corrected_256"][key]
        c_c = t["corrected_256"]
        at_target = plain_cost_at(r, target, key)
        at_err = plain_cost_at(r, e_c, key)
        dominated = [name for name in PLAIN_RUNS if r[name][key] <= e_c and t[name] <= c_c]
        out[H] = {"corrected_error": e_c, "corrected_cost_s": c_c, "meets_target": e_c <= target,
                  "plain_cost_at_target_s": at_target,
                  "speedup": (at_target / c_c) if (e_c <= target and at_target) else None,
                  "plain_cost_at_corrected_error_s": at_err,
                  "speedup_at_equal_error": (at_err / c_c) if at_err else None,
                  "dominated_by": dominated,
                  "gain_over_plain_256": r["plain_256"][key] / max(e_c, 1e-300)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--train-traj", type=int, default=500)
    ap.add_argument("--eval-traj", type=int, default=50)
    ap.add_argument("--snapshots", type=int, default=20)
    ap.add_argument("--every", type=int, default=250)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--t-start", type=int, default=2500)
    ap.add_argument("--n-fine", type=int, default=1024)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    pl = Pipeline(n_fine=args.n_fine)
    log = lambda s: print(s, flush=True)
    t0 = time.time()
    X, R = pl.generate(list(range(10000, 10000 + args.train_traj)), args.snapshots, args.every, log)
    t_gen = time.time() - t0
    net, hist, t_train = pl.train(X, R, args.epochs, args.batch, args.lr, log=log)
    del X, R
    res = pl.evaluate(net, list(range(20000, 20000 + args.eval_traj)), args.t_start, log=log)
    rep = {"train_trajectories": args.train_traj, "snapshots": args.snapshots, "every": args.every,
           "epochs": args.epochs, "batch": args.batch, "lr": args.lr, "loss_history": hist,
           "generate_seconds": t_gen, "train_seconds": t_train, "eval": res, "speedup_1e-3": speedup_at(res)}
    print(json.dumps(rep), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()
