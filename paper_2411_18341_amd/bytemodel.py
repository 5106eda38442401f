"""Algorithmic HBM bytes of the time-stepping kernels, per grid point.

"Algorithmic" counts each array a kernel must read or write exactly once per point
(halo re-reads served by caches are not counted).  These are the figures behind
the roofline numbers the benchmark reports.

paper_unfused_rk4 restates the read/write counts of Table 1 (Sec. 3.2.8): four
derivative kernels (3 reads, 1 write), three two-term sums (2 reads, 1 write) and
one five-term sum (5 reads, 1 write), 23 reads and 8 writes of complex buffers per
step, i.e. 2 (n_r + n_w) d bytes with d the size of one real number.
"""
from __future__ import annotations

# Table 1 of the paper: (reads, writes, launches per RK4 step), scalar, no reservoir
PAPER_TABLE1 = {"derivative": (3, 1, 4), "two_term_sum": (2, 1, 3), "five_term_sum": (5, 1, 1)}


def paper_unfused_rk4(real_bytes: int) -> dict:
    reads = sum(r * k for r, _, k in PAPER_TABLE1.values())
    writes = sum(w * k for _, w, k in PAPER_TABLE1.values())
    return {"reads": reads, "writes": writes, "bytes_per_point": 2 * (reads + writes) * real_bytes}


def rk4_stage_fused(real_bytes: int, reservoir: bool, has_v: bool, components: int = 1,
                    drive: bool = False) -> dict:
    """Bytes per point of the four stage-fused RK4 launches (stage 1..4) and of
    one whole step.  Complex arrays are 2*real_bytes per component, real arrays
    real_bytes per component, V real_bytes (shared by the components); with the
    coherent drive every stage also reads the complex drive profile."""
    c = 2 * real_bytes * components
    r = real_bytes * components if reservoir else 0
    v = real_bytes if has_v else 0
    v += c if drive else 0                     # the drive profile is read like V
    p = r                                      # pump, read by every stage with the reservoir
    s1 = (c + r + p + v) + (2 * c + 2 * r)     # read y=psi,n,P,V; write y2,acc (+n parts)
    s23 = (3 * c + 3 * r + p + v) + (2 * c + 2 * r)  # read y,psi,acc (+n parts),P,V; write y,acc
    s4 = (3 * c + 3 * r + p + v) + (c + r)     # read y,psi,acc,...; write psi,n
    return {"stage1": s1, "stage2": s23, "stage3": s23, "stage4": s4, "step": s1 + 2 * s23 + s4}


def state_minimum(real_bytes: int, reservoir: bool, has_v: bool, components: int = 1) -> int:
    """Whole-step floor: state read and written once, static fields read once."""
    c = 2 * real_bytes * components
    r = real_bytes * components if reservoir else 0
    return 2 * c + 2 * r + (r if reservoir else 0) + (real_bytes if has_v else 0)


def rk4_whole_step(real_bytes: int, reservoir: bool, has_v: bool, components: int = 1) -> dict:
    """Algorithmic bytes per point of the whole-step kernel (one launch per step):
    the state read and written once, pump and potential read once.  Reading the
    4-cell halo of each region again is redundant traffic, not counted here."""
    b = state_minimum(real_bytes, reservoir, has_v, components)
    return {"step": b}


def dopri5_attempt(real_bytes: int, reservoir: bool, has_v: bool, components: int = 1) -> dict:
    """Bytes per point of one attempted Dormand-Prince step as the stage kernels
    move them (first same as last: K1 comes from the previous step).  A restart pass
    forms y2 = psi + dt a21 K1 (reads psi, K1; writes y2); stage s = 2..6 reads y_s,
    psi, K_1..K_{s-1} (and P, V) and writes K_s and y_{s+1}; stage 7 reads y_7, psi
    and the K_j with b_j != bhat_j (all but K_2) and writes K_7.  Every complex pass
    has a reservoir counterpart when the reservoir is on."""
    c = 2 * real_bytes * components + (real_bytes * components if reservoir else 0)
    p = real_bytes * components if reservoir else 0
    v = real_bytes if has_v else 0
    restart = 3 * c
    stages = {s: (s + 1) * c + p + v + 2 * c for s in range(2, 7)}
    stages[7] = 7 * c + p + v + c
    out = {"restart": restart, **{f"stage{s}": b for s, b in stages.items()}}
    out["attempt"] = restart + sum(stages.values())
    return out


def wiener_noise(real_bytes: int, reservoir: bool, components: int = 1) -> int:
    """Bytes per point of the Wiener-increment pass: every complex value is read and
    written once, the reservoir (the amplitude's n) is read once."""
    return components * (4 * real_bytes + (real_bytes if reservoir else 0))


def imag_norm(real_bytes: int, components: int = 1) -> dict:
    """Bytes per point of the imaginary-time norm restoration: the partial sums read
    the complex state once, the scale pass reads and writes it once."""
    c = 2 * real_bytes * components
    return {"norm": c, "scale": 2 * c}
