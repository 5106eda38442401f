"""Seeded synthetic inputs for the solver: initial states, pumps and potentials.

This module holds no step of the time integration: it only builds the arrays a
run starts from, on the host, in float64, from numpy's PCG64 generator, so that
the GPU solver and the CPU oracle can be fed bit-identical inputs.  Random numbers
are always drawn here and handed over as arrays; the solver itself draws none.

Coordinates follow a grid symmetric about the origin,
    x_i = (i - (nx - 1)/2) dx,   y_j = (j - (ny - 1)/2) dy,
so centred potentials and pumps are mirror symmetric on the grid.

Workloads (units hbar = m = 1; the paper's own example parameter sets are not
part of its text, so these stand in for them):
  conservative  256^2, dx 0.1, periodic, V = r^2/2, g = 1, RK4 dt 1e-3, Gaussian
                (sigma 2) with seeded uniform phase noise of amplitude 0.01.
  driven        1024^2 (or any size), dx 0.2, periodic, g 0.01, g_r 0.02,
                gamma_c 0.15, gamma_r 0.225, R 0.01, ring pump 2 P_th centred at
                radius 20 with width 3, seeded complex white noise psi0 of
                amplitude 1e-3, n0 = 0, RK4 dt 0.02.
  spinor        4096^2, dx 0.1, zero boundaries, g 1, g_x -0.1, Delta_LT 0.1,
                Gaussian-correlated disorder (length 1, rms 0.05), x-linear Gaussian
                state of width 20, Dormand-Prince with tolerance 1e-6.
  spinor_driven the spinor grid with a reservoir per component: the driven
                workload's reservoir parameters and ring pump on both components,
                noise psi0 of amplitude 1e-3, n0 = 0.
  batch         256 driven instances on square grids drawn log-uniformly in
                [128, 1024], pump p_i P_th with p_i ~ U(0.5, 3), Gaussian spot of
                width L_i/10, seeded noise psi0.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def coords(nx: int, ny: int, dx: float, dy: float):
    """Grid coordinates (X, Y), each of shape (ny, nx), symmetric about 0."""
    x = (np.arange(nx, dtype=np.float64) - (nx - 1) / 2.0) * dx
    y = (np.arange(ny, dtype=np.float64) - (ny - 1) / 2.0) * dy
    return np.meshgrid(x, y, indexing="xy")


def random_state(shape, seed: int, amplitude: float = 1.0):
    """Complex white noise amplitude*(a + i b)/sqrt(2), a, b ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(shape)
    b = rng.standard_normal(shape)
    return amplitude * (a + 1j * b) / np.sqrt(2.0)


def random_field(shape, seed: int, lo: float = 0.0, hi: float = 1.0):
    """Real uniform field on [lo, hi)."""
    return np.random.default_rng(seed).uniform(lo, hi, shape)


# --------------------------------------------------------------- workloads

@dataclass
class Physics:
    """Equation parameters of a workload (Eq. 1 / Eqs. PULSE_psi, PULSE_res)."""
    nx: int
    ny: int
    dx: float
    dy: float
    bc_x: int = 0          # 0 periodic, 1 zero
    bc_y: int = 0
    components: int = 1
    reservoir: bool = False
    hbar: float = 1.0
    mass: float = 1.0
    g: float = 0.0
    g_x: float = 0.0
    g_r: float = 0.0
    R: float = 0.0
    gamma_c: float = 0.0
    gamma_r: float = 0.0
    delta_lt: float = 0.0
    dt: float = 1e-3

    def as_dict(self):
        return dict(self.__dict__)


def conservative(n: int = 256, seed: int = 1, dx: float = 0.1):
    """Scalar Hermitian GP in a harmonic trap: returns (physics, psi0, V)."""
    ph = Physics(nx=n, ny=n, dx=dx, dy=dx, g=1.0, dt=1e-3)
    X, Y = coords(n, n, dx, dx)
    r2 = X * X + Y * Y
    u = np.random.default_rng(seed).uniform(-1.0, 1.0, (n, n))
    psi = np.exp(-r2 / (2.0 * 2.0 ** 2)) * np.exp(1j * 0.01 * u)
    V = 0.5 * r2
    return ph, psi.reshape(1, n, n), V


def pump_threshold(gamma_c: float, gamma_r: float, R: float) -> float:
    """Homogeneous condensation threshold P_th = gamma_r gamma_c / R."""
    return gamma_r * gamma_c / R


def driven(n: int = 1024, seed: int = 2, dx: float = 0.2, ny: int | None = None):
    """Driven-dissipative scalar GP + reservoir with a ring pump of 2 P_th at
    radius 20 (width 3).  Returns (physics, psi0, n0, P)."""
    ny = n if ny is None else ny
    ph = Physics(nx=n, ny=ny, dx=dx, dy=dx, reservoir=True, g=0.01, g_r=0.02, R=0.01,
                 gamma_c=0.15, gamma_r=0.225, dt=0.02)
    X, Y = coords(n, ny, dx, dx)
    r = np.sqrt(X * X + Y * Y)
    pth = pump_threshold(ph.gamma_c, ph.gamma_r, ph.R)
    P = 2.0 * pth * np.exp(-((r - 20.0) ** 2) / (2.0 * 3.0 ** 2))
    psi = random_state((1, ny, n), seed, 1e-3)
    n0 = np.zeros((1, ny, n))
    return ph, psi, n0, P.reshape(1, ny, n)


def disorder(n: int, dx: float, seed: int, corr: float = 1.0, rms: float = 0.05):
    """Gaussian-correlated disorder: white N(0,1) noise convolved (periodically, by
    FFT) with exp(-r^2/corr^2), mean removed and scaled to the given rms."""
    w = np.random.default_rng(seed).standard_normal((n, n))
    k = np.fft.fftfreq(n, d=dx) * 2.0 * np.pi
    KX, KY = np.meshgrid(k, k, indexing="xy")
    # Fourier transform of exp(-r^2/corr^2) up to a constant factor
    kern = np.exp(-(KX * KX + KY * KY) * corr * corr / 4.0)
    v = np.real(np.fft.ifft2(np.fft.fft2(w) * kern))
    v -= v.mean()
    v *= rms / np.sqrt(np.mean(v * v))
    return v


def spinor(n: int = 4096, seed: int = 3, dx: float = 0.1, width: float = 20.0):
    """Two-component conservative GP with TE-TM coupling and disorder, zero
    boundaries.  Returns (physics, psi0 [2,n,n], V)."""
    ph = Physics(nx=n, ny=n, dx=dx, dy=dx, bc_x=1, bc_y=1, components=2, g=1.0, g_x=-0.1,
                 delta_lt=0.1, dt=1e-3)
    X, Y = coords(n, n, dx, dx)
    env = np.exp(-(X * X + Y * Y) / (2.0 * width * width)) / np.sqrt(2.0)
    psi = np.stack([env, env]).astype(np.complex128)
    V = disorder(n, dx, seed)
    return ph, psi, V


def spinor_driven(n: int = 4096, seed: int = 3, dx: float = 0.1):
    """The spinor workload with a reservoir per component (Eq. PULSE_res for each
    spin): the spinor's grid, boundaries, interactions, TE-TM coupling and disorder,
    the driven workload's reservoir parameters and ring pump (2 P_th at radius 20,
    width 3) on both components, seeded complex white noise psi0 of amplitude 1e-3,
    n0 = 0.  Returns (physics, psi0 [2,n,n], n0 [2,n,n], V, P [2,n,n])."""
    ph, _, V = spinor(n, seed=seed, dx=dx)
    ph.reservoir = True
    ph.g_r, ph.R, ph.gamma_c, ph.gamma_r = 0.02, 0.01, 0.15, 0.225
    X, Y = coords(n, n, dx, dx)
    r = np.sqrt(X * X + Y * Y)
    pth = pump_threshold(ph.gamma_c, ph.gamma_r, ph.R)
    ring = 2.0 * pth * np.exp(-((r - 20.0) ** 2) / (2.0 * 3.0 ** 2))
    psi = random_state((2, n, n), seed + 1, 1e-3)
    return ph, psi, np.zeros((2, n, n)), V, np.stack([ring, ring])


def batch_sizes(count: int = 256, seed: int = 4, lo: int = 128, hi: int = 1024):
    """Square grid sizes drawn log-uniformly in [lo, hi]."""
    u = np.random.default_rng(seed).uniform(np.log(lo), np.log(hi), count)
    return np.rint(np.exp(u)).astype(int)


def batch_pumps(count: int = 256, seed: int = 4, lo: float = 0.5, hi: float = 3.0):
    """Pump strengths p_i (in units of P_th) drawn uniformly in [lo, hi]."""
    rng = np.random.default_rng(seed + 7919)
    return rng.uniform(lo, hi, count)


def batch_instance(n: int, p: float, seed: int, dx: float = 0.2):
    """One driven instance: Gaussian pump spot p P_th exp(-r^2/(2 w^2)), w = L/10."""
    ph, psi, n0, _ = driven(n, seed=seed, dx=dx)
    X, Y = coords(n, n, dx, dx)
    w = n * dx / 10.0
    pth = pump_threshold(ph.gamma_c, ph.gamma_r, ph.R)
    P = p * pth * np.exp(-(X * X + Y * Y) / (2.0 * w * w))
    return ph, psi, n0, P.reshape(1, n, n)


def smooth_phase(n: int, dx: float, seed: int, corr: float = 5.0, rms: float = 2.0 * np.pi):
    """Seeded random phase field: white noise filtered with a Gaussian of correlation
    length `corr` (periodic, by FFT), scaled to the given rms."""
    w = np.random.default_rng(seed).standard_normal((n, n))
    k = np.fft.fftfreq(n, d=dx) * 2.0 * np.pi
    KX, KY = np.meshgrid(k, k, indexing="xy")
    th = np.real(np.fft.ifft2(np.fft.fft2(w) * np.exp(-(KX * KX + KY * KY) * corr * corr / 4.0)))
    return th * (rms / np.sqrt(np.mean(th * th)))


def ring_condensate(n: int = 1024, seed: int = 2, dx: float = 0.2):
    """Driven workload started from a condensate already seeded on the ring: density
    at the local homogeneous steady state max(P - P_th, 0)/gamma_c, a seeded smooth
    random phase, plus the 1e-3 complex white noise; reservoir at its local steady
    state (gamma_c/R where P > P_th, else P/gamma_r).  Returns (physics, psi0, n0, P)."""
    ph, noise, _, P = driven(n, seed=seed, dx=dx)
    pth = pump_threshold(ph.gamma_c, ph.gamma_r, ph.R)
    rho0 = np.maximum(P[0] - pth, 0.0) / ph.gamma_c
    psi = np.sqrt(rho0) * np.exp(1j * smooth_phase(n, dx, seed + 500000)) + noise[0]
    n0 = np.where(P[0] > pth, ph.gamma_c / ph.R, P[0] / ph.gamma_r)
    return ph, psi[None], n0[None], P
