"""Pins of the oracle's coherent drive (the E term of Eq. PULSE_psi) against exact
solutions of the driven linear problem.

A term -(i/hbar) E(r) exp(-i omega t) in d psi/dt, evaluated at each stage's own
time.  For a uniform state (no kinetic term) and for plane waves (eigenvectors of
the five-point stencil) every mode is a damped oscillator with a harmonic force,
  psi' = lambda psi + F exp(-i omega t),   F = -i E / hbar,
with the exact solution
  psi(t) = A exp(-i omega t) + (psi(t0) - A exp(-i omega t0)) exp(lambda (t - t0)),
  A = F / (-i omega - lambda).
The Runge-Kutta results converge to it at the order of the method only if every
stage sees the force at its own time, so the observed orders (4 for RK4, 5 for
Dormand-Prince) pin the stage times; the values pin the sign and the per-cell,
per-component application.  All run on the CPU in seconds.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import BC_PERIODIC, Physics


def exact(psi0, lam, F, omega, t0, t):
    A = F / (-1j * omega - lam)
    return A * np.exp(-1j * omega * t) + (psi0 - A * np.exp(-1j * omega * t0)) * np.exp(lam * (t - t0))


def uniform_case(E0=0.8 - 0.3j, V0=0.6, gam=0.4, omega=1.7, hbar=1.3, t0=0.7):
    ph = Physics(nx=4, ny=3, dx=0.5, dy=0.5, hbar=hbar, gamma_c=gam,
                 E=np.full((1, 3, 4), E0), omega=omega, t0=t0)
    lam = -1j * V0 / hbar - gam / 2
    F = -1j * E0 / hbar
    V = np.full((3, 4), V0)
    psi0 = np.full((1, 3, 4), 0.3 + 0.2j)
    return ph, V, psi0, lam, F, omega, t0


def rk4_error(dt, T=2.0):
    ph, V, psi0, lam, F, omega, t0 = uniform_case()
    steps = int(round(T / dt))
    out, _ = oracle.rk4(ph, psi0, V=V, dt=dt, steps=steps)
    want = exact(psi0[0, 0, 0], lam, F, omega, t0, t0 + steps * dt)
    return np.max(np.abs(out - want))


def test_rk4_driven_oscillator_fourth_order():
    e1, e2, e3 = rk4_error(0.1), rk4_error(0.05), rk4_error(0.025)
    assert e3 < 2e-7
    for a, b in ((e1, e2), (e2, e3)):
        assert 13.0 < a / b < 19.0, (a, b)


def dp_error(dt, T=2.0):
    ph, V, psi0, lam, F, omega, t0 = uniform_case()
    steps = int(round(T / dt))
    psi = psi0
    for k in range(steps):
        ph.t0 = t0 + k * dt
        psi, _, _, _ = oracle.dopri5_step(ph, psi, V=V, dt=dt)
    want = exact(psi0[0, 0, 0], lam, F, omega, t0, t0 + steps * dt)
    return np.max(np.abs(psi - want))


def test_dopri5_driven_oscillator_fifth_order():
    e1, e2 = dp_error(0.2), dp_error(0.1)
    assert e2 < 1e-7
    assert 26.0 < e1 / e2 < 38.0, (e1, e2)


def test_adaptive_run_follows_the_driven_solution():
    """The controller's time (attempts start at the time reached) drives the phase."""
    ph, V, psi0, lam, F, omega, t0 = uniform_case()
    ctrl = oracle.Controller(t=t0, dt=0.05)
    psi, _, ctrl = oracle.dopri5(ph, psi0, V=V, rtol=1e-10, atol=1e-10, accepted=40, ctrl=ctrl)
    want = exact(psi0[0, 0, 0], lam, F, omega, t0, ctrl.t)
    assert np.max(np.abs(psi - want)) < 1e-8


def test_plane_wave_drive_spinor_components():
    """A plane-wave drive on a periodic grid, different for the two components
    (decoupled: g = g_x = delta_lt = 0): each component follows the exact solution of
    its mode, lambda_k = -i (hbar kappa_k / 2m + V0/hbar) - gamma/2 with the discrete
    Laplacian symbol kappa_k."""
    nx, ny, dx, dy = 16, 12, 0.3, 0.25
    hbar, mass, V0, gam, omega, t0, dt, steps = 1.1, 0.9, 0.3, 0.2, 2.3, 0.4, 1e-3, 600
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    modes = [(3, 2, 0.7 + 0.1j), (-5, 1, -0.2 + 0.6j)]  # (m_x, m_y, amplitude) per component
    E = np.stack([a * np.exp(2j * np.pi * (mx * i / nx + my * j / ny)) for mx, my, a in modes])
    ph = Physics(nx=nx, ny=ny, dx=dx, dy=dy, components=2, hbar=hbar, mass=mass, gamma_c=gam,
                 E=E, omega=omega, t0=t0)
    V = np.full((ny, nx), V0)
    psi0 = np.zeros((2, ny, nx), np.complex128)
    out, _ = oracle.rk4(ph, psi0, V=V, dt=dt, steps=steps)
    for s, (mx, my, a) in enumerate(modes):
        kap = 4 / dx ** 2 * math.sin(math.pi * mx / nx) ** 2 + 4 / dy ** 2 * math.sin(math.pi * my / ny) ** 2
        lam = -1j * (hbar * kap / (2 * mass) + V0 / hbar) - gam / 2
        want = exact(0.0, lam, -1j * E[s] / hbar, omega, t0, t0 + steps * dt)
        err = np.max(np.abs(out[s] - want)) / np.max(np.abs(want))
        # RK4 truncation: |lambda dt| <= 0.02, about 600 (lambda dt)^5 / 120 = 2e-8
        assert err < 5e-8, (s, err)


def test_steady_residual_includes_the_drive():
    """In the driven steady state psi = A exp(-i omega t) the density is constant, so
    the observables' steady residual (taken with the drive at t0) vanishes; without
    the drive the same state decays at rate gamma."""
    ph, V, psi0, lam, F, omega, t0 = uniform_case()
    A = F / (-1j * omega - lam)
    psi = np.full((1, 3, 4), A * np.exp(-1j * omega * t0))
    assert oracle.observables(ph, psi, V=V)["steady_res_density"] < 1e-13
    ph.E = None
    assert oracle.observables(ph, psi, V=V)["steady_res_density"] == pytest.approx(ph.gamma_c, rel=1e-12)


def test_noisy_loop_keeps_the_drive_time():
    """With zero noise intensity the stochastic loop is the deterministic driven run,
    bit for bit (each of its steps starts at t0 + k dt)."""
    ph, V, psi0, lam, F, omega, t0 = uniform_case()
    a, _ = oracle.rk4(ph, psi0, V=V, dt=0.05, steps=9)
    b, _ = oracle.rk4_noise(ph, psi0, V=V, dt=0.05, steps=9, nu=0.0, seed=1)
    assert np.array_equal(a, b)
