"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test ties one part of the oracle (right-hand side, boundary rule, RK4 weights,
Dormand-Prince tableau, observables) to something other than the oracle itself:
closed-form solutions of the discrete linear problem, textbook continuum solutions,
exact invariants, the published Dormand-Prince method, or a brute-force dense
matrix formulation.  All run on the CPU in seconds.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.fft
from scipy.integrate import solve_ivp

import oracle
from oracle import BC_PERIODIC, BC_ZERO, Physics

RK4_POLY = [1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24]


def rk4_amp(z):
    """Stability function of classical RK4 (Eqs. rk4_K1-rk4_final on y' = lambda y)."""
    return sum(c * z ** k for k, c in enumerate(RK4_POLY))


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def kappa_periodic(N, d):
    m = np.arange(N)
    return 4.0 / d ** 2 * np.sin(np.pi * m / N) ** 2


def kappa_zero(N, d):
    p = np.arange(1, N + 1)
    return 4.0 / d ** 2 * np.sin(np.pi * p / (2.0 * (N + 1))) ** 2


# ---------------------------------------------------------------- P1, P2, P3

@pytest.mark.parametrize("bcx,bcy", [(BC_PERIODIC, BC_PERIODIC), (BC_ZERO, BC_ZERO),
                                     (BC_PERIODIC, BC_ZERO), (BC_ZERO, BC_PERIODIC)])
def test_linear_modes_exact(bcx, bcy):
    """Linear case (g = g_r = R = 0, constant V, constant loss): discrete plane waves
    (periodic) and sine modes (zero boundary, DST-I) are exact eigenvectors of the
    five-point operator, so n RK4 steps equal R(lambda dt)^n per mode with
    lambda = -i[(hbar/2m) kappa + V0/hbar] - gamma/2 (Eq. 1, Sec. 3.2.8 stencil)."""
    nx, ny, dx, dy = 16, 12, 0.3, 0.25
    hbar, mass, V0, gam, dt, steps = 1.3, 0.8, 0.7, 0.1, 2e-3, 40
    ph = Physics(nx=nx, ny=ny, dx=dx, dy=dy, bc_x=bcx, bc_y=bcy, hbar=hbar, mass=mass,
                 gamma_c=gam)
    rng = np.random.default_rng(5)
    psi0 = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    V = np.full((ny, nx), V0)
    out, _ = oracle.rk4(ph, psi0[None], V=V, dt=dt, steps=steps)

    def fwd(a):
        a = scipy.fft.fft(a, axis=1) if bcx == BC_PERIODIC else scipy.fft.dst(a, type=1, axis=1)
        a = scipy.fft.fft(a, axis=0) if bcy == BC_PERIODIC else scipy.fft.dst(a, type=1, axis=0)
        return a

    def inv(a):
        a = scipy.fft.ifft(a, axis=0) if bcy == BC_PERIODIC else scipy.fft.idst(a, type=1, axis=0)
        a = scipy.fft.ifft(a, axis=1) if bcx == BC_PERIODIC else scipy.fft.idst(a, type=1, axis=1)
        return a

    kx = kappa_periodic(nx, dx) if bcx == BC_PERIODIC else kappa_zero(nx, dx)
    ky = kappa_periodic(ny, dy) if bcy == BC_PERIODIC else kappa_zero(ny, dy)
    kap = ky[:, None] + kx[None, :]
    lam = -1j * (hbar / (2 * mass) * kap + V0 / hbar) - gam / 2
    exact = inv(fwd(psi0) * rk4_amp(lam * dt) ** steps)
    assert rel(out[0], exact) < 1e-13


def test_norm_parseval_rk4_dissipation():
    """Hermitian linear run: the oracle's norm observable equals
    dxdy sum_k |c_k|^2 |R(-i w_k dt)|^(2n) (Parseval), where |R(i t)|^2 = 1 - t^6/72 + t^8/576."""
    nx = ny = 32
    dx = 0.2
    ph = Physics(nx=nx, ny=ny, dx=dx, dy=dx)
    rng = np.random.default_rng(6)
    psi0 = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    dt, steps = 0.01, 25  # large |w dt| so that the RK4 norm loss is visible
    out, _ = oracle.rk4(ph, psi0[None], dt=dt, steps=steps)
    kap = kappa_periodic(ny, dx)[:, None] + kappa_periodic(nx, dx)[None, :]
    w = 0.5 * kap
    th = w * dt
    amp2 = 1 - th ** 6 / 72 + th ** 8 / 576
    assert np.allclose(amp2, np.abs(rk4_amp(-1j * th)) ** 2, rtol=1e-14, atol=0)
    c = np.fft.fft2(psi0)
    expect = dx * dx * np.sum(np.abs(c) ** 2 * amp2 ** steps) / (nx * ny)
    got = oracle.observables(ph, out)["norm"][0]
    assert abs(got - expect) / expect < 1e-12
    # the loss is real and resolved: strictly below the initial norm
    assert got < dx * dx * np.sum(np.abs(psi0) ** 2) * (1 - 1e-4)


# ---------------------------------------------------------------- P4, P5

def _gauss_spread_error(n, L, t, dt):
    dx = L / n
    ph = Physics(nx=n, ny=n, dx=dx, dy=dx)
    x = (np.arange(n) - (n - 1) / 2) * dx
    X, Y = np.meshgrid(x, x, indexing="xy")
    r2 = X * X + Y * Y
    s0 = 1.0
    psi0 = np.exp(-r2 / (2 * s0 ** 2))
    out, _ = oracle.rk4(ph, psi0[None], dt=dt, steps=int(round(t / dt)))
    st2 = s0 ** 2 * (1 + (t / s0 ** 2) ** 2)
    rho = (s0 ** 2 / st2) * np.exp(-r2 / st2)
    return np.max(np.abs(np.abs(out[0]) ** 2 - rho))


def test_free_gaussian_spreading_second_order():
    """Free particle (V = g = 0): a Gaussian spreads as rho = (s0^2/st^2) exp(-r^2/st^2),
    st^2 = s0^2 (1 + (hbar t / m s0^2)^2).  The five-point Laplacian makes the error
    O(dx^2): halving dx cuts it about four times."""
    e1 = _gauss_spread_error(64, 16.0, 0.5, 2e-3)
    e2 = _gauss_spread_error(128, 16.0, 0.5, 2e-3)
    assert e1 < 2e-2
    assert 3.6 < e1 / e2 < 4.4


def _harmonic_error(n, L, t, dt):
    dx = L / n
    ph = Physics(nx=n, ny=n, dx=dx, dy=dx)
    x = (np.arange(n) - (n - 1) / 2) * dx
    X, Y = np.meshgrid(x, x, indexing="xy")
    r2 = X * X + Y * Y
    psi0 = np.exp(-r2 / 2) / np.sqrt(np.pi)
    out, _ = oracle.rk4(ph, psi0[None], V=0.5 * r2, dt=dt, steps=int(round(t / dt)))
    return np.max(np.abs(out[0] - psi0 * np.exp(-1j * t)))


def test_harmonic_ground_state_phase():
    """2D harmonic oscillator (hbar = m = omega = 1): pi^(-1/2) exp(-r^2/2) is stationary
    with energy 1, so psi(t) = psi0 exp(-i t); the spatial error is O(dx^2)."""
    e1 = _harmonic_error(64, 12.8, 1.0, 2e-3)
    e2 = _harmonic_error(128, 12.8, 1.0, 2e-3)
    assert e1 < 5e-3
    assert 3.6 < e1 / e2 < 4.4


# ---------------------------------------------------------------- P6, P7

def _scalar_ode_rk4(psi, n, dt, steps, V0, g, g_r, R, gam, gam_r, P, hbar):
    """The same uniform system as a 0-D ODE, in plain Python complex floats."""
    def f(p, m):
        rho = p.real * p.real + p.imag * p.imag
        h = (V0 + g * rho + g_r * m) * p
        return (-(1j / hbar) * h + 0.5 * (R * m - gam) * p, P - (gam_r + R * rho) * m)

    for _ in range(steps):
        k1 = f(psi, n)
        k2 = f(psi + 0.5 * dt * k1[0], n + 0.5 * dt * k1[1])
        k3 = f(psi + 0.5 * dt * k2[0], n + 0.5 * dt * k2[1])
        k4 = f(psi + dt * k3[0], n + dt * k3[1])
        psi = psi + (1.0 / 6.0) * (k1[0] + 2.0 * k2[0] + 2.0 * k3[0] + k4[0]) * dt
        n = n + (1.0 / 6.0) * (k1[1] + 2.0 * k2[1] + 2.0 * k3[1] + k4[1]) * dt
    return psi, n


def _uniform_physics(**kw):
    base = dict(nx=3, ny=2, dx=0.5, dy=0.7, reservoir=True, hbar=1.1, g=0.01, g_r=0.02,
                R=0.01, gamma_c=0.15, gamma_r=0.225)
    base.update(kw)
    return Physics(**base)


def test_uniform_state_equals_scalar_ode():
    """A uniform periodic state stays uniform (the Laplacian of a constant is exactly
    zero), so every cell must follow the 0-D RK4 of the pointwise terms of
    Eqs. PULSE_psi / PULSE_res."""
    ph = _uniform_physics()
    V0, P0, dt, steps = 0.3, 5.0, 0.05, 300
    psi0, n0 = 0.2 + 0.1j, 1.5
    out, nout = oracle.rk4(ph, np.full((1, 2, 3), psi0), np.full((1, 2, 3), n0),
                           V=np.full((2, 3), V0), P=np.full((1, 2, 3), P0), dt=dt, steps=steps)
    ps, ns = _scalar_ode_rk4(psi0, n0, dt, steps, V0, ph.g, ph.g_r, ph.R, ph.gamma_c, ph.gamma_r,
                             P0, ph.hbar)
    assert np.all(np.abs(out - ps) <= 1e-14 * abs(ps))
    assert np.all(np.abs(nout - ns) <= 1e-14 * abs(ns))


@pytest.mark.parametrize("ratio", [2.0, 0.5])
def test_driven_steady_state(ratio):
    """Homogeneous driven-dissipative steady state (Eqs. PULSE_psi/PULSE_res):
    above threshold n* = gamma_c/R and |psi|^2 = (P - P_th)/gamma_c with
    P_th = gamma_r gamma_c/R, the condensate rotating at (V0 + g rho* + g_r n*)/hbar;
    below threshold psi -> 0 and n -> P/gamma_r."""
    ph = _uniform_physics(hbar=1.0)
    pth = ph.gamma_r * ph.gamma_c / ph.R
    P0, V0, dt = ratio * pth, 0.1, 0.05
    out, nout = oracle.rk4(ph, np.full((1, 2, 3), 1e-3 + 0j), np.zeros((1, 2, 3)),
                           V=np.full((2, 3), V0), P=np.full((1, 2, 3), P0), dt=dt, steps=80000)
    rho, n = np.abs(out[0, 0, 0]) ** 2, nout[0, 0, 0]
    if ratio > 1:
        rho_s, n_s = (P0 - pth) / ph.gamma_c, ph.gamma_c / ph.R
        assert abs(n - n_s) / n_s < 1e-6
        assert abs(rho - rho_s) / rho_s < 1e-6
        nxt, _ = oracle.rk4(ph, out, nout, V=np.full((2, 3), V0), P=np.full((1, 2, 3), P0),
                            dt=dt, steps=1)
        omega = -np.angle(nxt[0, 0, 0] / out[0, 0, 0]) / dt
        assert abs(omega - (V0 + ph.g * rho_s + ph.g_r * n_s)) < 1e-6
        obs = oracle.observables(ph, out, nout, np.full((2, 3), V0), np.full((1, 2, 3), P0))
        assert obs["steady_res_density"] < 1e-6 and obs["steady_res_reservoir"] < 1e-6
    else:
        assert rho < 1e-30
        assert abs(n - P0 / ph.gamma_r) / (P0 / ph.gamma_r) < 1e-9


def test_reservoir_only_closed_form():
    """psi = 0: dn/dt = P - gamma_r n, so RK4 gives n_k = n_inf + (n0 - n_inf) R(-gamma_r dt)^k."""
    ph = _uniform_physics(nx=5, ny=4)
    rng = np.random.default_rng(7)
    P = rng.uniform(0, 3, (1, 4, 5))
    n0 = rng.uniform(0, 3, (1, 4, 5))
    dt, k = 0.3, 37
    _, nout = oracle.rk4(ph, np.zeros((1, 4, 5)), n0, P=P, dt=dt, steps=k)
    ninf = P / ph.gamma_r
    expect = ninf + (n0 - ninf) * rk4_amp(-ph.gamma_r * dt) ** k
    assert np.max(np.abs(nout - expect) / np.abs(expect)) < 1e-13


# ---------------------------------------------------------------- P8

def _breathing_run(dt, T=1.0, n=48, dx=0.25):
    ph = Physics(nx=n, ny=n, dx=dx, dy=dx, g=2.0)
    x = (np.arange(n) - (n - 1) / 2) * dx
    X, Y = np.meshgrid(x, x, indexing="xy")
    r2 = X * X + Y * Y
    V = 0.5 * r2
    psi0 = np.exp(-r2 / 3.0) * np.exp(1j * (0.7 * X + 0.2 * Y * Y))
    e0 = oracle.observables(ph, psi0[None], V=V)
    out, _ = oracle.rk4(ph, psi0[None], V=V, dt=dt, steps=int(round(T / dt)))
    e1 = oracle.observables(ph, out, V=V)
    return ph, out, V, e0, e1


def test_energy_norm_drift_fourth_order():
    """Hermitian nonlinear run (gamma = 0): norm and discrete energy are conserved by
    the semi-discrete equation; RK4's drift over a fixed time falls at least 16x when
    dt halves."""
    _, _, _, a0, a1 = _breathing_run(0.02)
    _, _, _, b0, b1 = _breathing_run(0.01)
    de_a, de_b = abs(a1["energy"] - a0["energy"]), abs(b1["energy"] - b0["energy"])
    dn_a, dn_b = abs(a1["norm"][0] - a0["norm"][0]), abs(b1["norm"][0] - b0["norm"][0])
    assert de_a > 1e-9 and dn_a > 1e-11  # drift resolved above rounding
    assert de_a / de_b > 16 * 0.9
    assert dn_a / dn_b > 16 * 0.9


@pytest.mark.parametrize("bcx,bcy", [(BC_PERIODIC, BC_PERIODIC), (BC_ZERO, BC_ZERO), (BC_ZERO, BC_PERIODIC)])
def test_kinetic_energy_summation_by_parts(bcx, bcy):
    """e_kin (sum over all grid links of (hbar^2/2m)|forward difference|^2) equals
    -(hbar^2/2m) dxdy sum Re(psi* Lap psi), Lap the five-point stencil of Sec. 3.2.8
    applied with the same boundary rule."""
    nx, ny, dx, dy, hbar, mass = 9, 7, 0.4, 0.3, 1.2, 0.7
    ph = Physics(nx=nx, ny=ny, dx=dx, dy=dy, bc_x=bcx, bc_y=bcy, hbar=hbar, mass=mass)
    rng = np.random.default_rng(8)
    psi = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))

    def shift(a, s, axis, bc):
        if bc == BC_PERIODIC:
            return np.roll(a, s, axis=axis)
        out = np.zeros_like(a)
        if axis == 1:
            if s > 0:
                out[:, s:] = a[:, :-s]
            else:
                out[:, :s] = a[:, -s:]
        else:
            if s > 0:
                out[s:, :] = a[:-s, :]
            else:
                out[:s, :] = a[-s:, :]
        return out

    lap = ((shift(psi, 1, 1, bcx) + shift(psi, -1, 1, bcx) - 2 * psi) / dx ** 2
           + (shift(psi, 1, 0, bcy) + shift(psi, -1, 0, bcy) - 2 * psi) / dy ** 2)
    expect = -(hbar ** 2 / (2 * mass)) * dx * dy * np.sum(np.real(np.conj(psi) * lap))
    got = oracle.observables(ph, psi[None])["e_kin"]
    assert abs(got - expect) / abs(expect) < 1e-13


def test_plane_wave_energy_closed_form():
    """Plane wave exp(i k x) on a periodic grid: e_kin = (hbar^2/2m) A (4/dx^2) sin^2(k dx/2),
    e_int = (g/2) A, e_pot = V0 A, norm = A (A the domain area), steady residual 0."""
    nx, ny, dx, dy = 24, 10, 0.3, 0.4
    m = 5
    k = 2 * np.pi * m / (nx * dx)
    ph = Physics(nx=nx, ny=ny, dx=dx, dy=dy, g=0.9)
    x = np.arange(nx) * dx
    psi = np.tile(np.exp(1j * k * x), (ny, 1))
    o = oracle.observables(ph, psi[None], V=np.full((ny, nx), 0.25))
    A = nx * ny * dx * dy
    assert abs(o["norm"][0] - A) < 1e-12 * A
    assert abs(o["e_kin"] - 0.5 * A * 4 / dx ** 2 * np.sin(k * dx / 2) ** 2) < 1e-12 * o["e_kin"]
    assert abs(o["e_int"] - 0.45 * A) < 1e-12 * A
    assert abs(o["e_pot"] - 0.25 * A) < 1e-12 * A
    assert abs(o["max_density"] - 1) < 1e-14
    assert o["steady_res_density"] < 1e-12


# ---------------------------------------------------------------- P9: brute force

def _d2(N, bc):
    D = -2 * np.eye(N) + np.eye(N, k=1) + np.eye(N, k=-1)
    if bc == BC_PERIODIC:
        D[0, -1] += 1
        D[-1, 0] += 1
    return D


def _d1(N, bc):
    D = (np.eye(N, k=1) - np.eye(N, k=-1)) / 2
    if bc == BC_PERIODIC:
        D[-1, 0] += 0.5
        D[0, -1] -= 0.5
    return D


def _dense_rhs(ph, psi, n, V, P):
    """Right-hand side built from dense difference matrices (Kronecker products of
    1-D matrices, the sparse-matrix formulation of Sec. 3.1) and matrix-vector
    products, applied to flattened fields (index j*nx + i)."""
    nx, ny = ph.nx, ph.ny
    Ix, Iy = np.eye(nx), np.eye(ny)
    Dxx = np.kron(Iy, _d2(nx, ph.bc_x)) / ph.dx ** 2
    Dyy = np.kron(_d2(ny, ph.bc_y), Ix) / ph.dy ** 2
    Dxy = np.kron(_d1(ny, ph.bc_y), _d1(nx, ph.bc_x)) / (ph.dx * ph.dy)
    C = ph.components
    ps = psi.reshape(C, -1)
    v = np.zeros(nx * ny) if V is None else V.ravel()
    fp = np.zeros_like(ps)
    fn = None if n is None else np.zeros((C, nx * ny))
    for c in range(C):
        o = C - 1 - c
        rho = np.abs(ps[c]) ** 2
        rho_o = np.abs(ps[o]) ** 2 if C == 2 else 0
        nn = n.reshape(C, -1)[c] if ph.reservoir else 0
        H = -(ph.hbar ** 2 / (2 * ph.mass)) * (Dxx + Dyy) @ ps[c] + (v + ph.g * rho + ph.g_x * rho_o + ph.g_r * nn) * ps[c]
        if C == 2:
            sgn = 1 if c == 0 else -1
            H = H + ph.delta_lt * ((Dxx - Dyy) @ ps[o] - 2j * sgn * (Dxy @ ps[o]))
        fp[c] = -(1j / ph.hbar) * H + 0.5 * (ph.R * nn - ph.gamma_c) * ps[c]
        if ph.reservoir:
            fn[c] = P.reshape(C, -1)[c] - (ph.gamma_r + ph.R * rho) * nn
    return fp.reshape(psi.shape), (None if fn is None else fn.reshape(psi.shape))


def _dense_rk4(ph, psi, n, V, P, dt, steps):
    for _ in range(steps):
        k1 = _dense_rhs(ph, psi, n, V, P)
        k2 = _dense_rhs(ph, psi + 0.5 * dt * k1[0], None if n is None else n + 0.5 * dt * k1[1], V, P)
        k3 = _dense_rhs(ph, psi + 0.5 * dt * k2[0], None if n is None else n + 0.5 * dt * k2[1], V, P)
        k4 = _dense_rhs(ph, psi + dt * k3[0], None if n is None else n + dt * k3[1], V, P)
        psi = psi + dt / 6 * (k1[0] + 2 * k2[0] + 2 * k3[0] + k4[0])
        if n is not None:
            n = n + dt / 6 * (k1[1] + 2 * k2[1] + 2 * k3[1] + k4[1])
    return psi, n


@pytest.mark.parametrize("comps,res", [(1, False), (1, True), (2, False), (2, True)])
@pytest.mark.parametrize("bcx,bcy", [(BC_PERIODIC, BC_PERIODIC), (BC_ZERO, BC_ZERO), (BC_ZERO, BC_PERIODIC)])
@pytest.mark.parametrize("shape", [(3, 4), (8, 5)])
def test_dense_matrix_brute_force(comps, res, bcx, bcy, shape):
    nx, ny = shape
    ph = Physics(nx=nx, ny=ny, dx=0.35, dy=0.3, bc_x=bcx, bc_y=bcy, components=comps,
                 reservoir=res, hbar=0.9, mass=1.3, g=0.7, g_x=-0.2, g_r=0.3, R=0.2,
                 gamma_c=0.1, gamma_r=0.25, delta_lt=0.15 if comps == 2 else 0.0)
    rng = np.random.default_rng(9 + nx + 10 * comps)
    psi = rng.standard_normal((comps, ny, nx)) + 1j * rng.standard_normal((comps, ny, nx))
    n = rng.uniform(0, 1, (comps, ny, nx)) if res else None
    P = rng.uniform(0, 1, (comps, ny, nx)) if res else None
    V = rng.uniform(-1, 1, (ny, nx))
    f_o, fn_o = oracle.rhs(ph, psi, n, V, P)
    f_d, fn_d = _dense_rhs(ph, psi, n, V, P)
    assert rel(f_o, f_d) < 1e-13
    if res:
        assert rel(fn_o, fn_d) < 1e-13
    out, nout = oracle.rk4(ph, psi, n, V, P, dt=0.01, steps=10)
    ref, nref = _dense_rk4(ph, psi, n, V, P, 0.01, 10)
    assert rel(out, ref) < 1e-13
    if res:
        assert rel(nout, nref) < 1e-13


@pytest.mark.parametrize("bc", [BC_PERIODIC, BC_ZERO])
def test_linear_operator_hermitian(bc):
    """With gamma = R = 0 and no reservoir the linear part of the right-hand side is
    -(i/hbar) H with H Hermitian, including the TE-TM coupling (J_- = J_+^dagger).
    H is assembled column by column from the oracle itself."""
    nx, ny = 5, 4
    ph = Physics(nx=nx, ny=ny, dx=0.3, dy=0.45, bc_x=bc, bc_y=bc, components=2, hbar=1.2,
                 mass=0.9, delta_lt=0.2)
    V = np.random.default_rng(10).uniform(-1, 1, (ny, nx))
    M = 2 * nx * ny
    H = np.zeros((M, M), complex)
    for q in range(M):
        e = np.zeros(M, complex)
        e[q] = 1.0
        f, _ = oracle.rhs(ph, e.reshape(2, ny, nx), V=V)
        H[:, q] = 1j * ph.hbar * f.ravel()
    assert np.max(np.abs(H - H.conj().T)) < 1e-12 * np.max(np.abs(H))
    assert np.max(np.abs(H[: nx * ny, nx * ny:])) > 0.1  # the coupling is present


def test_tetm_plane_wave_symbol():
    """J_+ = Delta_LT (d_x - i d_y)^2 acting on exp(i k.r): the discrete symbol is
    Delta_LT (-kx2 + ky2 + 2 i sx sy), kx2 = (4/dx^2) sin^2(kx dx/2), sx = sin(kx dx)/dx,
    whose continuum limit Delta_LT (-kx^2 + ky^2 + 2 i kx ky) = -Delta_LT (kx - i ky)^2
    fixes the sign of the mixed term.  J_- has the conjugate mixed term."""
    nx, ny, dx, dy, d = 64, 48, 0.1, 0.125, 0.3
    ph = Physics(nx=nx, ny=ny, dx=dx, dy=dy, components=2, delta_lt=d)
    kx, ky = 2 * np.pi * 2 / (nx * dx), 2 * np.pi * 1 / (ny * dy)
    X, Y = np.meshgrid(np.arange(nx) * dx, np.arange(ny) * dy, indexing="xy")
    wave = np.exp(1j * (kx * X + ky * Y))
    kx2, ky2 = 4 / dx ** 2 * np.sin(kx * dx / 2) ** 2, 4 / dy ** 2 * np.sin(ky * dy / 2) ** 2
    sx, sy = np.sin(kx * dx) / dx, np.sin(ky * dy) / dy
    # psi_+ = 0, psi_- = wave: f_+ = -(i/hbar) J_+ psi_-  (kinetic part of psi_+ vanishes)
    f, _ = oracle.rhs(ph, np.stack([np.zeros_like(wave), wave]))
    sym_plus = d * (-kx2 + ky2 + 2j * sx * sy)
    assert rel(f[0], -1j * sym_plus * wave) < 1e-13
    sym_minus = d * (-kx2 + ky2 - 2j * sx * sy)
    f, _ = oracle.rhs(ph, np.stack([wave, np.zeros_like(wave)]))
    assert rel(f[1], -1j * sym_minus * wave) < 1e-13
    # continuum limit of the symbol, to O(dx^2)
    cont = d * (-kx ** 2 + ky ** 2 + 2j * kx * ky)
    assert abs(sym_plus - cont) / abs(cont) < 0.05
    assert abs(cont - (-d * (kx - 1j * ky) ** 2)) < 1e-12


# ---------------------------------------------------------------- P10

def test_mirror_symmetry_bitwise():
    """Mirror-symmetric inputs (x -> -x and y -> -y about the grid centre) stay mirror
    symmetric bit for bit: the stencil only swaps the order of commutative additions."""
    n = 17
    for bc in (BC_PERIODIC, BC_ZERO):
        ph = Physics(nx=n, ny=n - 4, dx=0.3, dy=0.3, bc_x=bc, bc_y=bc, reservoir=True, g=1.0,
                     g_r=0.5, R=0.1, gamma_c=0.2, gamma_r=0.3)
        rng = np.random.default_rng(11)
        a = rng.standard_normal((n - 4, n)) + 1j * rng.standard_normal((n - 4, n))
        a = a + a[:, ::-1]
        a = a + a[::-1, :]
        V = rng.uniform(0, 1, (n - 4, n))
        V = V + V[:, ::-1]
        V = V + V[::-1, :]
        P = np.abs(a) ** 2
        out, nout = oracle.rk4(ph, a[None], np.zeros((1, n - 4, n)), V, P[None], dt=0.01, steps=20)
        assert np.array_equal(out[0], out[0][:, ::-1]) and np.array_equal(out[0], out[0][::-1, :])
        assert np.array_equal(nout[0], nout[0][:, ::-1])


def test_spinor_mirror_with_component_swap():
    """The map y -> -y together with psi_+ <-> psi_- leaves the TE-TM terms invariant
    when V is symmetric in y (the mixed derivative changes sign, and so does the
    sign of its coefficient between the two components)."""
    nx, ny = 10, 9
    ph = Physics(nx=nx, ny=ny, dx=0.3, dy=0.3, bc_x=BC_ZERO, bc_y=BC_ZERO, components=2, g=1.0,
                 g_x=-0.1, delta_lt=0.1)
    rng = np.random.default_rng(12)
    p = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    psi = np.stack([p, p[::-1, :]])
    V = rng.uniform(0, 1, (ny, nx))
    V = V + V[::-1, :]
    out, _ = oracle.rk4(ph, psi, V=V, dt=0.01, steps=10)
    assert np.max(np.abs(out[1] - out[0][::-1, :])) < 1e-15 * np.max(np.abs(out))


# ---------------------------------------------------------------- P11: Dormand-Prince

def _tableau(golden_dir):
    with open(os.path.join(golden_dir, "dopri5_tableau.json")) as f:
        t = json.load(f)
    fr = lambda p: Fraction(p[0], p[1])
    A = [[fr(x) for x in row] + [Fraction(0)] * (7 - len(row)) for row in t["a"]]
    return A, [fr(x) for x in t["b"]], [fr(x) for x in t["bhat"]], [fr(x) for x in t["c"]], fr(t["stability_z6"])


def _series(A, w, terms=8):
    """Coefficients of 1 + z w^T (I - zA)^-1 1 (the stability function)."""
    coef, v = [Fraction(1)], [Fraction(1)] * 7
    for _ in range(terms - 1):
        coef.append(sum(x * y for x, y in zip(w, v)))
        v = [sum(A[i][j] * v[j] for j in range(7)) for i in range(7)]
    return coef


def test_dopri5_tableau_order_conditions(golden_dir):
    """The stored tableau satisfies the 17 order conditions through order 5 (b) and
    through order 4 (bhat), its row sums equal c, and its stability function is the
    degree-5 Taylor polynomial of exp plus z^6/600."""
    A, b, bh, c, z6 = _tableau(golden_dir)
    S = range(7)
    assert all(sum(A[i]) == c[i] for i in S)
    dot = lambda u, v: sum(x * y for x, y in zip(u, v))
    mv = lambda v: [dot(A[i], v) for i in S]
    c2 = [x * x for x in c]
    Ac, Acc = mv(c), mv(c2)
    conds = [([1] * 7, 1, 1), (c, Fraction(1, 2), 2), (c2, Fraction(1, 3), 3), (Ac, Fraction(1, 6), 3),
             ([x ** 3 for x in c], Fraction(1, 4), 4), ([x * y for x, y in zip(c, Ac)], Fraction(1, 8), 4),
             (Acc, Fraction(1, 12), 4), (mv(Ac), Fraction(1, 24), 4),
             ([x ** 4 for x in c], Fraction(1, 5), 5), ([x * x * y for x, y in zip(c, Ac)], Fraction(1, 10), 5),
             ([x * y for x, y in zip(c, Acc)], Fraction(1, 15), 5), ([x * y for x, y in zip(c, mv(Ac))], Fraction(1, 30), 5),
             ([y * y for y in Ac], Fraction(1, 20), 5), (mv([x ** 3 for x in c]), Fraction(1, 20), 5),
             (mv([x * y for x, y in zip(c, Ac)]), Fraction(1, 40), 5), (mv(Acc), Fraction(1, 60), 5),
             (mv(mv(Ac)), Fraction(1, 120), 5)]
    for v, rhs, order in conds:
        assert dot(b, v) == rhs
        if order <= 4:
            assert dot(bh, v) == rhs
    R = _series(A, b)
    assert R[:6] == [Fraction(1, math.factorial(k)) for k in range(6)] and R[6] == z6 and R[7] == 0


def test_dopri5_step_linear_stability_polynomial(golden_dir):
    """One oracle step on y' = lambda y (uniform state, constant V and loss) multiplies
    by R(lambda dt); the embedded error is (R - Rhat)(lambda dt) y, with R, Rhat the
    stability functions of the stored tableau."""
    A, b, bh, _, _ = _tableau(golden_dir)
    R, Rh = _series(A, b, 8), _series(A, bh, 8)
    ph = Physics(nx=2, ny=2, dx=1.0, dy=1.0, gamma_c=0.8)
    V0, dt = 1.7, 0.35
    lam = -1j * V0 - 0.4
    z = lam * dt
    y0 = 0.3 - 0.2j
    out, _, err, _ = oracle.dopri5_step(ph, np.full((1, 2, 2), y0), V=np.full((2, 2), V0), dt=dt)
    pr = sum(float(cf) * z ** k for k, cf in enumerate(R))
    prh = sum(float(cf) * z ** k for k, cf in enumerate(Rh))
    assert abs(out[0, 0, 0] - pr * y0) < 1e-15
    assert abs(err[0, 0, 0] - (pr - prh) * y0) < 1e-15


def _uniform_ode_reference(ph, psi0, n0, V0, P0, T):
    def f(t, u):
        p = u[0] + 1j * u[1]
        m = u[2]
        rho = abs(p) ** 2
        dp = -(1j / ph.hbar) * (V0 + ph.g * rho + ph.g_r * m) * p + 0.5 * (ph.R * m - ph.gamma_c) * p
        return [dp.real, dp.imag, P0 - (ph.gamma_r + ph.R * rho) * m]

    s = solve_ivp(f, (0, T), [psi0.real, psi0.imag, n0], method="DOP853", rtol=1e-13, atol=1e-15)
    u = s.y[:, -1]
    return u[0] + 1j * u[1], u[2]


def test_dopri5_fifth_order_convergence():
    """Fixed-step Dormand-Prince on a nonlinear uniform reservoir system converges
    with order 5 (solution) and its error estimate scales as dt^5 (order-4 embedding)."""
    ph = _uniform_physics(nx=2, ny=2, g=0.3, g_r=0.2, R=0.4, gamma_c=0.5, gamma_r=0.6)
    V0, P0, T = 0.2, 2.0, 2.0
    psi0, n0 = 0.5 + 0.3j, 1.0
    ref_p, ref_n = _uniform_ode_reference(ph, psi0, n0, V0, P0, T)
    errs, ests = [], []
    for steps in (16, 32, 64):
        dt = T / steps
        p, m = np.full((1, 2, 2), psi0), np.full((1, 2, 2), n0)
        first_err = None
        for _ in range(steps):
            p, m, e, _ = oracle.dopri5_step(ph, p, m, V=np.full((2, 2), V0), P=np.full((1, 2, 2), P0), dt=dt)
            if first_err is None:
                first_err = abs(e[0, 0, 0])
        errs.append(abs(p[0, 0, 0] - ref_p) + abs(m[0, 0, 0] - ref_n))
        ests.append(first_err)
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(4.7 < s < 5.5 for s in slopes), slopes
    est_slopes = [math.log2(ests[i] / ests[i + 1]) for i in range(2)]
    assert all(4.5 < s < 5.5 for s in est_slopes), est_slopes


def test_dopri5_controller_rules():
    """Adaptive runs: every attempt with err <= 1 is accepted and every other one is
    rejected; the next step is dt clamp(0.9 err^(-1/5), 0.2, 5) (at most 1 right after a
    rejection); tightening the tolerance 32x cuts the global error by roughly that factor."""
    ph = _uniform_physics(nx=2, ny=2, g=0.3, g_r=0.2, R=0.4, gamma_c=0.5, gamma_r=0.6)
    V0, P0 = 0.2, 2.0
    psi0, n0 = 0.5 + 0.3j, 1.0
    V, P = np.full((2, 2), V0), np.full((1, 2, 2), P0)
    psi, n, ctrl = oracle.dopri5(ph, np.full((1, 2, 2), psi0), np.full((1, 2, 2), n0), V, P,
                                 rtol=1e-6, atol=1e-6, accepted=30,
                                 ctrl=oracle.Controller(dt=0.9), history_cap=200)
    assert ctrl.accepted == 30 and ctrl.rejected >= 1  # dt0 = 0.9 is too large
    last_rej = False
    for k, (dt, err) in enumerate(ctrl.history):
        fmax = 1.0 if last_rej else 5.0
        fac = min(fmax, max(0.2, 0.9 * err ** -0.2)) if err > 0 else fmax
        if k + 1 < len(ctrl.history):
            assert abs(ctrl.history[k + 1][0] - dt * fac) < 1e-15 * dt
        last_rej = err > 1.0
    errs = []
    for tol in (1e-6, 1e-6 / 32):
        p, m, c = _dopri_to_time(ph, psi0, n0, V, P, tol, 2.0)
        ref_p, ref_n = _uniform_ode_reference(ph, psi0, n0, V0, P0, c.t)
        errs.append(abs(p - ref_p) + abs(m - ref_n))
    assert 8 < errs[0] / errs[1] < 200


def _dopri_to_time(ph, psi0, n0, V, P, tol, T):
    p, m = np.full((1, 2, 2), psi0), np.full((1, 2, 2), n0)
    c = oracle.Controller(dt=1e-3)
    while c.t < T:
        p, m, c = oracle.dopri5(ph, p, m, V, P, rtol=tol, atol=tol, accepted=1, ctrl=c)
        assert c.status == 0 and c.accepted < 100000
    return p[0, 0, 0], m[0, 0, 0], c


def test_dopri5_dt_underflow_status():
    """A step size below dt_min stops the run with status -5 and no state change."""
    ph = _uniform_physics(nx=2, ny=2)
    psi = np.full((1, 2, 2), 0.1 + 0j)
    n = np.full((1, 2, 2), 1.0)
    out, nout, c = oracle.dopri5(ph, psi, n, None, np.full((1, 2, 2), 1.0), rtol=1e-30,
                                 atol=1e-30, dt_min=1e-8, accepted=5, ctrl=oracle.Controller(dt=1e-3))
    assert c.status == -5 and c.accepted == 0
    assert np.array_equal(out, psi) and np.array_equal(nout, n)
