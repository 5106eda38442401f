"""Pins of the oracle's observables that the dynamics fix: the cross-spin energy,
the TE-TM energy, the reservoir-coupling energy and the reservoir total (Eq. 1;
Sec. 5, Eqs. PULSE_psi / PULSE_res).

Three independent routes, none of which re-types the observable's formula:

* Hamilton's equation.  In the conservative case (gamma_c = R = 0, reservoir frozen
  as a static potential) the right-hand side is -(i/hbar) dE/dpsi*: the directional
  derivative of the oracle's total energy along any eta equals
  2 dxdy Re<eta, i hbar f(psi)>, with f the oracle's right-hand side (which the
  dense-matrix brute force pins on its own).  E(psi + eps eta) is a quartic
  polynomial in eps, so the five-point difference below is exact up to rounding.
* Conservation.  The energy of a conservative spinor run (g, g_x, Delta_LT != 0), and of
  a run with a frozen reservoir (g_r n a static potential), drifts at RK4's fourth
  order: halving dt cuts the drift at least 16x.  With P = gamma_r = gamma_c = 0 the
  gain R n rho moves particles between condensate and reservoir, so norm + reservoir
  total is conserved the same way.
* Closed forms.  A uniform reservoir holds n times the domain area; with psi = 0 it
  relaxes as n_inf + (n0 - n_inf) R(-gamma_r dt)^k per step (exact discrete solution).
* The dense quadratic form.  With g = g_x = 0 the energy equals dxdy <psi|H|psi>, H
  assembled from Kronecker products of 1-D difference matrices.
"""
import numpy as np
import pytest

import oracle
from oracle import BC_PERIODIC, BC_ZERO, Physics
from test_oracle_imag_pins import dense_h

RK4_POLY = [1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24]


def rk4_amp(z):
    return sum(c * z ** k for k, c in enumerate(RK4_POLY))


def _energy(ph, psi, n, V, P):
    return oracle.observables(ph, psi, n, V, P)["energy"]


def _directional_derivative(ph, psi, eta, n, V, P, h=1e-3):
    """d/deps E(psi + eps eta) at eps = 0; exact for a polynomial of degree <= 4."""
    e = {s: _energy(ph, psi + s * h * eta, n, V, P) for s in (-2, -1, 1, 2)}
    return (e[-2] - 8 * e[-1] + 8 * e[1] - e[2]) / (12 * h)


GRADIENT_CASES = {
    "spinor_periodic": dict(nx=7, ny=6, dx=0.35, dy=0.3, bc_x=BC_PERIODIC, bc_y=BC_PERIODIC,
                            components=2, g=0.8, g_x=-0.35, delta_lt=0.12, hbar=1.1, mass=0.9),
    "spinor_zero": dict(nx=6, ny=7, dx=0.3, dy=0.4, bc_x=BC_ZERO, bc_y=BC_ZERO,
                        components=2, g=0.5, g_x=0.6, delta_lt=-0.2, hbar=0.8, mass=1.3),
    "spinor_mixed": dict(nx=8, ny=5, dx=0.25, dy=0.35, bc_x=BC_ZERO, bc_y=BC_PERIODIC,
                         components=2, g=1.2, g_x=-0.1, delta_lt=0.1),
    "spinor_tetm_only": dict(nx=6, ny=6, dx=0.3, dy=0.3, bc_x=BC_PERIODIC, bc_y=BC_ZERO,
                             components=2, delta_lt=0.25),
    "spinor_cross_only": dict(nx=5, ny=6, dx=0.3, dy=0.3, components=2, g_x=0.9),
    "scalar_frozen_reservoir": dict(nx=7, ny=5, dx=0.3, dy=0.45, bc_x=BC_ZERO, reservoir=True,
                                    g=0.7, g_r=1.4, gamma_r=0.3),
    "spinor_frozen_reservoir": dict(nx=5, ny=6, dx=0.4, dy=0.3, bc_y=BC_ZERO, components=2,
                                    reservoir=True, g=0.4, g_x=-0.2, g_r=0.9, delta_lt=0.15),
}


@pytest.mark.parametrize("case", sorted(GRADIENT_CASES))
def test_energy_is_the_hamiltonian_of_the_rhs(case):
    """dE/d eps along eta = 2 dxdy Re<eta, i hbar f(psi)> (conservative right-hand side:
    gamma_c = R = 0, so every term of f_psi is -(i/hbar) times the derivative of one
    energy term)."""
    ph = Physics(**GRADIENT_CASES[case])
    rng = np.random.default_rng(100 + sorted(GRADIENT_CASES).index(case))
    shape = (ph.components, ph.ny, ph.nx)
    psi = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    V = rng.uniform(-1, 1, (ph.ny, ph.nx))
    n = rng.uniform(0, 2, shape) if ph.reservoir else None
    P = rng.uniform(0, 1, shape) if ph.reservoir else None
    f_psi, _ = oracle.rhs(ph, psi, n, V, P)
    dA = ph.dx * ph.dy
    for trial in range(3):
        eta = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        got = _directional_derivative(ph, psi, eta, n, V, P)
        expect = 2 * dA * np.real(np.vdot(eta, 1j * ph.hbar * f_psi))
        scale = 2 * dA * np.linalg.norm(eta) * np.linalg.norm(ph.hbar * f_psi)
        assert abs(got - expect) < 1e-10 * scale, (case, trial, got, expect)


@pytest.mark.parametrize("bc", [BC_PERIODIC, BC_ZERO])
def test_linear_spinor_energy_is_the_dense_quadratic_form(bc):
    """g = g_x = 0: e_kin + e_pot + e_tetm = dxdy <psi|H|psi> with the Hermitian H of the
    kinetic, potential and TE-TM terms assembled from Kronecker products; e_int,
    e_cross vanish."""
    ph = Physics(nx=6, ny=5, dx=0.3, dy=0.4, bc_x=bc, bc_y=bc, components=2, hbar=1.1, mass=0.8,
                 delta_lt=0.17)
    rng = np.random.default_rng(41 + bc)
    V = rng.uniform(-1, 1, (ph.ny, ph.nx))
    psi = rng.standard_normal((2, ph.ny, ph.nx)) + 1j * rng.standard_normal((2, ph.ny, ph.nx))
    H = dense_h(ph, V)
    u = psi.ravel()
    quad = ph.dx * ph.dy * np.real(np.vdot(u, H @ u))
    o = oracle.observables(ph, psi, V=V)
    assert o["e_int"] == 0.0 and o["e_cross"] == 0.0
    assert o["energy"] == pytest.approx(quad, rel=1e-13)
    # the TE-TM part alone: the off-diagonal blocks of H
    N = ph.nx * ph.ny
    off = np.zeros_like(H)
    off[:N, N:] = H[:N, N:]
    off[N:, :N] = H[N:, :N]
    assert o["e_tetm"] == pytest.approx(ph.dx * ph.dy * np.real(np.vdot(u, off @ u)), rel=1e-12)


def _drift(ph, psi0, n0, V, P, dt, T, key):
    o0 = oracle.observables(ph, psi0, n0, V, P)
    psi, n = oracle.rk4(ph, psi0, n0, V, P, dt=dt, steps=int(round(T / dt)))
    o1 = oracle.observables(ph, psi, n, V, P)
    return abs(key(o1) - key(o0)), o0


def _spinor_start(ph, seed):
    rng = np.random.default_rng(seed)
    x = (np.arange(ph.nx) - (ph.nx - 1) / 2) * ph.dx
    y = (np.arange(ph.ny) - (ph.ny - 1) / 2) * ph.dy
    X, Y = np.meshgrid(x, y, indexing="xy")
    env = np.exp(-(X ** 2 + Y ** 2) / 4.0)
    psi = np.stack([env * np.exp(1j * (0.6 * X + 0.3 * Y)), 0.7 * env * np.exp(-1j * 0.4 * X * Y)])
    psi = psi * (1 + 0.05 * rng.standard_normal(psi.shape))
    return psi


def test_spinor_energy_conserved_at_fourth_order():
    """Conservative spinor with g, g_x and Delta_LT != 0: the total energy (e_cross and
    e_tetm included) is an invariant of the semi-discrete equation, so its RK4 drift
    over a fixed time falls >= 16x when dt halves; with e_cross or e_tetm dropped the
    sum is not conserved at all."""
    ph = Physics(nx=24, ny=24, dx=0.35, dy=0.35, bc_x=BC_ZERO, bc_y=BC_PERIODIC, components=2,
                 g=1.5, g_x=-0.8, delta_lt=0.3)
    psi0 = _spinor_start(ph, 5)
    x = (np.arange(ph.nx) - (ph.nx - 1) / 2) * ph.dx
    V = 0.3 * (x[None, :] ** 2 + x[:, None] ** 2) / 4
    da, o0 = _drift(ph, psi0, None, V, None, 0.02, 0.8, lambda o: o["energy"])
    db, _ = _drift(ph, psi0, None, V, None, 0.01, 0.8, lambda o: o["energy"])
    assert abs(o0["e_cross"]) > 0.05 * abs(o0["energy"]) and abs(o0["e_tetm"]) > 1e-3 * abs(o0["energy"])
    assert da > 1e-12 and da / db > 16 * 0.9, (da, db)


def test_frozen_reservoir_energy_conserved_at_fourth_order():
    """R = gamma_r = P = gamma_c = 0: n never changes and g_r n acts as a static potential,
    so the energy with e_res is conserved at RK4's order."""
    ph = Physics(nx=20, ny=22, dx=0.3, dy=0.4, bc_x=BC_PERIODIC, bc_y=BC_ZERO, reservoir=True,
                 g=0.9, g_r=2.5)
    rng = np.random.default_rng(9)
    x = (np.arange(ph.nx) - (ph.nx - 1) / 2) * ph.dx
    y = (np.arange(ph.ny) - (ph.ny - 1) / 2) * ph.dy
    X, Y = np.meshgrid(x, y, indexing="xy")
    psi0 = (np.exp(-(X ** 2 + Y ** 2) / 3.0) * np.exp(0.8j * X))[None]
    n0 = (1.0 + 0.5 * np.cos(1.3 * X) * np.sin(0.9 * Y) + 0.1 * rng.uniform(0, 1, X.shape))[None]
    P = np.zeros_like(n0)
    da, o0 = _drift(ph, psi0, n0, None, P, 0.02, 1.0, lambda o: o["energy"])
    db, _ = _drift(ph, psi0, n0, None, P, 0.01, 1.0, lambda o: o["energy"])
    assert abs(o0["e_res"]) > 0.2 * abs(o0["energy"])
    assert da > 1e-12 and da / db > 16 * 0.9, (da, db)


def test_particle_exchange_conserves_norm_plus_reservoir():
    """P = gamma_r = gamma_c = 0: d rho/dt carries + R n rho and dn/dt carries - R n rho, so
    dxdy sum(rho + n) is an invariant; its RK4 drift falls >= 16x when dt halves
    (dxdy != 1, so the reservoir total's area factor matters)."""
    ph = Physics(nx=18, ny=16, dx=0.5, dy=0.7, bc_x=BC_ZERO, reservoir=True, g=0.3, g_r=0.5, R=0.4)
    rng = np.random.default_rng(12)
    psi0 = (0.8 + 0.3 * rng.uniform(-1, 1, (1, ph.ny, ph.nx))) * np.exp(1j * rng.uniform(0, 1, (1, ph.ny, ph.nx)))
    n0 = 1.0 + rng.uniform(0, 1, (1, ph.ny, ph.nx))
    P = np.zeros_like(n0)
    tot = lambda o: o["norm"][0] + o["reservoir"]   # noqa: E731
    da, o0 = _drift(ph, psi0, n0, None, P, 0.04, 2.0, tot)
    db, _ = _drift(ph, psi0, n0, None, P, 0.02, 2.0, tot)
    # the exchange itself is large: the norm alone changes by a sizeable fraction
    psi1, n1 = oracle.rk4(ph, psi0, n0, None, P, dt=0.04, steps=50)
    o1 = oracle.observables(ph, psi1, n1, None, P)
    assert abs(o1["norm"][0] - o0["norm"][0]) > 0.3 * o0["norm"][0]
    assert da > 1e-13 and da / db > 16 * 0.9, (da, db)


def test_reservoir_total_closed_forms():
    """A uniform reservoir n0 holds n0 times the domain area; with psi = 0 and uniform P it
    follows the exact discrete relaxation n_inf + (n0 - n_inf) R(-gamma_r dt)^k."""
    ph = Physics(nx=11, ny=9, dx=0.3, dy=0.7, components=2, reservoir=True, gamma_r=0.6, R=0.2)
    area = ph.nx * ph.dx * ph.ny * ph.dy
    n0, Pv, dt, k = 2.5, 0.9, 0.05, 13
    psi = np.zeros((2, ph.ny, ph.nx), complex)
    n = np.full((2, ph.ny, ph.nx), n0)
    P = np.full((2, ph.ny, ph.nx), Pv)
    o = oracle.observables(ph, psi, n, None, P)
    assert o["reservoir"] == pytest.approx(2 * n0 * area, rel=1e-14)
    _, nk = oracle.rk4(ph, psi, n, None, P, dt=dt, steps=k)
    ninf = Pv / ph.gamma_r
    expect = 2 * area * (ninf + (n0 - ninf) * rk4_amp(-ph.gamma_r * dt) ** k)
    assert oracle.observables(ph, psi, nk, None, P)["reservoir"] == pytest.approx(expect, rel=1e-13)


def test_uniform_state_energy_terms():
    """Uniform spinor amplitudes a+, a- and reservoir n on a periodic grid: no gradient and
    no TE-TM term (every difference of a constant is 0), and the densities' energies are
    the point values times the area."""
    ph = Physics(nx=8, ny=6, dx=0.4, dy=0.25, components=2, reservoir=True, g=0.7, g_x=-0.3, g_r=1.1,
                 delta_lt=0.2)
    area = ph.nx * ph.dx * ph.ny * ph.dy
    a = np.array([0.9 + 0.4j, -0.3 + 1.1j])
    psi = np.ones((2, ph.ny, ph.nx)) * a[:, None, None]
    n = np.ones((2, ph.ny, ph.nx)) * np.array([1.7, 0.6])[:, None, None]
    P = np.zeros_like(n)
    o = oracle.observables(ph, psi, n, None, P)
    rp, rm = abs(a[0]) ** 2, abs(a[1]) ** 2
    assert abs(o["e_kin"]) < 1e-13 and abs(o["e_tetm"]) < 1e-13
    assert o["e_cross"] == pytest.approx(-0.3 * rp * rm * area, rel=1e-13)
    assert o["e_res"] == pytest.approx(1.1 * (1.7 * rp + 0.6 * rm) * area, rel=1e-13)
    assert o["reservoir"] == pytest.approx((1.7 + 0.6) * area, rel=1e-14)
