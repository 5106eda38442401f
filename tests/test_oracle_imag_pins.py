"""Pins of the oracle's imaginary-time propagation (t -> -i tau, named in Sec. 6)
against the eigen-decomposition of a dense Hamiltonian built independently of it.

For the linear problem (g = 0) a step multiplies each eigenmode v_k of H by the
RK4 polynomial R(-E_k dtau/hbar) and then rescales the whole state, so the ratio
of any two mode coefficients after one step is known exactly; repeated steps leave
the ground state.  With g > 0 the converged state is a stationary solution of the
Gross-Pitaevskii equation, H[psi] psi = mu psi.  H is assembled from Kronecker
products of 1-D difference matrices (the sparse-matrix form of Sec. 3.1), not
from the oracle.  All run on the CPU in seconds.
"""
import numpy as np
import pytest

import oracle
from oracle import BC_PERIODIC, BC_ZERO, Physics
from test_oracle_pins import _d1, _d2

RK4_POLY = [1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24]


def rk4_amp(z):
    return sum(c * z ** k for k, c in enumerate(RK4_POLY))


def dense_h(ph, V, rho=None):
    """Hermitian H acting on the flattened state [components][ny][nx]: kinetic,
    potential, g|psi_s|^2 (with the given densities), TE-TM coupling."""
    nx, ny = ph.nx, ph.ny
    Ix, Iy = np.eye(nx), np.eye(ny)
    Dxx = np.kron(Iy, _d2(nx, ph.bc_x)) / ph.dx ** 2
    Dyy = np.kron(_d2(ny, ph.bc_y), Ix) / ph.dy ** 2
    Dxy = np.kron(_d1(ny, ph.bc_y), _d1(nx, ph.bc_x)) / (ph.dx * ph.dy)
    C, N = ph.components, nx * ny
    H = np.zeros((C * N, C * N), complex)
    for c in range(C):
        diag = V.ravel() + (0 if rho is None else ph.g * rho[c])
        H[c * N:(c + 1) * N, c * N:(c + 1) * N] = -(ph.hbar ** 2 / (2 * ph.mass)) * (Dxx + Dyy) + np.diag(diag)
        if C == 2:
            o = 1 - c
            sgn = 1 if c == 0 else -1
            H[c * N:(c + 1) * N, o * N:(o + 1) * N] = ph.delta_lt * ((Dxx - Dyy) - 2j * sgn * Dxy)
    return H


def cases():
    return [
        Physics(nx=6, ny=5, dx=0.4, dy=0.3, bc_x=BC_PERIODIC, bc_y=BC_ZERO, hbar=1.2, mass=0.8),
        Physics(nx=5, ny=4, dx=0.35, dy=0.4, bc_x=BC_ZERO, bc_y=BC_ZERO, components=2, hbar=0.9, mass=1.1,
                delta_lt=0.15),
    ]


@pytest.mark.parametrize("k", [0, 1])
def test_one_step_mode_ratios_exact(k):
    ph = cases()[k]
    rng = np.random.default_rng(20 + k)
    V = rng.uniform(-1, 1, (ph.ny, ph.nx))
    H = dense_h(ph, V)
    assert np.allclose(H, H.conj().T)
    E, vec = np.linalg.eigh(H)
    coef = np.zeros(len(E), complex)
    coef[[0, 1, 4]] = [0.8, 0.5 - 0.2j, 0.3j]
    psi0 = (vec @ coef).reshape(ph.components, ph.ny, ph.nx)
    dt = 0.02
    out = oracle.rk4_imag(ph, psi0, V=V, dt=dt, steps=1)
    c1 = vec.conj().T @ out.ravel()
    amp = rk4_amp(-E * dt / ph.hbar)
    for j in (1, 4):
        assert c1[j] / c1[0] == pytest.approx(coef[j] / coef[0] * amp[j] / amp[0], rel=1e-12)
    assert np.max(np.abs(np.delete(c1, [0, 1, 4]))) < 1e-12
    # the norm is the starting norm
    n0 = ph.dx * ph.dy * np.sum(np.abs(psi0) ** 2)
    assert ph.dx * ph.dy * np.sum(np.abs(out) ** 2) == pytest.approx(n0, rel=1e-13)


@pytest.mark.parametrize("k", [0, 1])
def test_converges_to_the_dense_ground_state(k):
    ph = cases()[k]
    rng = np.random.default_rng(30 + k)
    V = rng.uniform(-1, 1, (ph.ny, ph.nx))
    E, vec = np.linalg.eigh(dense_h(ph, V))
    psi0 = rng.standard_normal((ph.components, ph.ny, ph.nx)) + 1j * rng.standard_normal((ph.components, ph.ny, ph.nx))
    dt = 0.02
    steps = int(np.ceil(40 * ph.hbar / ((E[1] - E[0]) * dt)))
    out = oracle.rk4_imag(ph, psi0, V=V, dt=dt, steps=steps)
    u = out.ravel() / np.linalg.norm(out)
    assert abs(np.vdot(vec[:, 0], u)) == pytest.approx(1.0, abs=1e-12)
    assert np.real(np.vdot(u, dense_h(ph, V) @ u)) == pytest.approx(E[0], rel=1e-11)


def _nonlinear_run(dt, T=30.0):
    n, d, g = 20, 0.4, 2.0
    ph = Physics(nx=n, ny=n, dx=d, dy=d, bc_x=BC_ZERO, bc_y=BC_ZERO, g=g)
    x = (np.arange(n) - (n - 1) / 2) * d
    V = 0.5 * (x[None, :] ** 2 + x[:, None] ** 2)
    psi0 = np.exp(-(x[None, :] ** 2 + x[:, None] ** 2))[None] * (1 + 0j)
    psi0 *= np.sqrt(3.0 / (d * d * np.sum(np.abs(psi0) ** 2)))   # norm 3
    out = oracle.rk4_imag(ph, psi0, V=V, dt=dt, steps=int(round(T / dt)))
    assert d * d * np.sum(np.abs(out) ** 2) == pytest.approx(3.0, rel=1e-12)
    H = dense_h(ph, V, rho=np.abs(out.reshape(1, -1)) ** 2)
    u = out.ravel()
    mu = np.real(np.vdot(u, H @ u)) / np.real(np.vdot(u, u))
    res = np.linalg.norm(H @ u - mu * u) / np.linalg.norm(u)
    return res, mu, np.linalg.eigvalsh(dense_h(ph, V))[0]


def test_nonlinear_ground_state_is_stationary():
    """g > 0 in a harmonic trap: the converged state keeps the starting norm and
    solves H[psi] psi = mu psi up to the scheme's first-order splitting error (a full
    step runs at the unnormalized amplitude, then the norm is restored), so the
    residual halves with dtau and vanishes in the limit; the interaction raises mu
    above the linear ground energy."""
    r1, mu1, E0 = _nonlinear_run(0.01)
    r2, mu2, _ = _nonlinear_run(0.005)
    assert 1.9 < r1 / r2 < 2.1, (r1, r2)
    assert r1 < 1.0 * 0.01                     # O(dtau) with a modest constant
    assert abs(2 * r2 - r1) < 0.01 * r1        # first-order extrapolation to zero
    assert mu1 > E0 + 0.1 and abs(mu1 - mu2) < 1e-3


def test_rejects_dissipative_equation():
    ph = Physics(nx=4, ny=4, dx=1.0, dy=1.0, gamma_c=0.1)
    with pytest.raises(ValueError):
        oracle.rk4_imag(ph, np.ones((1, 4, 4)), dt=0.01, steps=1)
