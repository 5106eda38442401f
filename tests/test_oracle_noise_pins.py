"""Pins of the oracle's stochastic part: the counter-based generator, the Gaussian
transform, the Wiener increment of Sec. 5 (truncated Wigner) and its effect on the
linear dynamics.

The generator is pinned to the published known-answer vectors of Philox4x32-10
(Salmon et al., SC'11); the counter layout to one of them; the Gaussian pairs to
the standard normal distribution; the increment to the correlations the paper
states; and the stochastic RK4 loop to the exact mean occupation of the linear
problem, whose Fourier modes are independent damped oscillators driven by white
noise.  All run on the CPU in seconds.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import BC_PERIODIC, BC_ZERO, Physics

RK4_POLY = [1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24]

# Known-answer vectors of Philox4x32-10: (counter, key, output).
PHILOX_KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,out", PHILOX_KAT)
def test_philox_known_answers(ctr, key, out):
    assert oracle.philox(ctr, key) == out


@pytest.mark.parametrize("odd", [0, 1])
def test_gauss_pair_counter_layout(odd):
    """Cell pair index q // 2, component, step (low, high word) form the counter and
    the seed (low, high word) the key; the even cell of the pair takes output words
    0 and 1, the odd cell words 2 and 3.  The third known-answer vector read that way
    gives the uniforms (x + 1/2) 2^-32 of those words, and Box-Muller of them."""
    ctr, key, out = PHILOX_KAT[2]
    step = ctr[2] | (ctr[3] << 32)
    seed = key[0] | (key[1] << 32)
    g = oracle.gauss_pair(2 * ctr[0] + odd, ctr[1], step, seed)
    u1 = (out[2 * odd] + 0.5) / 2.0 ** 32
    u2 = (out[2 * odd + 1] + 0.5) / 2.0 ** 32
    r = math.sqrt(-2.0 * math.log(u1))
    assert g[0] == pytest.approx(r * math.cos(2 * math.pi * u2), rel=1e-14, abs=1e-15)
    assert g[1] == pytest.approx(r * math.sin(2 * math.pi * u2), rel=1e-14, abs=1e-15)


def _noise_draws(ph, n_steps, seed, n=None):
    """Increments alone (psi starts at zero each step), shape (steps, comps, ny, nx)."""
    zero = np.zeros((ph.components, ph.ny, ph.nx), np.complex128)
    return np.stack([oracle.noise(ph, zero, n, dt=1.0, nu=1.0, seed=seed, step=k) for k in range(n_steps)])


def test_gaussian_pairs_are_standard_normal():
    """With gamma_c dt / (4 dV) = 1 the increment's real and imaginary parts are the
    raw Gaussian pair: each standard normal (KS test), uncorrelated with each other,
    across cells, across components and across steps."""
    ph = Physics(nx=64, ny=32, dx=0.5, dy=0.5, components=2, gamma_c=1.0)  # dt/(4 dV) = 1
    w = _noise_draws(ph, 24, seed=12345)
    x = np.concatenate([w.real.ravel(), w.imag.ravel()])
    assert stats.kstest(x, "norm").pvalue > 1e-4
    assert abs(x.mean()) < 5 / math.sqrt(x.size)
    assert abs(x.var() - 1.0) < 5 * math.sqrt(2.0 / x.size)
    assert abs(stats.kurtosis(x, fisher=False) - 3.0) < 5 * math.sqrt(24.0 / x.size)
    m = w.size
    lim = 5 / math.sqrt(m)
    assert abs(np.mean(w.real * w.imag)) < lim                                    # <dW dW> = 0 ...
    assert abs(np.mean(w.real ** 2 - w.imag ** 2)) < 2 * lim                      # ... both parts
    assert abs(np.mean((w[:, :, :, 1:] * np.conj(w[:, :, :, :-1])).real)) < 2 * lim  # cells
    assert abs(np.mean((w[:, 1] * np.conj(w[:, 0])).real)) < 4 * lim             # components
    assert abs(np.mean((w[1:] * np.conj(w[:-1])).real)) < 2 * lim                # steps


def test_seed_and_step_select_the_stream():
    ph = Physics(nx=16, ny=8, dx=1.0, dy=1.0, gamma_c=1.0)
    zero = np.zeros((1, 8, 16), np.complex128)
    a = oracle.noise(ph, zero, None, 1e-2, 1.0, seed=7, step=3)
    assert np.array_equal(a, oracle.noise(ph, zero, None, 1e-2, 1.0, seed=7, step=3))
    assert not np.any(a == oracle.noise(ph, zero, None, 1e-2, 1.0, seed=8, step=3))
    assert not np.any(a == oracle.noise(ph, zero, None, 1e-2, 1.0, seed=7, step=4))
    assert not np.any(a == oracle.noise(ph, zero, None, 1e-2, 1.0, seed=7, step=3 + (1 << 32)))


def test_increment_correlation_follows_gain_and_loss():
    """<dW dW*> = nu (R n + gamma_c) dt / (2 dV) per cell (Sec. 5), with the cell's own
    reservoir value: four reservoir levels, many steps, both components."""
    nx, ny, dx, dy = 32, 16, 0.4, 0.3
    R, gam, nu, dt = 0.7, 0.2, 0.6, 0.05
    ph = Physics(nx=nx, ny=ny, dx=dx, dy=dy, components=2, reservoir=True, R=R, gamma_c=gam)
    levels = np.array([0.0, 0.5, 2.0, 8.0])
    n = np.broadcast_to(np.repeat(levels, nx * ny * 2 // 4).reshape(2, ny, nx), (2, ny, nx)).copy()
    zero = np.zeros((2, ny, nx), np.complex128)
    steps = 300
    w = np.stack([oracle.noise(ph, zero, n, dt, nu, seed=99, step=k) for k in range(steps)])
    dV = dx * dy
    for lv in levels:
        sel = n == lv
        s = w[:, sel]
        want = nu * (R * lv + gam) * dt / (2 * dV)
        got = np.mean(np.abs(s) ** 2)
        assert got == pytest.approx(want, rel=6 * math.sqrt(1.0 / s.size)), lv
        assert abs(np.mean(s * s)) < 6 * want / math.sqrt(s.size), lv


def test_zero_intensity_is_the_deterministic_step():
    ph = Physics(nx=12, ny=10, dx=0.5, dy=0.5, reservoir=True, g=0.3, g_r=0.2, R=0.5,
                 gamma_c=0.3, gamma_r=0.4)
    rng = np.random.default_rng(2)
    psi = rng.standard_normal((1, 10, 12)) + 1j * rng.standard_normal((1, 10, 12))
    n = rng.random((1, 10, 12))
    P = rng.random((1, 10, 12))
    a = oracle.rk4(ph, psi, n, P=P, dt=1e-2, steps=5)
    b = oracle.rk4_noise(ph, psi, n, P=P, dt=1e-2, steps=5, nu=0.0, seed=4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_step_index_runs_on_across_calls():
    ph = Physics(nx=12, ny=10, dx=0.5, dy=0.5, g=0.3, gamma_c=0.3)
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((1, 10, 12)) + 1j * rng.standard_normal((1, 10, 12))
    whole, _ = oracle.rk4_noise(ph, psi, dt=1e-2, steps=4, nu=1.0, seed=11, step0=20)
    part, _ = oracle.rk4_noise(ph, psi, dt=1e-2, steps=3, nu=1.0, seed=11, step0=20)
    part, _ = oracle.rk4_noise(ph, part, dt=1e-2, steps=1, nu=1.0, seed=11, step0=23)
    assert np.array_equal(whole, part)


def _kappa(N, d, bc):
    if bc == BC_PERIODIC:
        return 4.0 / d ** 2 * np.sin(np.pi * np.arange(N) / N) ** 2
    return 4.0 / d ** 2 * np.sin(np.pi * np.arange(1, N + 1) / (2.0 * (N + 1))) ** 2


@pytest.mark.parametrize("bc", [BC_PERIODIC, BC_ZERO])
def test_linear_occupation_exact_and_half_quantum(bc):
    """Linear, lossy field (g = R = 0, constant V) driven by the noise from psi = 0.
    Plane waves (periodic) and sine modes (zero boundary) are orthonormal eigenmodes
    of the stencil, and an orthonormal transform keeps the per-cell white noise white
    with the same variance D = nu gamma dt / (2 dV).  A step multiplies mode k by the
    RK4 amplification lambda_k and adds its noise, so after m steps
    <|psi_k|^2> = D (1 - |lambda_k|^(2m)) / (1 - |lambda_k|^2), exactly; the mean
    over cells is the mean over modes.  For gamma dt << 1 and m gamma dt >> 1 that is
    nu / (2 dV) per cell: the half quantum per mode of the Wigner vacuum."""
    nx = ny = 32
    dx = dy = 0.5
    hbar, mass, V0, gam, nu, dt = 1.0, 1.0, 0.4, 1.0, 1.0, 0.01
    ph = Physics(nx=nx, ny=ny, dx=dx, dy=dy, bc_x=bc, bc_y=bc, hbar=hbar, mass=mass, gamma_c=gam)
    V = np.full((ny, nx), V0)
    first, last, seeds = 400, 800, 12
    acc = 0.0
    for seed in range(seeds):
        psi = np.zeros((1, ny, nx), np.complex128)
        for k in range(last):
            psi, _ = oracle.rk4_noise(ph, psi, V=V, dt=dt, steps=1, nu=nu, seed=1000 + seed, step0=k)
            if k + 1 > first:
                acc += np.mean(np.abs(psi) ** 2)
    got = acc / (seeds * (last - first))

    kap = _kappa(nx, dx, bc)[None, :] + _kappa(ny, dy, bc)[:, None]
    z = dt * (-1j * (hbar / (2 * mass) * kap + V0 / hbar) - gam / 2)
    lam2 = np.abs(sum(c * z ** j for j, c in enumerate(RK4_POLY))) ** 2
    D = nu * gam * dt / (2 * dx * dy)
    m = np.arange(first + 1, last + 1)[:, None, None]
    want = np.mean(D * (1 - lam2[None] ** m) / (1 - lam2[None]))
    # about 5 standard errors: 1024 modes x 12 seeds x 4 correlation times
    assert got == pytest.approx(want, rel=0.025)
    assert got == pytest.approx(nu / (2 * dx * dy), rel=0.03)
