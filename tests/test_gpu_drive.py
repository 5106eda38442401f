"""GPU parity of the coherent drive (the E term of Eq. PULSE_psi) against the oracle,
through the C-ABI.

The drive -(i/hbar) E_s(r) exp(-i omega t) enters every stage at that stage's own
time; the stage-fused RK4 kernels read the four phasors of the current step from
device memory (written per step from the device step index, so graph replays keep
the phase), and the Dormand-Prince stages get theirs from the host.  Element-wise
parity to relative L2 1e-12 (complex128) and 1e-5 (complex64) on small ragged grids
(driven with and without V, spinor with reservoir, both boundary rules, direct
launches and graph replays; the streaming walks of one component and of the spinor
without reservoirs), together with the noise, after a phx_set_info to an
arbitrary time, for RK45 (same accept/reject sequence), and for the observables'
residual; at 2048^2 the plane-wave response against the exact driven solution on
every cell.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import C64, C128, TOL, GpuRun, oracle_physics, quantize, rel_l2, replay_attempts
from paper_2411_18341_amd import inputs, phx
from test_gpu_rk4 import workload

pytestmark = pytest.mark.gpu

OMEGA = 1.3


def drive_profile(ph, seed, amp=0.8):
    """A smooth complex spot per component (different for the two components)."""
    X, Y = inputs.coords(ph.nx, ph.ny, ph.dx, ph.dy)
    rng = np.random.default_rng(seed)
    out = []
    for s in range(ph.components):
        x0, y0 = rng.uniform(-1, 1, 2) * 0.3 * np.array([X.max(), Y.max()])
        w = 0.25 * max(X.max(), Y.max())
        ph0 = rng.uniform(0, 2 * np.pi)
        out.append(amp * np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / (2 * w * w) + 1j * (ph0 + 0.5 * X)))
    return np.stack(out)


def oracle_drive(ph, E, t0=0.0):
    op = oracle_physics(ph)
    op.E, op.omega, op.t0 = E, OMEGA, t0
    return op


def quantize_e(precision, E):
    return E.astype(np.complex64).astype(np.complex128) if precision == C64 else E


@pytest.mark.parametrize("family", [phx.PHX_KERNEL_STAGE, phx.PHX_KERNEL_AUTO])
@pytest.mark.parametrize("graph_steps", [-1, 2])
@pytest.mark.parametrize("precision", [C64, C128])
@pytest.mark.parametrize("kind,bc", [("driven", (0, 0)), ("driven_v", (1, 0)), ("driven_v", (0, 1)),
                                     ("spinor_res", (0, 1)), ("spinor_res", (1, 1))])
def test_drive_parity(kind, bc, precision, graph_steps, family):
    ph, psi, n, V, P = workload(kind, 97, 61, bc, seed=4)
    q = quantize(precision, psi, n, V, P)
    E = quantize_e(precision, drive_profile(ph, 5))
    run = GpuRun(ph, *q, precision=precision, E=E, drive_omega=OMEGA, graph_steps=graph_steps, kernel=family)
    assert run.solver.handle is not None
    run.step(7)
    g_psi, g_n = run.state()
    run.close()
    o_psi, o_n = oracle.rk4(oracle_drive(ph, E), *q, dt=ph.dt, steps=7)
    d_psi, _ = oracle.rk4(oracle_physics(ph), *q, dt=ph.dt, steps=7)
    assert rel_l2(d_psi, o_psi) > 100 * TOL[precision]  # the drive is visible
    e_psi = rel_l2(g_psi, o_psi)
    e_n = rel_l2(g_n, o_n) if ph.reservoir else 0.0
    print(f"{kind} bc={bc} graph={graph_steps} family={family}: psi {e_psi:.3e} n {e_n:.3e}")
    assert e_psi <= TOL[precision] and e_n <= TOL[precision]


@pytest.mark.parametrize("family", [phx.PHX_KERNEL_STAGE, phx.PHX_KERNEL_AUTO])
@pytest.mark.parametrize("precision", [C64, C128])
def test_drive_with_noise(precision, family):
    ph, psi, n, V, P = workload("driven", 90, 70, (0, 0), seed=6)
    q = quantize(precision, psi, n, V, P)
    E = quantize_e(precision, drive_profile(ph, 7))
    run = GpuRun(ph, *q, precision=precision, E=E, drive_omega=OMEGA, noise=0.7, seed=31, graph_steps=4,
                 kernel=family)
    run.step(9)
    g_psi, g_n = run.state()
    run.close()
    o_psi, o_n = oracle.rk4_noise(oracle_drive(ph, E), *q, dt=ph.dt, steps=9, nu=0.7, seed=31, step0=0)
    assert rel_l2(g_psi, o_psi) <= TOL[precision] and rel_l2(g_n, o_n) <= TOL[precision]


@pytest.mark.parametrize("family", [phx.PHX_KERNEL_STAGE, phx.PHX_KERNEL_AUTO])
@pytest.mark.parametrize("graph_steps", [-1, 2])
def test_drive_after_set_info(graph_steps, family):
    """phx_set_info to an arbitrary (t, step) restarts the drive's clock there, also
    for a graph captured before the call."""
    ph, psi, n, V, P = workload("driven_v", 100, 64, (0, 1), seed=9)
    E = drive_profile(ph, 8)
    run = GpuRun(ph, psi, n, V, P, precision=C128, E=E, drive_omega=OMEGA, graph_steps=graph_steps,
                 kernel=family)
    run.step(4)  # captures a graph (graph_steps 2) with the old clock
    mid_psi, mid_n = run.state()
    run.solver.set_info(t=37.25, steps_accepted=1000)
    run.step(6)
    g_psi, g_n = run.state()
    info = run.solver.info()
    run.close()
    o_psi, o_n = oracle.rk4(oracle_drive(ph, E, t0=37.25), mid_psi, mid_n, V, P, dt=ph.dt, steps=6)
    assert info["steps_accepted"] == 1006
    assert rel_l2(g_psi, o_psi) <= TOL[C128] and rel_l2(g_n, o_n) <= TOL[C128]


@pytest.mark.parametrize("precision", [C64, C128])
def test_drive_rk45_parity(precision):
    ph, psi, n, V, P = workload("spinor_res", 80, 64, (1, 0), seed=10)
    q = quantize(precision, psi, n, V, P)
    E = quantize_e(precision, drive_profile(ph, 11, amp=2.0))
    run = GpuRun(ph, *q, precision=precision, E=E, drive_omega=OMEGA, integrator=phx.PHX_RK45, rtol=1e-6,
                 atol=1e-6, dt=1e-3, dt_min=1e-12)
    run.solver.log_attempts(1000)
    run.step(12)
    info = run.solver.info()
    att = run.solver.attempts()
    g_psi, g_n = run.state()
    run.close()
    tol = TOL[precision]
    if precision == C128:  # the oracle's own controller takes the same decisions
        o_psi, o_n, ctrl = oracle.dopri5(oracle_drive(ph, E), *q, rtol=1e-6, atol=1e-6, dt_min=1e-12,
                                         accepted=12, ctrl=oracle.Controller(dt=1e-3))
        assert info["steps_accepted"] == ctrl.accepted == 12
        assert info["steps_rejected"] == ctrl.rejected
        assert abs(info["t"] - ctrl.t) <= tol * ctrl.t
        assert rel_l2(g_psi, o_psi) <= tol and rel_l2(g_n, o_n) <= tol
    # both precisions: the oracle replays the GPU's attempts (the drive at each
    # attempt's own time), states compared at the same time
    r_psi, r_n, r_t, errs = replay_attempts(oracle_drive(ph, E), *q, att, 1e-6, 1e-6)
    assert r_t == info["t"] and int(att[:, 2].sum()) == 12
    assert np.allclose(att[:, 1], errs, rtol=1e-9 if precision == C128 else 0.1)
    assert rel_l2(g_psi, r_psi) <= tol and rel_l2(g_n, r_n) <= tol


@pytest.mark.parametrize("precision", [C64, C128])
def test_drive_observables_residual(precision):
    ph, psi, n, V, P = workload("driven_v", 77, 55, (1, 1), seed=12)
    q = quantize(precision, psi, n, V, P)
    E = quantize_e(precision, drive_profile(ph, 13))
    run = GpuRun(ph, *q, precision=precision, E=E, drive_omega=OMEGA)
    run.step(3)
    g_psi, g_n = run.state()
    obs = run.observables()
    t = run.solver.info()["t"]
    run.close()
    o = oracle.observables(oracle_drive(ph, E, t0=t), g_psi, g_n, q[2], q[3])
    tol = 1e-12 if precision == C128 else 1e-5  # the residual goes through the kernel-precision RHS
    assert obs["steady_res_density"] == pytest.approx(o["steady_res_density"], rel=tol)
    ou = oracle.observables(oracle_physics(ph), g_psi, g_n, q[2], q[3])
    assert abs(ou["steady_res_density"] - o["steady_res_density"]) > 10 * tol * o["steady_res_density"]


@pytest.mark.parametrize("precision", [C64, C128])
@pytest.mark.parametrize("rows", [40, 64])
def test_drive_streaming_shapes(rows, precision):
    """The driven streaming kernel for both band heights on ragged grids of several
    strips and bands, both y boundary rules, odd and even step counts over two calls
    (the phasors follow the device step index)."""
    for bc, (nx, ny) in (((0, 0), (130, 97)), ((1, 1), (57, 203)), ((0, 1), (200, 131))):
        ph, psi, n, V, P = workload("driven_v", nx, ny, bc, seed=11)
        q = quantize(precision, psi, n, V, P)
        E = quantize_e(precision, drive_profile(ph, 12))
        run = GpuRun(ph, *q, precision=precision, E=E, drive_omega=OMEGA, kernel=phx.PHX_KERNEL_STEP,
                     tile_wx=1, tile_rows=rows, graph_steps=2)
        run.step(5)
        run.step(4)
        g_psi, g_n = run.state()
        run.close()
        o_psi, o_n = oracle.rk4(oracle_drive(ph, E), *q, dt=ph.dt, steps=9)
        assert rel_l2(g_psi, o_psi) <= TOL[precision] and rel_l2(g_n, o_n) <= TOL[precision], (bc, rows)


@pytest.mark.parametrize("precision", [C64, C128])
@pytest.mark.parametrize("rows", [40, 64])
def test_drive_spinor_streaming(rows, precision):
    """The spinor (no reservoirs) on its streaming walk with the drive: a profile per
    component, both band heights, ragged grids of several strips and bands, three
    boundary mixes, odd and even step counts over two calls; the same with the kernel
    family left to the library, which picks this walk."""
    for bc, (nx, ny) in (((0, 0), (130, 97)), ((1, 1), (57, 150)), ((0, 1), (200, 83))):
        ph, psi, n, V, P = workload("spinor", nx, ny, bc, seed=13)
        q = quantize(precision, psi, n, V, P)
        E = quantize_e(precision, drive_profile(ph, 14))
        o_psi, _ = oracle.rk4(oracle_drive(ph, E), *q, dt=ph.dt, steps=9)
        for kw in (dict(kernel=phx.PHX_KERNEL_STEP, tile_wx=1, tile_rows=rows), dict()):
            run = GpuRun(ph, *q, precision=precision, E=E, drive_omega=OMEGA, graph_steps=2, **kw)
            run.step(5)
            run.step(4)
            g_psi, _ = run.state()
            run.close()
            assert rel_l2(g_psi, o_psi) <= TOL[precision], (bc, rows, kw)


def test_drive_family_and_rejections():
    ph, psi, n, V, P = workload("driven", 64, 48, (0, 0))
    E = drive_profile(ph, 1)
    with pytest.raises(phx.PhxError) as e:  # region shapes take no drive
        GpuRun(ph, psi, n, V, P, precision=C64, E=E, kernel=phx.PHX_KERNEL_STEP, tile_wx=8, tile_rows=4)
    assert e.value.status == phx.PHX_EINVAL
    with pytest.raises(phx.PhxError) as e:  # nor bands other than 40 and 64 rows
        GpuRun(ph, psi, n, V, P, precision=C64, E=E, kernel=phx.PHX_KERNEL_STEP, tile_wx=1, tile_rows=88)
    assert e.value.status == phx.PHX_EINVAL
    ph2, psi2, n2, V2, P2 = workload("spinor_res", 64, 48, (0, 0))
    with pytest.raises(phx.PhxError) as e:  # the spinor with reservoirs and the drive: stage-fused only
        GpuRun(ph2, psi2, n2, V2, P2, precision=C64, E=drive_profile(ph2, 2), kernel=phx.PHX_KERNEL_STEP,
               tile_wx=1, tile_rows=40)
    assert e.value.status == phx.PHX_EUNSUPPORTED
    with pytest.raises(phx.PhxError) as e:
        GpuRun(ph, psi, n, V, P, precision=C64, E=E, drive=False)  # profile without drive
    assert e.value.status == phx.PHX_EINVAL
    with pytest.raises(phx.PhxError) as e:
        GpuRun(ph, psi, n, V, P, precision=C64, drive=True)  # drive without profile
    assert e.value.status == phx.PHX_EINVAL


@pytest.mark.parametrize("precision", [C64, C128])
def test_plane_wave_drive_2048_exact(precision):
    """A linear lossy field (g = 0, constant V) on a 2048^2 periodic grid driven by a
    plane wave from psi = 0: every cell follows the exact driven-oscillator solution
    of its mode, A (exp(-i omega t) - exp(lambda t)) with A = F/(-i omega - lambda),
    F = -i E/hbar and lambda = -i(hbar kappa/2m + V0/hbar) - gamma/2, up to RK4's
    truncation error (|lambda dt| = 0.004, omega dt = 0.011: far below 1e-7 after 400
    steps)."""
    n, d, V0, gam, dt, steps, omega = 2048, 0.5, 0.3, 0.2, 0.01, 400, 1.1
    mx, my, amp = 37, -21, 0.6 - 0.2j
    ph = inputs.Physics(nx=n, ny=n, dx=d, dy=d, gamma_c=gam, dt=dt)
    idx = np.arange(n)
    Erow = np.exp(2j * np.pi * mx * idx / n)
    Ecol = np.exp(2j * np.pi * my * idx / n)
    E = (amp * Ecol[:, None] * Erow[None, :])[None]
    run = GpuRun(ph, np.zeros((1, n, n), np.complex128), None, np.full((n, n), V0), None,
                 precision=precision, E=E, drive_omega=omega)
    run.step(steps)
    g_psi, _ = run.state()
    run.close()
    kap = 4 / d ** 2 * (np.sin(np.pi * mx / n) ** 2 + np.sin(np.pi * my / n) ** 2)
    lam = -1j * (0.5 * kap + V0) - gam / 2
    t = steps * dt
    A = (-1j * E[0]) / (-1j * omega - lam)
    want = A * (np.exp(-1j * omega * t) - np.exp(lam * t))
    err = np.linalg.norm(g_psi[0] - want) / np.linalg.norm(want)
    print(f"plane-wave drive 2048^2: rel L2 {err:.3e}")
    assert err <= (TOL[precision] if precision == C64 else 1e-7)
