"""CPU oracle for the PHOENIX solver (arXiv 2411.18341) -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, double-precision reference that the GPU path is
checked against.  Only the test suite, the smoke check and the CPU-baseline leg of
the benchmark may import it; the product library never does, and it shares no
code with it.  The arithmetic lives in ``phx_oracle.c`` (complex128, one loop nest
per definition, built with ``-ffp-contract=off``); this module only loads that
library with ctypes and marshals numpy arrays.

Parity status of each function (what pins it, see ``tests/test_oracle_pins.py``):
  rhs, rk4         -- pinned: discrete plane-wave / sine-mode closed forms (periodic and
                      zero boundaries), dense-matrix brute force on tiny grids, uniform
                      state vs a scalar ODE, reservoir-only closed form, mirror symmetry,
                      Gaussian spreading and harmonic ground state (continuum limits).
  dopri5_step      -- pinned: stability polynomial of the Dormand-Prince tableau on
                      y' = lambda y, fifth-order convergence on a nonlinear uniform state,
                      fourth-order embedded error.
  dopri5           -- controller pinned by hand-computed accept/reject sequences on a
                      scalar problem; the accepted-step sequence of long runs is
                      otherwise parity unpinned (controller constants are a choice).
  observables      -- pinned: Parseval norm, summation-by-parts kinetic identity,
                      closed-form energy of plane waves, uniform-state values; the cross,
                      TE-TM and reservoir energies and the reservoir total by Hamilton's
                      equation (the energy's directional derivative equals the one the
                      right-hand side implies), the dense quadratic form, fourth-order
                      energy conservation of spinor and frozen-reservoir runs, and the
                      conserved norm + reservoir total of particle exchange
                      (tests/test_oracle_observable_pins.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "phx_oracle.c")
_LIB = os.path.join(_HERE, "libphx_oracle.so")

BC_PERIODIC = 0
BC_ZERO = 1


def compile_library(src: str, out: str) -> str:
    """Compile an oracle source with gcc (plain C99 + OpenMP, no FMA contraction)."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", tmp, src, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Build the oracle library next to its source when it is missing or stale."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_library(_SRC, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("components", ctypes.c_int32), ("reservoir", ctypes.c_int32),
        ("hbar", ctypes.c_double), ("mass", ctypes.c_double),
        ("g", ctypes.c_double), ("g_x", ctypes.c_double), ("g_r", ctypes.c_double),
        ("R", ctypes.c_double), ("gamma_c", ctypes.c_double), ("gamma_r", ctypes.c_double),
        ("delta_lt", ctypes.c_double),
        ("E", ctypes.c_void_p), ("omega", ctypes.c_double), ("t0", ctypes.c_double),
    ]


class _Obs(ctypes.Structure):
    _fields_ = [
        ("norm", ctypes.c_double * 2), ("reservoir", ctypes.c_double),
        ("energy", ctypes.c_double), ("e_kin", ctypes.c_double), ("e_pot", ctypes.c_double),
        ("e_int", ctypes.c_double), ("e_cross", ctypes.c_double), ("e_tetm", ctypes.c_double),
        ("e_res", ctypes.c_double), ("max_density", ctypes.c_double),
        ("steady_res_density", ctypes.c_double), ("steady_res_reservoir", ctypes.c_double),
        ("nonfinite", ctypes.c_int64),
    ]


class _Ctrl(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt", ctypes.c_double),
                ("accepted", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("last_rejected", ctypes.c_int32), ("status", ctypes.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        # PHX_ORACLE_LIB loads a deliberately altered build (the mutation tests use it
        # to show that the pins reject a planted mistake).
        path = os.environ.get("PHX_ORACLE_LIB") or build()
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        lib.orc_rhs.argtypes = [P(_Params), vp, vp, vp, vp, vp, vp]
        lib.orc_rk4.argtypes = [P(_Params), vp, vp, vp, vp, ctypes.c_double, ctypes.c_int64]
        lib.orc_dopri5_step.argtypes = [P(_Params), vp, vp, vp, vp, ctypes.c_double, vp, vp, vp, vp]
        lib.orc_error_norm.argtypes = [P(_Params), vp, vp, vp, vp, vp, vp, ctypes.c_double, ctypes.c_double]
        lib.orc_error_norm.restype = ctypes.c_double
        lib.orc_dopri5.argtypes = [P(_Params), vp, vp, vp, vp, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int64, P(_Ctrl),
                                   vp, ctypes.c_int64]
        lib.orc_rhs_t.argtypes = [P(_Params), vp, vp, vp, vp, vp, vp]
        lib.orc_rk4_imag.argtypes = [P(_Params), vp, vp, ctypes.c_double, ctypes.c_int64]
        lib.orc_observables.argtypes = [P(_Params), vp, vp, vp, vp, P(_Obs)]
        u32p = P(ctypes.c_uint32)
        lib.orc_philox.argtypes = [u32p, u32p, u32p]
        lib.orc_gauss_pair.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_uint64,
                                       P(ctypes.c_double)]
        lib.orc_noise.argtypes = [P(_Params), vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                  ctypes.c_int64]
        lib.orc_rk4_noise.argtypes = [P(_Params), vp, vp, vp, vp, ctypes.c_double, ctypes.c_int64,
                                      ctypes.c_double, ctypes.c_uint64, ctypes.c_int64]
        _lib = lib
    return _lib


@dataclass
class Physics:
    """Grid and equation parameters (Eq. 1 and Eqs. PULSE_psi/PULSE_res)."""
    nx: int
    ny: int
    dx: float
    dy: float
    bc_x: int = BC_PERIODIC
    bc_y: int = BC_PERIODIC
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
    E: object = None        # coherent drive profile E_s(r), [components][ny][nx] complex, or None
    omega: float = 0.0      # drive frequency: E_s(r, t) = E_s(r) exp(-i omega t)
    t0: float = 0.0         # time at the start of a call

    def _c(self) -> _Params:
        e = None
        if self.E is not None:
            e = np.ascontiguousarray(np.asarray(self.E, dtype=np.complex128)).reshape(
                self.components, self.ny, self.nx)
            self._e_keep = e  # the library reads it during the call
        return _Params(self.nx, self.ny, self.dx, self.dy, self.bc_x, self.bc_y, self.components,
                       int(bool(self.reservoir)), self.hbar, self.mass, self.g, self.g_x, self.g_r,
                       self.R, self.gamma_c, self.gamma_r, self.delta_lt,
                       None if e is None else e.ctypes.data_as(ctypes.c_void_p), float(self.omega),
                       float(self.t0))


def _cplx(a, shape):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    if a.size != int(np.prod(shape)):
        raise ValueError(f"psi has {a.size} entries, expected {shape}")
    return a.reshape(shape).copy()


def _real(a, shape, required):
    if a is None:
        if required:
            raise ValueError("array required")
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.size != int(np.prod(shape)):
        raise ValueError(f"array has {a.size} entries, expected {shape}")
    return a.reshape(shape).copy()


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _shapes(ph: Physics):
    comp = (ph.components, ph.ny, ph.nx)
    return comp, comp, (ph.ny, ph.nx)


def rhs(ph: Physics, psi, n=None, V=None, P=None):
    """Time derivative (f_psi, f_n) of the coupled state at every cell (with the
    drive, when set, at time ph.t0)."""
    lib = _load()
    sp, sn, sv = _shapes(ph)
    psi = _cplx(psi, sp)
    n = _real(n, sn, ph.reservoir)
    P = _real(P, sn, ph.reservoir)
    V = _real(V, sv, False)
    fp = np.zeros(sp, np.complex128)
    fn = np.zeros(sn, np.float64) if ph.reservoir else None
    lib.orc_rhs_t(ctypes.byref(ph._c()), _ptr(psi), _ptr(n), _ptr(V), _ptr(P), _ptr(fp), _ptr(fn))
    return fp, fn


def rk4(ph: Physics, psi, n=None, V=None, P=None, dt=1e-3, steps=1):
    """Advance (psi, n) by `steps` RK4 steps; returns new arrays."""
    lib = _load()
    sp, sn, sv = _shapes(ph)
    psi = _cplx(psi, sp)
    n = _real(n, sn, ph.reservoir)
    P = _real(P, sn, ph.reservoir)
    V = _real(V, sv, False)
    lib.orc_rk4(ctypes.byref(ph._c()), _ptr(psi), _ptr(n), _ptr(V), _ptr(P), float(dt), int(steps))
    return psi, n


def dopri5_step(ph: Physics, psi, n=None, V=None, P=None, dt=1e-3):
    """One Dormand-Prince step: returns (psi5, n5, e_psi, e_n)."""
    lib = _load()
    sp, sn, sv = _shapes(ph)
    psi = _cplx(psi, sp)
    n = _real(n, sn, ph.reservoir)
    P = _real(P, sn, ph.reservoir)
    V = _real(V, sv, False)
    po = np.zeros(sp, np.complex128)
    pe = np.zeros(sp, np.complex128)
    no = np.zeros(sn, np.float64) if ph.reservoir else None
    ne = np.zeros(sn, np.float64) if ph.reservoir else None
    lib.orc_dopri5_step(ctypes.byref(ph._c()), _ptr(psi), _ptr(n), _ptr(V), _ptr(P), float(dt),
                        _ptr(po), _ptr(no), _ptr(pe), _ptr(ne))
    return po, no, pe, ne


def error_norm(ph: Physics, psi, n, psi_new, n_new, e_psi, e_n, rtol, atol):
    lib = _load()
    sp, sn, _ = _shapes(ph)
    a = [_cplx(psi, sp), _real(n, sn, ph.reservoir), _cplx(psi_new, sp),
         _real(n_new, sn, ph.reservoir), _cplx(e_psi, sp), _real(e_n, sn, ph.reservoir)]
    return lib.orc_error_norm(ctypes.byref(ph._c()), *[_ptr(x) for x in a], float(rtol), float(atol))


@dataclass
class Controller:
    """Adaptive-step state: time, next dt, counters."""
    t: float = 0.0
    dt: float = 1e-3
    accepted: int = 0
    rejected: int = 0
    last_rejected: int = 0
    status: int = 0
    history: list = field(default_factory=list)


def dopri5(ph: Physics, psi, n=None, V=None, P=None, *, rtol=1e-6, atol=1e-6, dt_min=1e-12,
           dt_max=np.inf, accepted=1, ctrl: Controller | None = None, history_cap=0):
    """Adaptive Dormand-Prince run until `accepted` more steps are accepted.

    Returns (psi, n, ctrl); ctrl.history holds (dt, err) of every attempt when
    history_cap > 0."""
    lib = _load()
    sp, sn, sv = _shapes(ph)
    psi = _cplx(psi, sp)
    n = _real(n, sn, ph.reservoir)
    P = _real(P, sn, ph.reservoir)
    V = _real(V, sv, False)
    ctrl = ctrl or Controller()
    c = _Ctrl(ctrl.t, ctrl.dt, ctrl.accepted, ctrl.rejected, ctrl.last_rejected, 0)
    hist = np.zeros(2 * max(history_cap, 1), np.float64)
    lib.orc_dopri5(ctypes.byref(ph._c()), _ptr(psi), _ptr(n), _ptr(V), _ptr(P), float(rtol),
                   float(atol), float(dt_min), float(dt_max), int(accepted), ctypes.byref(c),
                   _ptr(hist) if history_cap > 0 else None, int(history_cap))
    attempts = (c.accepted - ctrl.accepted) + (c.rejected - ctrl.rejected)
    h = [tuple(hist[2 * i:2 * i + 2]) for i in range(min(attempts, history_cap))]
    out = Controller(c.t, c.dt, c.accepted, c.rejected, c.last_rejected, c.status,
                     list(ctrl.history) + h)
    return psi, n, out


def observables(ph: Physics, psi, n=None, V=None, P=None) -> dict:
    """Norm, reservoir total, energy terms, max density, steady residuals."""
    lib = _load()
    sp, sn, sv = _shapes(ph)
    psi = _cplx(psi, sp)
    n = _real(n, sn, ph.reservoir)
    P = _real(P, sn, ph.reservoir)
    V = _real(V, sv, False)
    o = _Obs()
    lib.orc_observables(ctypes.byref(ph._c()), _ptr(psi), _ptr(n), _ptr(V), _ptr(P), ctypes.byref(o))
    d = {k: getattr(o, k) for k, _ in _Obs._fields_ if k != "norm"}
    d["norm"] = (o.norm[0], o.norm[1])
    return d


def philox(counter, key):
    """Philox4x32-10 of a 4-word counter and a 2-word key (4 uint32)."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xffffffff for v in counter])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    out = (ctypes.c_uint32 * 4)()
    _load().orc_philox(c, k, out)
    return tuple(int(v) for v in out)


def gauss_pair(q: int, comp: int, step: int, seed: int):
    """The two standard normals of cell q, component comp, step `step`."""
    out = (ctypes.c_double * 2)()
    _load().orc_gauss_pair(q, comp, step, seed, out)
    return out[0], out[1]


def noise(ph: Physics, psi, n, dt: float, nu: float, seed: int, step: int):
    """Adds the Wiener increment of step `step`; returns the new psi."""
    lib = _load()
    sp, sn, _ = _shapes(ph)
    psi = _cplx(psi, sp)
    n = _real(n, sn, ph.reservoir)
    lib.orc_noise(ctypes.byref(ph._c()), _ptr(psi), _ptr(n), float(dt), float(nu), int(seed), int(step))
    return psi


def rk4_noise(ph: Physics, psi, n=None, V=None, P=None, dt=1e-3, steps=1, nu=1.0, seed=0, step0=0):
    """`steps` RK4 steps, each followed by its Wiener increment; returns new arrays."""
    lib = _load()
    sp, sn, sv = _shapes(ph)
    psi = _cplx(psi, sp)
    n = _real(n, sn, ph.reservoir)
    P = _real(P, sn, ph.reservoir)
    V = _real(V, sv, False)
    lib.orc_rk4_noise(ctypes.byref(ph._c()), _ptr(psi), _ptr(n), _ptr(V), _ptr(P), float(dt), int(steps),
                      float(nu), int(seed), int(step0))
    return psi, n


def rk4_imag(ph: Physics, psi, V=None, dt=1e-3, steps=1):
    """`steps` imaginary-time RK4 steps, each restoring the norm psi had at the call's
    start; returns the new psi.  The conservative equation only."""
    if ph.reservoir or ph.gamma_c or ph.R or ph.E is not None:
        raise ValueError("imaginary time needs the conservative equation")
    lib = _load()
    sp, _, sv = _shapes(ph)
    psi = _cplx(psi, sp)
    V = _real(V, sv, False)
    lib.orc_rk4_imag(ctypes.byref(ph._c()), _ptr(psi), _ptr(V), float(dt), int(steps))
    return psi


def num_threads() -> int:
    """OpenMP threads the oracle's loops use."""
    lib = _load()
    lib.orc_num_threads.restype = ctypes.c_int
    return int(lib.orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the oracle's later loops (for timing it on fewer cores)."""
    lib = _load()
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    lib.orc_set_num_threads.restype = None
    lib.orc_set_num_threads(int(n))
