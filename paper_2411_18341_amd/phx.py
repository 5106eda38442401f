"""ctypes binding of libphx (include/phx.h): the same entry points under the same
names, plus a small `Solver` convenience wrapper.

This layer only marshals arguments: every step of the time integration runs in the
HIP kernels of libphx.so.  PyTorch supplies device memory and the current HIP
stream.  If the library has not been built the first call raises; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libphx.so")

# enums of phx.h
PHX_OK, PHX_EINVAL, PHX_EWORKSPACE, PHX_EHIP, PHX_ENONFINITE, PHX_EDTMIN, PHX_EUNSUPPORTED, PHX_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
PHX_BC_PERIODIC, PHX_BC_ZERO = 0, 1
PHX_C64, PHX_C128 = 0, 1
PHX_RK4, PHX_RK45 = 0, 1
PHX_KERNEL_AUTO, PHX_KERNEL_STAGE, PHX_KERNEL_STEP = 0, 1, 2

STATUS_NAMES = {0: "PHX_OK", -1: "PHX_EINVAL", -2: "PHX_EWORKSPACE", -3: "PHX_EHIP",
                -4: "PHX_ENONFINITE", -5: "PHX_EDTMIN", -6: "PHX_EUNSUPPORTED", -7: "PHX_ESTATE"}


class phx_config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("components", ctypes.c_int32), ("reservoir", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("integrator", ctypes.c_int32),
        ("hbar", ctypes.c_double), ("mass", ctypes.c_double),
        ("g", ctypes.c_double), ("g_x", ctypes.c_double), ("g_r", ctypes.c_double),
        ("R", ctypes.c_double), ("gamma_c", ctypes.c_double), ("gamma_r", ctypes.c_double),
        ("delta_lt", ctypes.c_double),
        ("dt", ctypes.c_double), ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
        ("dt_min", ctypes.c_double), ("dt_max", ctypes.c_double),
        ("kernel", ctypes.c_int32), ("tile_wx", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
        ("graph_steps", ctypes.c_int32),
        ("noise", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("drive_omega", ctypes.c_double), ("drive", ctypes.c_int32), ("imag_time", ctypes.c_int32),
    ]


class phx_fields(ctypes.Structure):
    _fields_ = [("psi", ctypes.c_void_p), ("n", ctypes.c_void_p), ("V", ctypes.c_void_p),
                ("P", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("E", ctypes.c_void_p)]


class phx_obs(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_double * 2), ("reservoir", ctypes.c_double),
                ("energy", ctypes.c_double), ("e_kin", ctypes.c_double), ("e_pot", ctypes.c_double),
                ("e_int", ctypes.c_double), ("e_cross", ctypes.c_double), ("e_tetm", ctypes.c_double),
                ("e_res", ctypes.c_double), ("max_density", ctypes.c_double),
                ("steady_res_density", ctypes.c_double), ("steady_res_reservoir", ctypes.c_double),
                ("nonfinite", ctypes.c_int64), ("norm_renorm", ctypes.c_double * 2)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("norm", "norm_renorm")}
        d["norm"] = (self.norm[0], self.norm[1])
        d["norm_renorm"] = (self.norm_renorm[0], self.norm_renorm[1])
        return d


class phx_info(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt", ctypes.c_double),
                ("steps_accepted", ctypes.c_int64), ("steps_rejected", ctypes.c_int64),
                ("last_rejected", ctypes.c_int32), ("nonfinite", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


PHX_MAX_KERNEL_KINDS = 24


class phx_timing(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("name", (ctypes.c_char * 32) * PHX_MAX_KERNEL_KINDS),
                ("launches", ctypes.c_int64 * PHX_MAX_KERNEL_KINDS),
                ("ms_total", ctypes.c_double * PHX_MAX_KERNEL_KINDS)]

    def as_dict(self):
        return {self.name[k].value.decode(): {"launches": self.launches[k], "ms_total": self.ms_total[k]}
                for k in range(self.count)}


class phx_tune_result(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int32), ("tile_wx", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("best_us", ctypes.c_double), ("default_us", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class phx_instance(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("param_index", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("offset", ctypes.c_int64), ("seed", ctypes.c_uint64)]


class phx_batch_desc(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("instances", ctypes.POINTER(phx_instance)), ("params", ctypes.POINTER(phx_config)),
                ("n_params", ctypes.c_int32), ("check_finite", ctypes.c_int32),
                ("total_cells", ctypes.c_int64),
                ("psi", ctypes.c_void_p), ("n", ctypes.c_void_p), ("P", ctypes.c_void_p),
                ("V", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("step0", ctypes.c_int64)]


class phx_cnn_config(ctypes.Structure):
    _fields_ = [("in_channels", ctypes.c_int32), ("hidden", ctypes.c_int32), ("out_channels", ctypes.c_int32),
                ("height", ctypes.c_int32), ("width", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


class phx_cnn_buffers(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("adam_m", ctypes.c_void_p), ("adam_v", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


# names of every exported entry point (kept in step with include/phx.h)
ENTRY_POINTS = ("phx_workspace_bytes", "phx_create", "phx_step", "phx_observables", "phx_get_info",
                "phx_set_info", "phx_destroy", "phx_last_error", "phx_log_attempts", "phx_set_timing",
                "phx_kernel_times",
                "phx_autotune", "phx_batch_workspace_bytes", "phx_batch_step", "phx_cnn_sizes",
                "phx_cnn_param_offsets", "phx_cnn_create", "phx_cnn_destroy", "phx_cnn_forward",
                "phx_cnn_gradients", "phx_cnn_adam", "phx_cnn_train_step", "phx_coarsen",
                "phx_corrector_features", "phx_corrector_residual", "phx_corrector_apply",
                "phx_stream_copy", "phx_walk_pattern", "phx_observables_static")

_lib = None


def load(path: str | None = None):
    """Load libphx.so (built by `paper_2411_18341_amd.build`); raises if absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build the HIP library first "
                           "(python -m paper_2411_18341_amd.build)")
    lib = ctypes.CDLL(p)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    st = ctypes.c_int
    lib.phx_workspace_bytes.argtypes = [P(phx_config), P(ctypes.c_size_t)]
    lib.phx_workspace_bytes.restype = st
    lib.phx_create.argtypes = [P(phx_config), P(phx_fields), vp, P(vp)]
    lib.phx_create.restype = st
    lib.phx_step.argtypes = [vp, ctypes.c_int64, P(phx_info)]
    lib.phx_step.restype = st
    lib.phx_observables.argtypes = [vp, P(phx_obs)]
    lib.phx_observables.restype = st
    lib.phx_get_info.argtypes = [vp, P(phx_info)]
    lib.phx_get_info.restype = st
    lib.phx_set_info.argtypes = [vp, P(phx_info)]
    lib.phx_set_info.restype = st
    lib.phx_destroy.argtypes = [vp]
    lib.phx_destroy.restype = None
    lib.phx_last_error.argtypes = []
    lib.phx_last_error.restype = ctypes.c_char_p
    lib.phx_log_attempts.argtypes = [vp, vp, ctypes.c_int64, vp]
    lib.phx_log_attempts.restype = st
    lib.phx_set_timing.argtypes = [vp, ctypes.c_int32]
    lib.phx_set_timing.restype = st
    lib.phx_kernel_times.argtypes = [vp, P(phx_timing)]
    lib.phx_kernel_times.restype = st
    lib.phx_autotune.argtypes = [vp, ctypes.c_int32, P(phx_tune_result)]
    lib.phx_autotune.restype = st
    lib.phx_batch_workspace_bytes.argtypes = [P(phx_batch_desc), P(ctypes.c_size_t)]
    lib.phx_batch_workspace_bytes.restype = st
    lib.phx_batch_step.argtypes = [P(phx_batch_desc), ctypes.c_int64, vp]
    lib.phx_batch_step.restype = st
    i32, i64, dbl, flt = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_float
    lib.phx_cnn_sizes.argtypes = [P(phx_cnn_config), P(i64), P(ctypes.c_size_t)]
    lib.phx_cnn_param_offsets.argtypes = [P(phx_cnn_config), P(i64), P(i64), P(i32), P(i32), P(i32)]
    lib.phx_cnn_create.argtypes = [P(phx_cnn_config), P(phx_cnn_buffers), vp, P(vp)]
    lib.phx_cnn_destroy.argtypes = [vp]
    lib.phx_cnn_destroy.restype = None
    lib.phx_cnn_forward.argtypes = [vp, vp, i32, vp]
    lib.phx_cnn_gradients.argtypes = [vp, vp, vp, i32, vp, vp]
    lib.phx_cnn_adam.argtypes = [vp, vp, i32, flt, flt, flt, flt]
    lib.phx_cnn_train_step.argtypes = [vp, vp, vp, i32, i32, flt, vp]
    lib.phx_coarsen.argtypes = [i32, vp, vp, vp, i32, i32, i32, vp, vp, vp, vp]
    lib.phx_corrector_features.argtypes = [i32, vp, vp, vp, i32, i32, dbl, dbl, dbl, vp, vp]
    lib.phx_corrector_residual.argtypes = [i32, vp, vp, vp, vp, i32, i32, dbl, dbl, vp, vp]
    lib.phx_corrector_apply.argtypes = [i32, vp, vp, vp, i32, i32, dbl, dbl, vp]
    lib.phx_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.phx_stream_copy.restype = st
    lib.phx_walk_pattern.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp]
    lib.phx_walk_pattern.restype = st
    lib.phx_observables_static.argtypes = [P(phx_config), P(phx_fields), ctypes.c_double, vp, P(phx_obs)]
    lib.phx_observables_static.restype = st
    for name in ("phx_cnn_sizes", "phx_cnn_param_offsets", "phx_cnn_create", "phx_cnn_forward",
                 "phx_cnn_gradients", "phx_cnn_adam", "phx_cnn_train_step", "phx_coarsen",
                 "phx_corrector_features", "phx_corrector_residual", "phx_corrector_apply"):
        getattr(lib, name).restype = st
    if path is None:
        _lib = lib
    return lib


class PhxError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _check(status: int):
    if status != PHX_OK:
        raise PhxError(status, (load().phx_last_error() or b"").decode())


# ------------------------------------------------------------ C-ABI mirrors

def phx_workspace_bytes(cfg: phx_config) -> int:
    out = ctypes.c_size_t(0)
    _check(load().phx_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)))
    return out.value


def phx_create(cfg: phx_config, fields: phx_fields, stream: int | None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(load().phx_create(ctypes.byref(cfg), ctypes.byref(fields), stream or None, ctypes.byref(h)))
    return h


def phx_step(h, n_steps: int) -> phx_info:
    info = phx_info()
    _check(load().phx_step(h, int(n_steps), ctypes.byref(info)))
    return info


def phx_observables(h) -> phx_obs:
    o = phx_obs()
    _check(load().phx_observables(h, ctypes.byref(o)))
    return o


def phx_get_info(h) -> phx_info:
    info = phx_info()
    _check(load().phx_get_info(h, ctypes.byref(info)))
    return info


def phx_set_info(h, info: phx_info) -> None:
    _check(load().phx_set_info(h, ctypes.byref(info)))


def phx_destroy(h) -> None:
    load().phx_destroy(h)


def phx_last_error() -> str:
    return (load().phx_last_error() or b"").decode()


def phx_log_attempts(h, log, cap: int, count) -> None:
    """log: host float64 array of >= 3*cap entries (or None to stop); count: host int64
    array of one entry (both numpy, kept alive by the caller while logging)."""
    lp = None if log is None else log.ctypes.data_as(ctypes.c_void_p)
    cp = None if count is None else count.ctypes.data_as(ctypes.c_void_p)
    _check(load().phx_log_attempts(h, lp, int(cap), cp))


def phx_set_timing(h, enable: bool) -> None:
    _check(load().phx_set_timing(h, int(bool(enable))))


def phx_kernel_times(h) -> phx_timing:
    out = phx_timing()
    _check(load().phx_kernel_times(h, ctypes.byref(out)))
    return out


def phx_autotune(h, reps: int = 10) -> phx_tune_result:
    out = phx_tune_result()
    _check(load().phx_autotune(h, int(reps), ctypes.byref(out)))
    return out


def phx_batch_workspace_bytes(desc: phx_batch_desc) -> int:
    out = ctypes.c_size_t(0)
    _check(load().phx_batch_workspace_bytes(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def phx_batch_step(desc: phx_batch_desc, n_steps: int, stream: int | None) -> None:
    _check(load().phx_batch_step(ctypes.byref(desc), int(n_steps), stream or None))


def phx_observables_static(cfg: phx_config, fields: phx_fields, t: float, stream: int | None) -> phx_obs:
    out = phx_obs()
    _check(load().phx_observables_static(ctypes.byref(cfg), ctypes.byref(fields), float(t), stream or None,
                                         ctypes.byref(out)))
    return out


def observables_static(cfg: phx_config, psi, n=None, V=None, P=None, E=None, t: float = 0.0, stream=None) -> dict:
    """Observables of the given device tensors without a handle or workspace (the
    library's allocation-free entry point), on `stream` (default: torch's current)."""
    ptr = lambda x: None if x is None else x.data_ptr()
    fields = phx_fields(ptr(psi), ptr(n), ptr(V), ptr(P), None, 0, ptr(E))
    return phx_observables_static(cfg, fields, t, _stream_handle(stream, psi.device)).as_dict()


def phx_stream_copy(dst, src, nbytes: int, stream: int | None) -> None:
    _check(load().phx_stream_copy(dst, src, int(nbytes), stream or None))


def stream_copy(dst, src, stream=None) -> None:
    """Copy tensor src into tensor dst (same byte size, CUDA, contiguous) with the
    library's streaming copy kernel on `stream` (default: torch's current stream)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("dst and src must be contiguous and of equal byte size")
    phx_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                    _stream_handle(stream, src.device))


def phx_walk_pattern(psi_out, n_out, psi_in, n_in, P, nx: int, ny: int, band_rows: int, stream: int | None) -> None:
    _check(load().phx_walk_pattern(psi_out, n_out, psi_in, n_in, P, int(nx), int(ny), int(band_rows),
                                   stream or None))


def walk_pattern(psi_out, n_out, psi_in, n_in, P, band_rows: int = 0, stream=None) -> None:
    """The wide whole-step walk's loads and stores without its arithmetic (psi_out =
    psi_in, n_out = n_in + P) on complex64 psi and float32 n, P tensors of shape
    [ny, nx] or [1, ny, nx] (CUDA, contiguous), on `stream` (default: torch's current)."""
    import torch
    ny, nx = psi_in.shape[-2:]
    for t, dt in ((psi_out, torch.complex64), (psi_in, torch.complex64), (n_out, torch.float32),
                  (n_in, torch.float32), (P, torch.float32)):
        if t.dtype != dt or tuple(t.shape[-2:]) != (ny, nx) or t.numel() != nx * ny or not t.is_contiguous():
            raise ValueError("walk_pattern takes contiguous complex64 psi and float32 n, P of one shape")
    v = lambda t: ctypes.c_void_p(t.data_ptr())
    phx_walk_pattern(v(psi_out), v(n_out), v(psi_in), v(n_in), v(P), nx, ny, band_rows,
                     _stream_handle(stream, psi_in.device))


# ------------------------------------------------------------ conveniences

def make_config(nx, ny, dx, dy=None, *, bc_x=PHX_BC_PERIODIC, bc_y=PHX_BC_PERIODIC, components=1,
                reservoir=False, precision=PHX_C64, integrator=PHX_RK4, hbar=1.0, mass=1.0, g=0.0,
                g_x=0.0, g_r=0.0, R=0.0, gamma_c=0.0, gamma_r=0.0, delta_lt=0.0, dt=1e-3,
                rtol=1e-6, atol=1e-6, dt_min=1e-12, dt_max=float("inf"),
                kernel=PHX_KERNEL_AUTO, tile_wx=0, tile_rows=0, graph_steps=0, noise=0.0,
                seed=0, drive=False, drive_omega=0.0, imag_time=False) -> phx_config:
    return phx_config(int(nx), int(ny), float(dx), float(dx if dy is None else dy), int(bc_x), int(bc_y),
                      int(components), int(bool(reservoir)), int(precision), int(integrator),
                      float(hbar), float(mass), float(g), float(g_x), float(g_r), float(R),
                      float(gamma_c), float(gamma_r), float(delta_lt), float(dt), float(rtol),
                      float(atol), float(dt_min), float(dt_max), int(kernel), int(tile_wx),
                      int(tile_rows), int(graph_steps), float(noise), int(seed) & (2 ** 64 - 1),
                      float(drive_omega), int(bool(drive)), int(bool(imag_time)))


def config_from_physics(ph, **kw) -> phx_config:
    """phx_config from a workload description with the fields of inputs.Physics."""
    d = dict(nx=ph.nx, ny=ph.ny, dx=ph.dx, dy=ph.dy, bc_x=ph.bc_x, bc_y=ph.bc_y,
             components=ph.components, reservoir=ph.reservoir, hbar=ph.hbar, mass=ph.mass, g=ph.g,
             g_x=ph.g_x, g_r=ph.g_r, R=ph.R, gamma_c=ph.gamma_c, gamma_r=ph.gamma_r,
             delta_lt=ph.delta_lt, dt=ph.dt)
    d.update(kw)
    nx, ny, dx = d.pop("nx"), d.pop("ny"), d.pop("dx")
    return make_config(nx, ny, dx, **d)


# ------------------------------------------------------------ tuning cache

def tune_cache_path() -> str:
    """JSON file of tuned tile shapes (PHX_TUNE_CACHE, else ~/.cache/phx_tune.json)."""
    return os.environ.get("PHX_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "phx_tune.json")


def tune_key(cfg: phx_config, has_v: bool, device_name: str = "") -> str:
    return (f"{device_name}|k{cfg.kernel}|p{cfg.precision}|{cfg.nx}x{cfg.ny}|c{cfg.components}|"
            f"r{cfg.reservoir}|v{int(has_v)}|bc{cfg.bc_x}{cfg.bc_y}")


def _read_cache(path):
    import json
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def cached_shape(cfg: phx_config, has_v: bool, device_name: str = ""):
    """(tile_wx, tile_rows) stored for this configuration, or None."""
    v = _read_cache(tune_cache_path()).get(tune_key(cfg, has_v, device_name))
    return None if v is None else (int(v["tile_wx"]), int(v["tile_rows"]))


def store_shape(cfg: phx_config, has_v: bool, result: phx_tune_result, device_name: str = "") -> None:
    import json
    path = tune_cache_path()
    d = _read_cache(path)
    d[tune_key(cfg, has_v, device_name)] = result.as_dict()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + f".{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1)
    os.replace(tmp, path)


def torch_dtypes(precision: int):
    import torch
    return (torch.complex64, torch.float32) if precision == PHX_C64 else (torch.complex128, torch.float64)


class Solver:
    """A handle bound to torch tensors on the current GPU and stream.

    psi: complex tensor [components, ny, nx] (complex64 for PHX_C64, complex128 for
    PHX_C128); n, P: real [components, ny, nx] when the reservoir is on; V: real
    [ny, nx] or None.  The tensors are updated in place by `step`."""

    def __init__(self, cfg: phx_config, psi, n=None, V=None, P=None, stream=None, E=None):
        import torch
        cdt, rdt = torch_dtypes(cfg.precision)
        shape = (cfg.components, cfg.ny, cfg.nx)
        if psi.dtype != cdt or tuple(psi.shape) != shape or not psi.is_contiguous() or not psi.is_cuda:
            raise ValueError(f"psi must be a contiguous {cdt} CUDA tensor of shape {shape}")
        if E is not None and (E.dtype != cdt or tuple(E.shape) != shape or not E.is_contiguous() or not E.is_cuda):
            raise ValueError(f"E must be a contiguous {cdt} CUDA tensor of shape {shape}")
        for name, t, shp in (("n", n, shape), ("P", P, shape), ("V", V, (cfg.ny, cfg.nx))):
            if t is not None and (t.dtype != rdt or tuple(t.shape) != shp or not t.is_contiguous() or not t.is_cuda):
                raise ValueError(f"{name} must be a contiguous {rdt} CUDA tensor of shape {shp}")
        self.cfg = cfg
        self.psi, self.n, self.V, self.P, self.E = psi, n, V, P, E
        nbytes = phx_workspace_bytes(cfg)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=psi.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(psi.device)
        ptr = lambda t: None if t is None else t.data_ptr()
        self.fields = phx_fields(ptr(psi), ptr(n), ptr(V), ptr(P), self.workspace.data_ptr(), nbytes, ptr(E))
        self.handle = phx_create(cfg, self.fields, self.stream.cuda_stream)

    def step(self, n_steps: int = 1) -> dict:
        return phx_step(self.handle, n_steps).as_dict()

    def observables(self) -> dict:
        return phx_observables(self.handle).as_dict()

    def info(self) -> dict:
        return phx_get_info(self.handle).as_dict()

    def set_info(self, **kw) -> None:
        cur = phx_get_info(self.handle)
        for k, v in kw.items():
            setattr(cur, k, v)
        phx_set_info(self.handle, cur)

    def log_attempts(self, cap: int) -> None:
        """Start logging RK45 attempts (dt, error norm, accepted) into a host array of
        `cap` entries; `attempts()` returns the entries logged so far."""
        import numpy as np
        self._att_log = np.zeros(3 * max(int(cap), 1), np.float64)
        self._att_count = np.zeros(1, np.int64)
        phx_log_attempts(self.handle, self._att_log, int(cap), self._att_count)

    def attempts(self):
        """[k, 3] array of (dt, err, accepted) of the attempts logged so far."""
        return self._att_log[:3 * int(self._att_count[0])].reshape(-1, 3).copy()

    def set_timing(self, enable: bool = True) -> None:
        phx_set_timing(self.handle, enable)

    def kernel_times(self) -> dict:
        return phx_kernel_times(self.handle).as_dict()

    def autotune(self, reps: int = 10, use_cache: bool = True) -> dict:
        """Pick the fastest tile shape for this grid (phx_autotune); results are
        cached per device and configuration in the JSON tuning cache."""
        import torch
        dev = torch.cuda.get_device_name(self.psi.device)
        has_v = self.V is not None
        if use_cache:
            shp = cached_shape(self.cfg, has_v, dev)
            if shp is not None and shp != (self.cfg.tile_wx, self.cfg.tile_rows):
                cfg = phx_config.from_buffer_copy(self.cfg)
                cfg.tile_wx, cfg.tile_rows = shp
                phx_destroy(self.handle)
                self.cfg = cfg
                self.handle = phx_create(cfg, self.fields, self.stream.cuda_stream)
                return {"tile_wx": shp[0], "tile_rows": shp[1], "cached": True}
        r = phx_autotune(self.handle, reps)
        if use_cache:
            store_shape(self.cfg, has_v, r, dev)
        d = r.as_dict()
        d["cached"] = False
        return d

    def close(self):
        if getattr(self, "handle", None):
            phx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Packed torch buffers for many one-component instances and a persistent
    batched stepper (phx_batch_step).

    grids: list of (nx, ny); params: list of phx_config (physics, boundaries, dt);
    param_index: per-instance index into params.  Instance k's cells are
    psi[offsets[k] : offsets[k] + nx*ny] (row-major), likewise n, P, V."""

    def __init__(self, grids, params, param_index=None, precision=PHX_C64, device="cuda:0",
                 with_v=False, check_finite=False, seeds=None):
        import torch
        self.torch = torch
        self.grids = [(int(a), int(b)) for a, b in grids]
        self.precision = precision
        cdt, rdt = torch_dtypes(precision)
        align = 64  # keep every slice 256-byte aligned for the complex array
        offs, o = [], 0
        for nx, ny in self.grids:
            offs.append(o)
            o += (nx * ny + align - 1) // align * align
        self.offsets = offs
        self.total = o
        res = bool(params[0].reservoir)
        self.psi = torch.zeros(o, dtype=cdt, device=device)
        self.n = torch.zeros(o, dtype=rdt, device=device) if res else None
        self.P = torch.zeros(o, dtype=rdt, device=device) if res else None
        self.V = torch.zeros(o, dtype=rdt, device=device) if with_v else None
        pidx = param_index if param_index is not None else [0] * len(self.grids)
        sd = seeds if seeds is not None else [0] * len(self.grids)
        self._inst = (phx_instance * len(self.grids))(*[
            phx_instance(nx, ny, int(p), 0, off, int(s) & (2 ** 64 - 1))
            for (nx, ny), p, off, s in zip(self.grids, pidx, offs, sd)])
        self._params = (phx_config * len(params))(*params)
        ptr = lambda t: None if t is None else t.data_ptr()
        self.desc = phx_batch_desc(len(self.grids), precision, self._inst, self._params, len(params),
                                   int(check_finite), o, ptr(self.psi), ptr(self.n), ptr(self.P), ptr(self.V),
                                   None, 0)
        nbytes = phx_batch_workspace_bytes(self.desc)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        self.desc.workspace = self.workspace.data_ptr()
        self.desc.workspace_bytes = nbytes

    def view(self, t, k):
        nx, ny = self.grids[k]
        return t[self.offsets[k]:self.offsets[k] + nx * ny].view(ny, nx)

    def stacked(self, t):
        """All instances as one grid of count*ny rows (instances of one size whose
        slices are contiguous, i.e. nx*ny a multiple of 64); for pointwise and
        block-local kernels."""
        nx, ny = self.grids[0]
        if any(g != (nx, ny) for g in self.grids) or (nx * ny) % 64:
            raise ValueError("stacked view needs equal grids with nx*ny a multiple of 64")
        return t[:len(self.grids) * nx * ny].view(len(self.grids) * ny, nx)

    def step(self, n_steps: int, stream=None):
        """n_steps batched steps; the noise step index (desc.step0) runs on across calls."""
        s = stream if stream is not None else self.torch.cuda.current_stream(self.psi.device)
        phx_batch_step(self.desc, n_steps, s.cuda_stream)
        self.desc.step0 += n_steps


# ------------------------------------------------------------ learned corrector

def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream, device=None):
    import torch
    return (stream if stream is not None else torch.cuda.current_stream(device)).cuda_stream


def phx_cnn_sizes(cfg: phx_cnn_config):
    n = ctypes.c_int64(0)
    ws = ctypes.c_size_t(0)
    _check(load().phx_cnn_sizes(ctypes.byref(cfg), ctypes.byref(n), ctypes.byref(ws)))
    return n.value, ws.value


def phx_cnn_param_offsets(cfg: phx_cnn_config):
    w = (ctypes.c_int64 * 4)()
    b = (ctypes.c_int64 * 4)()
    kp = (ctypes.c_int32 * 4)()
    ci = (ctypes.c_int32 * 4)()
    co = (ctypes.c_int32 * 4)()
    _check(load().phx_cnn_param_offsets(ctypes.byref(cfg), w, b, kp, ci, co))
    return list(w), list(b), list(kp), list(ci), list(co)


def phx_coarsen(precision, psi_f, n_f, P_f, nx_f, ny_f, factor, psi_c, n_c, P_c, stream=None):
    _check(load().phx_coarsen(precision, _p(psi_f), _p(n_f), _p(P_f), nx_f, ny_f, factor, _p(psi_c), _p(n_c),
                              _p(P_c), _stream_handle(stream)))


def phx_corrector_features(precision, psi, n, P, nx, ny, s_psi, s_n, s_p, x, stream=None):
    _check(load().phx_corrector_features(precision, _p(psi), _p(n), _p(P), nx, ny, float(s_psi), float(s_n),
                                         float(s_p), _p(x), _stream_handle(stream)))


def phx_corrector_residual(precision, psi_ref, n_ref, psi, n, nx, ny, s_psi, s_n, r, stream=None):
    _check(load().phx_corrector_residual(precision, _p(psi_ref), _p(n_ref), _p(psi), _p(n), nx, ny, float(s_psi),
                                         float(s_n), _p(r), _stream_handle(stream)))


def phx_corrector_apply(precision, psi, n, y, nx, ny, s_psi, s_n, stream=None):
    _check(load().phx_corrector_apply(precision, _p(psi), _p(n), _p(y), nx, ny, float(s_psi), float(s_n),
                                      _stream_handle(stream)))


class Corrector:
    """The corrector network on the current GPU: FP32 master parameters and Adam
    moments as torch tensors, BF16 MFMA kernels in libphx."""

    def __init__(self, height, width, max_batch, in_channels=4, hidden=32, out_channels=3, device="cuda:0",
                 stream=None):
        import torch
        self.torch = torch
        self.cfg = phx_cnn_config(in_channels, hidden, out_channels, height, width, max_batch)
        self.n_params, ws = phx_cnn_sizes(self.cfg)
        self.w_off, self.b_off, self.kp, self.cinp, self.coutp = phx_cnn_param_offsets(self.cfg)
        self.channels = [in_channels, hidden, hidden, hidden, out_channels]
        self.params = torch.zeros(self.n_params, dtype=torch.float32, device=device)
        self.adam_m = torch.zeros_like(self.params)
        self.adam_v = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)
        self.workspace = torch.empty(max(ws, 256), dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
        self.buf = phx_cnn_buffers(self.params.data_ptr(), self.adam_m.data_ptr(), self.adam_v.data_ptr(),
                                   self.workspace.data_ptr(), ws)
        h = ctypes.c_void_p()
        _check(load().phx_cnn_create(ctypes.byref(self.cfg), ctypes.byref(self.buf), self.stream.cuda_stream,
                                     ctypes.byref(h)))
        self.handle = h
        self.step_count = 0

    # parameters as lists of (w [c_out][c_in][3][3], b [c_out]) numpy arrays
    def set_weights(self, layers):
        import numpy as np
        flat = np.zeros(self.n_params, np.float32)
        for l, (w, b) in enumerate(layers):
            co, ci = w.shape[:2]
            W = np.zeros((self.coutp[l], self.kp[l]), np.float32)
            for t in range(9):
                W[:co, t * self.cinp[l]:t * self.cinp[l] + ci] = w[:, :, t // 3, t % 3]
            flat[self.w_off[l]:self.w_off[l] + W.size] = W.ravel()
            flat[self.b_off[l]:self.b_off[l] + co] = b
        self.params.copy_(self.torch.from_numpy(flat))

    def unpack(self, flat):
        import numpy as np
        flat = np.asarray(flat, np.float64)
        out = []
        for l in range(4):
            co, ci = self.channels[l + 1], self.channels[l]
            W = flat[self.w_off[l]:self.w_off[l] + self.coutp[l] * self.kp[l]].reshape(self.coutp[l], self.kp[l])
            w = np.zeros((co, ci, 3, 3))
            for t in range(9):
                w[:, :, t // 3, t % 3] = W[:co, t * self.cinp[l]:t * self.cinp[l] + ci]
            out.append((w, flat[self.b_off[l]:self.b_off[l] + co].copy()))
        return out

    def get_weights(self):
        return self.unpack(self.params.cpu().numpy())

    def init_random(self, seed=0, scale=1.0):
        """He-style initialization, seeded on the host."""
        import numpy as np
        rng = np.random.default_rng(seed)
        layers = []
        for l in range(4):
            ci, co = self.channels[l], self.channels[l + 1]
            std = scale * np.sqrt(2.0 / (9 * ci))
            if l == 3:
                std *= 0.1  # start close to "no correction"
            layers.append((rng.standard_normal((co, ci, 3, 3)) * std, np.zeros(co)))
        self.set_weights(layers)
        self.adam_m.zero_()
        self.adam_v.zero_()
        self.step_count = 0

    def forward(self, x, y=None):
        b = x.shape[0]
        if y is None:
            y = self.torch.empty((b, self.cfg.height, self.cfg.width, self.cfg.out_channels), dtype=self.torch.float32,
                                 device=x.device)
        _check(load().phx_cnn_forward(self.handle, _p(x), b, _p(y)))
        return y

    def gradients(self, x, target):
        _check(load().phx_cnn_gradients(self.handle, _p(x), _p(target), x.shape[0], _p(self.grads), _p(self.loss)))
        return self.grads

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, grads=None):
        self.step_count += 1
        g = self.grads if grads is None else grads
        _check(load().phx_cnn_adam(self.handle, _p(g), self.step_count, lr, beta1, beta2, eps))

    def train_step(self, x, target, lr):
        self.step_count += 1
        _check(load().phx_cnn_train_step(self.handle, _p(x), _p(target), x.shape[0], self.step_count, lr,
                                         _p(self.loss)))
        return self.loss

    def close(self):
        if getattr(self, "handle", None):
            load().phx_cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
