"""Host-side checks of the C-ABI boundary that need no GPU: the library loads and
exports every entry point declared in include/phx.h, the ctypes structures match
the C layout, configuration validation rejects bad input with the documented
status, and the byte model reproduces Table 1 of the paper."""
import json
import os
import re
import subprocess

import pytest

from paper_2411_18341_amd import bytemodel, phx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "phx.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(phx_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_entry_point():
    lib = phx.load()
    names = header_functions()
    assert set(names) == set(phx.ENTRY_POINTS), (names, phx.ENTRY_POINTS)
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", phx.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (phx_\w+)", out))
    assert set(names) <= exported


def _c_layout():
    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "phx.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m));
int main(void) {
  printf("phx_config %zu\n", sizeof(phx_config)); F(phx_config, dx) F(phx_config, bc_x) F(phx_config, hbar)
  F(phx_config, delta_lt) F(phx_config, dt) F(phx_config, dt_max) F(phx_config, kernel) F(phx_config, tile_rows) F(phx_config, graph_steps) F(phx_config, noise) F(phx_config, seed) F(phx_config, drive_omega) F(phx_config, drive) F(phx_config, imag_time)
  printf("phx_fields %zu\n", sizeof(phx_fields)); F(phx_fields, workspace_bytes)
  printf("phx_obs %zu\n", sizeof(phx_obs)); F(phx_obs, energy) F(phx_obs, max_density) F(phx_obs, nonfinite) F(phx_obs, norm_renorm)
  printf("phx_info %zu\n", sizeof(phx_info)); F(phx_info, steps_rejected) F(phx_info, nonfinite)
  printf("phx_timing %zu\n", sizeof(phx_timing)); F(phx_timing, launches) F(phx_timing, ms_total)
  printf("phx_tune_result %zu\n", sizeof(phx_tune_result)); F(phx_tune_result, best_us) F(phx_tune_result, default_us)
  printf("phx_instance %zu\n", sizeof(phx_instance)); F(phx_instance, offset) F(phx_instance, seed)
  printf("phx_batch_desc %zu\n", sizeof(phx_batch_desc)); F(phx_batch_desc, params) F(phx_batch_desc, psi)
  F(phx_batch_desc, workspace_bytes) F(phx_fields, E) F(phx_batch_desc, step0)
  return 0; }
'''
    return prog


def test_ctypes_structures_match_c_layout(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(_c_layout())
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines():
        k, v = line.split()
        got[k] = int(v)
    import ctypes
    for cname, cls in (("phx_config", phx.phx_config), ("phx_fields", phx.phx_fields), ("phx_obs", phx.phx_obs),
                       ("phx_info", phx.phx_info), ("phx_timing", phx.phx_timing),
                       ("phx_tune_result", phx.phx_tune_result), ("phx_instance", phx.phx_instance),
                       ("phx_batch_desc", phx.phx_batch_desc)):
        assert got[cname] == ctypes.sizeof(cls), cname
        for key, off in got.items():
            if key.startswith(cname + "."):
                field = key.split(".", 1)[1]
                assert getattr(cls, field).offset == off, key


def good_config(**kw):
    d = dict(g=1.0, dt=1e-3)
    d.update(kw)
    return phx.make_config(64, 48, 0.1, **d)


def test_workspace_bytes_scale_with_precision_and_reservoir():
    a = phx.phx_workspace_bytes(good_config(kernel=phx.PHX_KERNEL_STAGE))
    b = phx.phx_workspace_bytes(good_config(kernel=phx.PHX_KERNEL_STAGE, precision=phx.PHX_C128))
    c = phx.phx_workspace_bytes(good_config(kernel=phx.PHX_KERNEL_STAGE, reservoir=True))
    assert 0 < a < b and a < c
    # stage kernels: three complex buffers (two stage arguments and the running sum)
    assert a >= 3 * 64 * 48 * 8
    # whole-step kernel: two more state buffers (alternate steps; the tuner's trials)
    d = phx.phx_workspace_bytes(good_config(kernel=phx.PHX_KERNEL_STEP))
    assert 2 * 64 * 48 * 8 <= d < a
    assert phx.phx_workspace_bytes(good_config()) == d  # AUTO picks the whole-step kernel
    # spinor: the streaming whole-step kernel (two state buffers of both components,
    # with the reservoir two of both reservoirs), bands of 40 or 64 rows, also in
    # imaginary time and with the drive (without reservoirs)
    s = phx.phx_workspace_bytes(good_config(kernel=phx.PHX_KERNEL_STEP, components=2, delta_lt=0.1))
    assert 2 * 2 * 64 * 48 * 8 <= s
    assert phx.phx_workspace_bytes(good_config(components=2, delta_lt=0.1)) == s
    sr = phx.phx_workspace_bytes(good_config(kernel=phx.PHX_KERNEL_STEP, components=2, reservoir=True))
    assert sr >= s + 2 * 2 * 64 * 48 * 4
    for bad in (dict(tile_wx=8, tile_rows=4), dict(tile_wx=1, tile_rows=88)):
        with pytest.raises(phx.PhxError) as e:
            phx.phx_workspace_bytes(good_config(kernel=phx.PHX_KERNEL_STEP, components=2, **bad))
        assert e.value.status == phx.PHX_EINVAL, bad
    # with the drive: the streaming kernel without reservoirs, the stage-fused kernels with them
    sd = phx.phx_workspace_bytes(good_config(kernel=phx.PHX_KERNEL_STEP, components=2, drive=True, tile_wx=1,
                                             tile_rows=64))
    assert phx.phx_workspace_bytes(good_config(components=2, drive=True)) == sd
    with pytest.raises(phx.PhxError) as e:
        phx.phx_workspace_bytes(good_config(kernel=phx.PHX_KERNEL_STEP, components=2, drive=True, reservoir=True))
    assert e.value.status == phx.PHX_EUNSUPPORTED
    si = phx.phx_workspace_bytes(good_config(kernel=phx.PHX_KERNEL_STEP, components=2, delta_lt=0.1,
                                             imag_time=True, tile_wx=1, tile_rows=40))
    assert phx.phx_workspace_bytes(good_config(components=2, delta_lt=0.1, imag_time=True)) == si


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("ny", -3), ("dx", 0.0), ("dy", float("nan")), ("bc_x", 2), ("components", 3),
    ("reservoir", 2), ("precision", 5), ("integrator", 9), ("hbar", 0.0), ("mass", -1.0),
    ("g", float("inf")), ("dt", 0.0), ("dt", 1.0), ("kernel", 7),
    ("tile_wx", 5), ("tile_rows", 5), ("tile_rows", 65), ("noise", -1.0), ("noise", float("nan")),
    ("drive", 2), ("drive_omega", float("inf")), ("imag_time", 2),
])
def test_invalid_config_rejected(field, value):
    cfg = good_config()
    setattr(cfg, field, value)
    with pytest.raises(phx.PhxError) as e:
        phx.phx_workspace_bytes(cfg)
    assert e.value.status == phx.PHX_EINVAL
    assert phx.phx_last_error()


def test_noise_config_validation():
    """Wiener noise: RK4 only; it adds one 256-byte slot (the step index) to the
    workspace; the seed takes all 64 bits."""
    base = phx.phx_workspace_bytes(good_config())
    assert phx.phx_workspace_bytes(good_config(noise=1.0, seed=2 ** 64 - 1)) == base + 256
    assert phx.phx_workspace_bytes(good_config(noise=1.0, kernel=phx.PHX_KERNEL_STAGE)) == \
        phx.phx_workspace_bytes(good_config(kernel=phx.PHX_KERNEL_STAGE)) + 256
    with pytest.raises(phx.PhxError) as e:
        phx.phx_workspace_bytes(good_config(noise=1.0, integrator=phx.PHX_RK45))
    assert e.value.status == phx.PHX_EUNSUPPORTED


def test_drive_config_validation():
    """Coherent drive: one component runs on the streaming whole-step kernel with bands
    of 40 or 64 rows (region shapes and other bands rejected), the stage-fused family on
    request or for the spinor; RK4 adds the step-index slot and four stage phasors."""
    stage = phx.phx_workspace_bytes(good_config(kernel=phx.PHX_KERNEL_STAGE))
    step = phx.phx_workspace_bytes(good_config())
    assert phx.phx_workspace_bytes(good_config(drive=True, drive_omega=1.5)) == step + 256 + 256
    assert phx.phx_workspace_bytes(good_config(drive=True, kernel=phx.PHX_KERNEL_STAGE)) == stage + 256 + 256
    phx.phx_workspace_bytes(good_config(drive=True, kernel=phx.PHX_KERNEL_STEP, tile_wx=1, tile_rows=64))
    for bad in (dict(tile_wx=8, tile_rows=4), dict(tile_wx=1, tile_rows=88)):
        with pytest.raises(phx.PhxError) as e:
            phx.phx_workspace_bytes(good_config(drive=True, kernel=phx.PHX_KERNEL_STEP, **bad))
        assert e.value.status == phx.PHX_EINVAL, bad
    rk45 = phx.phx_workspace_bytes(good_config(integrator=phx.PHX_RK45))
    assert phx.phx_workspace_bytes(good_config(integrator=phx.PHX_RK45, drive=True)) == rk45


def test_imag_time_config_validation():
    """Imaginary time: the conservative equation; one component runs on the streaming
    whole-step kernel, one-column or wide walk (region shapes rejected), two on the spinor
    walk, the stage-fused family on request; RK4's stability bound on the negative real
    axis (2.78) replaces the imaginary-axis one."""
    stage = phx.phx_workspace_bytes(good_config(kernel=phx.PHX_KERNEL_STAGE))
    step = phx.phx_workspace_bytes(good_config())
    assert phx.phx_workspace_bytes(good_config(imag_time=True, kernel=phx.PHX_KERNEL_STAGE)) == stage + 256 + 256
    assert phx.phx_workspace_bytes(good_config(imag_time=True)) == step + 256 + 256
    phx.phx_workspace_bytes(good_config(imag_time=True, tile_wx=1, tile_rows=64))
    phx.phx_workspace_bytes(good_config(imag_time=True, tile_wx=2, tile_rows=0))    # the wide walk
    phx.phx_workspace_bytes(good_config(imag_time=True, tile_wx=3, tile_rows=8))
    phx.phx_workspace_bytes(good_config(imag_time=True, components=2, delta_lt=0.1))   # spinor walk
    for bad in (dict(reservoir=True), dict(gamma_c=0.1), dict(R=0.1), dict(noise=1.0), dict(drive=True),
                dict(tile_wx=8, tile_rows=4)):
        with pytest.raises(phx.PhxError) as e:
            phx.phx_workspace_bytes(good_config(imag_time=True, **bad))
        assert e.value.status == phx.PHX_EINVAL, bad
    with pytest.raises(phx.PhxError) as e:
        phx.phx_workspace_bytes(good_config(imag_time=True, integrator=phx.PHX_RK45))
    assert e.value.status == phx.PHX_EUNSUPPORTED
    lam = 0.5 * 4 * (2 / 0.1 ** 2)  # hbar/2m * 4 (1/dx^2 + 1/dy^2)
    phx.phx_workspace_bytes(good_config(dt=2.7 / lam))                 # real time: bound 2.83
    phx.phx_workspace_bytes(good_config(dt=2.75 / lam, imag_time=True))
    with pytest.raises(phx.PhxError):
        phx.phx_workspace_bytes(good_config(dt=2.8 / lam, imag_time=True))


def test_rk45_tolerance_validation():
    cfg = good_config(integrator=phx.PHX_RK45, rtol=0.0, atol=0.0)
    with pytest.raises(phx.PhxError) as e:
        phx.phx_workspace_bytes(cfg)
    assert e.value.status == phx.PHX_EINVAL
    cfg = good_config(integrator=phx.PHX_RK45, dt_min=1e-3, dt_max=1e-4)
    with pytest.raises(phx.PhxError):
        phx.phx_workspace_bytes(cfg)


def test_grid_size_limit():
    cfg = phx.make_config(65536, 32768, 0.1, g=1.0, dt=1e-3)
    with pytest.raises(phx.PhxError) as e:
        phx.phx_workspace_bytes(cfg)
    assert e.value.status == phx.PHX_EINVAL


def test_create_rejects_bad_fields_without_touching_the_gpu():
    """Field validation happens on the host before any HIP call."""
    cfg = good_config(reservoir=True)
    ws = phx.phx_workspace_bytes(cfg)
    bad = [phx.phx_fields(None, 256, None, 512, 1024, ws),          # psi NULL
           phx.phx_fields(256, None, None, 512, 1024, ws),          # reservoir without n
           phx.phx_fields(256 + 8, 512, None, 768, 1024, ws)]       # misaligned psi
    for f in bad:
        with pytest.raises(phx.PhxError) as e:
            phx.phx_create(cfg, f, None)
        assert e.value.status == phx.PHX_EINVAL
    with pytest.raises(phx.PhxError) as e:
        phx.phx_create(cfg, phx.phx_fields(256, 512, None, 768, 1024, ws - 1), None)
    assert e.value.status == phx.PHX_EWORKSPACE


def test_byte_model_reproduces_table1(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "table1_rw_counts.json")))
    for k, v in g["kernels"].items():
        assert bytemodel.PAPER_TABLE1[k] == (v["reads"], v["writes"], v["launches_per_step"])
    m32, m64 = bytemodel.paper_unfused_rk4(4), bytemodel.paper_unfused_rk4(8)
    assert (m32["reads"], m32["writes"]) == (g["rk4_iteration"]["reads"], g["rk4_iteration"]["writes"])
    assert m32["bytes_per_point"] == g["bytes_per_point_per_step"]["fp32"]
    assert m64["bytes_per_point"] == g["bytes_per_point_per_step"]["fp64"]


def test_stage_fused_byte_model():
    # scalar, no reservoir, no V, complex64: 3 launches of (read 3 c + write 2 c) ...
    m = bytemodel.rk4_stage_fused(4, False, False)
    assert m["stage1"] == 8 + 16 and m["stage2"] == 24 + 16 and m["stage4"] == 24 + 8
    assert m["step"] == 136
    # driven-dissipative physics (reservoir, pump, no V): 220 B per point and step
    assert bytemodel.rk4_stage_fused(4, True, False)["step"] == 220
    assert bytemodel.rk4_stage_fused(8, True, False)["step"] == 440
    assert bytemodel.state_minimum(4, True, False) == 28


def test_tile_shape_validation_per_family():
    # stage-fused kernels: waves across x in {1, 2, 4}, rows 1..64
    phx.phx_workspace_bytes(good_config(kernel=phx.PHX_KERNEL_STAGE, tile_wx=2, tile_rows=64))
    with pytest.raises(phx.PhxError):
        phx.phx_workspace_bytes(good_config(kernel=phx.PHX_KERNEL_STAGE, tile_wx=8, tile_rows=4))
    # whole-step kernel: only the instantiated region shapes
    phx.phx_workspace_bytes(good_config(tile_wx=16, tile_rows=4))
    phx.phx_workspace_bytes(good_config(tile_wx=8, tile_rows=8))
    phx.phx_workspace_bytes(good_config(precision=phx.PHX_C128, tile_wx=16, tile_rows=2))
    for bad in [(4, 4), (16, 8), (2, 3)]:
        with pytest.raises(phx.PhxError) as e:
            phx.phx_workspace_bytes(good_config(tile_wx=bad[0], tile_rows=bad[1]))
        assert e.value.status == phx.PHX_EINVAL
    # streaming form: tile_wx 1 with the instantiated band lengths, state under 2 GiB
    for band in (40, 64, 88, 112):
        phx.phx_workspace_bytes(good_config(tile_wx=1, tile_rows=band))
    phx.phx_workspace_bytes(good_config(precision=phx.PHX_C128, tile_wx=1, tile_rows=64))
    for bad in [(1, 44), (1, 16)]:
        with pytest.raises(phx.PhxError):
            phx.phx_workspace_bytes(good_config(tile_wx=bad[0], tile_rows=bad[1]))
    # wide streaming form: tile_wx 2 (8-row ring) or 3 (12-row ring), bands of 8..4096
    # rows or 0 (chosen per device), complex64 on grids of even width
    for shape in [(2, 0), (3, 0), (2, 40), (3, 200), (2, 4096)]:
        phx.phx_workspace_bytes(good_config(tile_wx=shape[0], tile_rows=shape[1]))
    for bad in [(2, 3), (3, 5000), (2, -1)]:
        with pytest.raises(phx.PhxError) as e:
            phx.phx_workspace_bytes(good_config(tile_wx=bad[0], tile_rows=bad[1]))
        assert e.value.status == phx.PHX_EINVAL
    with pytest.raises(phx.PhxError):
        phx.phx_workspace_bytes(good_config(precision=phx.PHX_C128, tile_wx=2, tile_rows=40))
    odd = good_config(tile_wx=3, tile_rows=64)
    odd.nx = 255
    with pytest.raises(phx.PhxError) as e:
        phx.phx_workspace_bytes(odd)
    assert e.value.status == phx.PHX_EINVAL
    big = good_config(tile_wx=1, tile_rows=40)
    big.nx, big.ny = 16384, 16384          # 2 GiB of complex64 state
    with pytest.raises(phx.PhxError) as e:
        phx.phx_workspace_bytes(big)
    assert e.value.status == phx.PHX_EINVAL
    big.tile_wx, big.tile_rows = 8, 8      # the region form has no such limit
    phx.phx_workspace_bytes(big)


def test_tune_cache_roundtrip(tmp_path, monkeypatch):
    monkeypatch.setenv("PHX_TUNE_CACHE", str(tmp_path / "tune.json"))
    cfg = good_config()
    assert phx.cached_shape(cfg, False, "dev") is None
    r = phx.phx_tune_result(phx.PHX_KERNEL_STEP, 8, 4, 5, 10.0, 12.0)
    phx.store_shape(cfg, False, r, "dev")
    assert phx.cached_shape(cfg, False, "dev") == (8, 4)
    assert phx.cached_shape(cfg, True, "dev") is None


def _desc(grids, offsets, total, params=None, ws=1 << 30):
    params = params or [phx.make_config(8, 8, 0.2, reservoir=True, g=0.01, R=0.01, gamma_c=0.15,
                                        gamma_r=0.225, dt=0.02)]
    inst = (phx.phx_instance * len(grids))(*[phx.phx_instance(nx, ny, 0, 0, o)
                                             for (nx, ny), o in zip(grids, offsets)])
    pa = (phx.phx_config * len(params))(*params)
    d = phx.phx_batch_desc(len(grids), phx.PHX_C64, inst, pa, len(params), 0, total, 256, 512, 768,
                           None, 1024, ws)
    d._keep = (inst, pa)
    return d


def test_batch_descriptor_validation():
    ok = _desc([(10, 10), (20, 5)], [0, 100], 200)
    assert phx.phx_batch_workspace_bytes(ok) > 200 * 8
    bad_cases = [
        _desc([(10, 10), (20, 5)], [0, 50], 200),        # overlap
        _desc([(10, 10), (20, 5)], [0, 150], 200),       # past total_cells
        _desc([(0, 10)], [0], 200),                      # empty grid
        _desc([(10, 10)], [-1], 200),                    # negative offset
    ]
    for d in bad_cases:
        with pytest.raises(phx.PhxError) as e:
            phx.phx_batch_workspace_bytes(d)
        assert e.value.status == phx.PHX_EINVAL
    d = _desc([(10, 10)], [0], 200)
    d.instances[0].param_index = 3
    with pytest.raises(phx.PhxError):
        phx.phx_batch_workspace_bytes(d)
    unstable = _desc([(10, 10)], [0], 200, params=[phx.make_config(8, 8, 0.2, dt=1.0)])
    with pytest.raises(phx.PhxError):
        phx.phx_batch_workspace_bytes(unstable)
    small = _desc([(10, 10)], [0], 200, ws=16)
    with pytest.raises(phx.PhxError) as e:
        phx.phx_batch_step(small, 1, None)
    assert e.value.status == phx.PHX_EWORKSPACE


def test_profile_kernel_names():
    """Kernel names in rocprofv3 output map to the kinds the counter records use."""
    from paper_2411_18341_amd.profiling import kernel_kind
    cases = {
        "void phx::rk4_stream_kernel<float, true, false, false, false, 40, false>(phx::StepArgs<float>)": "rk4_step_1x40",
        "void phx::rk4_stream_kernel<double, false, true, true, true, 64, true>(phx::StepArgs<double>)": "rk4_step_1x64",
        "void phx::rk4_stream_drive_kernel<float, true, false, false, false, 64>(phx::StepArgs<float>)": "rk4_step_1x64",
        "void phx::rk4_step_kernel<float, true, false, false, 12, 6>(phx::StepArgs<float>)": "rk4_step_12x6",
        "void phx::rk4_stage_kernel<float, 1, true, false, 3>(phx::Rk4Args<float>)": "rk4_stage3",
        "void (anonymous namespace)::wiener_noise_kernel<float, true>(float2*, float const*)": "wiener_noise",
        "void phx::rk4_stream_wide_kernel<true, false, false, false, 8, 3, 3, false>(phx::StepArgs<float>)":
            "rk4_step_wide8",
        "void phx::rk4_stream_wide_kernel<false, true, true, true, 12, 6, 2, true>(phx::StepArgs<float>)":
            "rk4_step_wide12",
        "void phx::rk4_stream_wide_kernel<true, false, false, false, 8, 3, 2, false, true, false>(phx::StepArgs<float>)":
            "rk4_step_wide8",   # with the noise drawn in the step
        "void phx::rk4_stream_wide_kernel<false, true, false, false, 12, 6, 2, true, false, true>(phx::StepArgs<float>)":
            "rk4_step_wide12",  # imaginary time
    }
    for name, kind in cases.items():
        assert kernel_kind(name) == kind, name


def test_walk_pattern_rejects_bad_arguments_without_touching_the_gpu():
    """phx_walk_pattern (measurement only) validates on the host: NULL or unaligned
    pointers, odd or empty grids, band heights outside 8..4096, a psi of 2 GiB or
    more, outputs that overlap the inputs."""
    vp = lambda a: phx.ctypes.c_void_p(a)
    base = [vp(0x100000), vp(0x200000), vp(0x300000), vp(0x400000), vp(0x500000)]
    cases = [
        ([None] + base[1:], 64, 64, 0),
        ([vp(0x100010)] + base[1:], 64, 64, 0),
        (base, 63, 64, 0),
        (base, 64, 0, 0),
        (base, 64, 64, 7),
        (base, 64, 64, 5000),
        (base, 16384, 16384, 0),
        ([vp(0x300000)] + base[1:], 64, 64, 0),   # psi_out on psi_in
    ]
    for ptrs, nx, ny, rows in cases:
        with pytest.raises(phx.PhxError) as e:
            phx.phx_walk_pattern(*ptrs, nx, ny, rows, None)
        assert e.value.status == phx.PHX_EINVAL, (nx, ny, rows)
