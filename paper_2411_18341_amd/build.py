"""Builds libphx.so (the HIP/gfx950 solver library) in-tree with hipcc.

Every translation unit under csrc/ is compiled for gfx950 only, with packed FP32
instructions disabled, and linked into paper_2411_18341_amd/libphx.so next to
this file.  Run as `python -m paper_2411_18341_amd.build`.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libphx.so")
BUILD_DIR = os.path.join(HERE, "_build")
SOURCES = ["rk4_step.hip", "rk4_stream_spinor_res_f40.hip", "rk4_stream_spinor_res_f64.hip", "rk4_stream_spinor_res_d40.hip", "rk4_stream_spinor_res_d64.hip", "rk4_stream_spinor_imag_f.hip", "rk4_stream_spinor_imag_d.hip", "rk4_stream_spinor_drive_f.hip", "rk4_stream_spinor_drive_d.hip", "runtime.hip", "rk4.hip", "reduce.hip", "dopri5.hip", "batch.hip", "autotune.hip", "cnn.hip", "noise.hip", "drive.hip", "imag.hip", "rk4_stream_drive.hip", "rk4_stream_spinor.hip", "rk4_stream_wide.hip", "copy.hip", "static_obs.hip"]

ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC,
]

# The streaming whole-step kernels keep their row rings in registers only when the
# walk's 24-row loop is unrolled completely (every ring index is then a constant);
# the two-component walk with reservoirs is larger than LLVM's default size limit
# for a requested full unroll, so its unit raises that limit.
_FULL_UNROLL = ["-mllvm", "-pragma-unroll-threshold=40000"]
EXTRA_FLAGS = {f"rk4_stream_spinor{t}.hip": _FULL_UNROLL
               for t in ("", "_res_f40", "_res_f64", "_res_d40", "_res_d64", "_imag_f", "_imag_d", "_drive_f", "_drive_d")}
# the wide walk with the Wiener increment drawn at its final store (a generator call
# per position) likewise exceeds the default limit
EXTRA_FLAGS["rk4_stream_wide.hip"] = _FULL_UNROLL
# Units whose streaming kernels are checked for private (scratch) memory: a ring
# that is not in registers makes the walk several times slower.
STREAM_SOURCES = {"rk4_step.hip", "rk4_stream_drive.hip", "rk4_stream_wide.hip", "batch.hip"} | set(EXTRA_FLAGS)
_USAGE = "-Rpass-analysis=kernel-resource-usage"


def _scratch_kernels(stderr: str) -> list:
    """(kernel, bytes per lane) of every streaming kernel with scratch memory, read
    from the compiler's resource-usage remarks."""
    out, name = [], None
    for line in stderr.splitlines():
        if "Function Name:" in line:
            name = line.split("Function Name:")[1].split("[")[0].strip()
        elif "ScratchSize [bytes/lane]:" in line and name and ("stream" in name or "batch_wide" in name):
            size = int(line.split("ScratchSize [bytes/lane]:")[1].split("[")[0])
            if size:
                out.append((name, size))
    return out


# A store of more than 64 bits must not have its data registers rewritten by the very
# next instruction: on gfx950 the store may still be reading them (the compiler keeps
# a wait state only when the store's scalar offset is a constant).  The streaming
# kernels put the whole offset of such stores in the VGPR operand; this finds any
# store in the device assembly whose data a VALU instruction rewrites within
# `min_gap` instructions of straight-line code.
_WIDE_STORE = re.compile(r"^(buffer|global|flat)_store_dwordx(3|4)\s+(\S+)")
_VREGS = re.compile(r"v\[(\d+):(\d+)\]|(?<![\w\[])v(\d+)\b")


def _vregs(operand: str) -> set:
    out = set()
    for m in _VREGS.finditer(operand):
        if m.group(3) is not None:
            out.add(int(m.group(3)))
        else:
            out.update(range(int(m.group(1)), int(m.group(2)) + 1))
    return out


def store_data_hazards(asm: str, min_gap: int = 1) -> list:
    """(function, store, writer) for each store of more than 64 bits followed, with fewer
    than `min_gap` instructions in between, by a VALU write to one of its data VGPRs."""
    found, func, body = [], None, []

    def scan():
        for i, inst in enumerate(body):
            m = _WIDE_STORE.match(inst)
            if not m:
                continue
            ops = [o.strip() for o in inst.split(None, 1)[1].split(",")]
            data = _vregs(ops[0] if m.group(1) == "buffer" else ops[1])
            for k, nxt in enumerate(body[i + 1:i + 1 + min_gap]):
                if nxt == "<label>" or nxt.startswith(("s_branch", "s_cbranch", "s_setpc")):
                    break
                op = nxt.split(None, 1)
                if (op[0].startswith("v_") and not op[0].startswith(("v_cmp", "v_readlane", "v_readfirstlane"))
                        and len(op) > 1 and _vregs(op[1].split(",")[0]) & data):
                    found.append((func, inst, nxt))
                    break

    for line in asm.splitlines():
        s = line.strip()
        head = re.match(r"^([A-Za-z_.$][\w.$]*):", s)
        if head and not s.startswith("."):
            scan()
            func, body = head.group(1), []
            continue
        if head:  # a block label
            body.append("<label>")
            continue
        if not s or s.startswith((";", ".")):
            continue
        body.append(s.split(";")[0].strip())
    scan()
    return found


def device_asm(src: str) -> str:
    """gfx950 assembly of one source of the library, compiled with the build's flags."""
    out = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".s")
    os.makedirs(BUILD_DIR, exist_ok=True)
    cmd = [hipcc(), *FLAGS, *EXTRA_FLAGS.get(src, []), "--cuda-device-only", "-S",
           os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc -S failed on {src}:\n{r.stderr}")
    with open(out) as f:
        return f.read()


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the HIP library cannot be built")
    return path


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    extra = EXTRA_FLAGS.get(src, []) + ([_USAGE] if src in STREAM_SOURCES else [])
    cmd = [hipcc(), *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    spilled = _scratch_kernels(r.stderr)
    if spilled:
        raise RuntimeError(f"streaming kernels of {src} use scratch memory: {spilled}")
    if r.stderr.strip():
        # hipcc's host pass does not know the packed-fp32 feature; keep other warnings
        lines = [l for l in r.stderr.splitlines()
                 if "packed-fp32-ops" not in l and "kernel-resource-usage" not in l and l.strip()
                 and not re.match(r"^\s*\d*\s*\|", l) and not l.startswith("In file included")]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")
    return obj


def build(jobs: int = 8) -> str:
    """Compile all sources (in parallel) and link libphx.so; returns its path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
