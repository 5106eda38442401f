"""MI355X (gfx950) solver for the 2D dissipative nonlinear Schroedinger /
Gross-Pitaevskii equation of arXiv 2411.18341 (PHOENIX).

The time integration runs in the HIP library libphx.so (C interface in
include/phx.h); `phx` is its ctypes binding, `inputs` builds seeded synthetic
workloads, `bytemodel` holds the algorithmic byte counts used for roofline
figures, and `build` compiles the library.  Submodules are imported on use so
that importing the input generators never loads the GPU library.
"""
import importlib

__all__ = ["phx", "inputs", "bytemodel", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
