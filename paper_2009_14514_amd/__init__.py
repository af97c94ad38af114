"""Regional time stepping (RTS) SPH on AMD MI355X.

The simulation runs in librts.so (HIP, gfx950) behind the C ABI declared in
include/rts.h.  ``_rts`` binds that ABI with ctypes; ``sim.Simulation`` adds
torch-allocated device memory and streams; ``scenes`` builds seeded inputs.
"""
from . import scenes  # noqa: F401

__all__ = ["scenes", "sim", "_rts"]
