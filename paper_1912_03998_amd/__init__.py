"""MI355X hybrid beam tracer: HIP kernels behind the C ABI of include/bt.h.

`bt` is the ctypes binding (same names as the C entry points); `tracer.Session`
keeps a context and a resident mesh for repeated runs.
"""
from . import bt  # noqa: F401

__all__ = ["bt"]
