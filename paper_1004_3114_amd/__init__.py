"""Wallace's normal generator (Brent 1997) on MI355X: the pool-regeneration
pass as hand-written HIP kernels behind a C ABI (include/wallace.h).

Python side: ``wallace`` (ctypes binding), ``workloads`` (seeded shapes of
the benchmark configurations), ``build`` (compiles libwallace.so in-tree).
"""
from . import workloads  # noqa: F401

__all__ = ["workloads"]
