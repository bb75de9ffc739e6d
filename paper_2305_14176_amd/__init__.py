"""MI355X-native (gfx950) Yee FDTD time step behind a C ABI (``include/yee.h``).

``YeeSolver`` (in :mod:`.solver`) wraps one context of ``libyee.so``;
:mod:`.workloads` draws the seeded synthetic inputs.  Importing this package
loads nothing; the HIP library is loaded on first use and a missing library
is an error (there is no CPU fallback).
"""

__all__ = ["YeeSolver"]


def __getattr__(name):
    if name == "YeeSolver":
        from .solver import YeeSolver
        return YeeSolver
    raise AttributeError(name)
