"""sdq: stabilized DQMC Green's functions on MI355X (gfx950).

Python binding over the C ABI declared in include/sdq.h.  The binding only
marshals arguments; every step of the method runs in the HIP library
libsdq.so.  `workloads` builds seeded synthetic inputs.
"""
__all__ = ["workloads"]


def __getattr__(name):
    if name in ("binding", "sdq"):
        from . import binding
        return binding
    raise AttributeError(name)
