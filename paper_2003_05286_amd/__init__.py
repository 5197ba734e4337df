"""sdq: stabilized DQMC Green's functions on MI355X (gfx950).

`binding` is the Python binding over the C ABI declared in include/sdq.h;
it only marshals arguments, every step of the method runs in the HIP library
libsdq.so.  `workloads` builds seeded synthetic inputs.
"""
__all__ = ["binding", "workloads"]
