"""MI355X (gfx950) acoustic wave propagation: 25-point radius-4 stencil,
leapfrog time stepping, damping layer, point sources and receivers.

The compute path is the HIP library `libwave.so` behind the C ABI in
`include/wave.h`; `paper_2009_04619_amd.wave` is its ctypes binding (import
it explicitly: it loads torch and the library).  Build with
`python -m paper_2009_04619_amd.build`.
"""
__all__ = ["build", "wave"]


def build(verbose: bool = False) -> str:
    from .build import build as _b
    return _b(verbose=verbose)
