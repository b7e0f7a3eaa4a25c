"""MI355X-native basis-expansion (SCF) N-body hot path.

The compute path lives in ``libscf.so`` (HIP kernels for gfx950 behind a C
ABI declared in ``include/scf.h``); :mod:`paper_2602_13385_amd.scf` is the thin
ctypes binding and :mod:`paper_2602_13385_amd.inputs` the seeded synthetic
input generators.  Submodules are imported lazily so that the generators can
be used on machines without a GPU.
"""
__all__ = ["inputs", "scf"]
