"""MI355X-native multilayer thin-film shallow-water lattice Boltzmann solver.

The solver lives in ``libmlfilm.so`` (HIP kernels for gfx950 behind the C ABI
declared in ``include/mlfilm.h``); :mod:`paper_2409_16659_amd.mlfilm` is the
thin ctypes binding and :mod:`paper_2409_16659_amd.inputs` draws seeded
synthetic films.  Importing the package loads nothing native.
"""
__all__ = ["inputs", "mlfilm"]
