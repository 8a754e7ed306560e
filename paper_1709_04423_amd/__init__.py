"""MI355X-native split-step Crank-Nicolson (SSCN) Gross-Pitaevskii solver.

The numerics run in hand-written HIP kernels for gfx950 behind a C-ABI library
(``libgp.so``, declared in ``include/gp.h``); ``binding`` is a thin ctypes layer
over it.  Submodules are imported on demand so that input generation works on a
machine without a GPU.
"""
__all__ = ["binding", "inputs", "adjoint", "workflow"]
