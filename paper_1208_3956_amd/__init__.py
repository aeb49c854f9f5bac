"""MI355X-native PML-transmission double-sweep Helmholtz solver (HIP, gfx950).

The compute path is the C ABI of libhelm.so (include/helm.h); `_lib` is its ctypes
binding with the same names and `solver.Helmholtz` a torch-facing wrapper.  Importing
this package does not load the library; the first call does, and fails loudly if it
has not been built (`python -m paper_1208_3956_amd.build`).
"""
__all__ = ["Helmholtz", "SolveResult", "solve_batch", "HelmMisfit", "misfit", "build"]


def __getattr__(name):
    if name in ("Helmholtz", "SolveResult", "solve_batch"):
        from . import solver
        return getattr(solver, name)
    if name in ("HelmMisfit", "misfit"):
        from . import autograd
        return getattr(autograd, name)
    if name == "build":
        from .build import build
        return build
    raise AttributeError(name)
