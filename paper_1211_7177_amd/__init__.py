"""MI355X-native fast-multipole Nystrom EFIE operator and BEM solver.

The compute path is libfmbem.so (hand-written HIP for gfx950, C ABI declared
in include/fmbem.h); this package is its thin Python binding.  Importing a
name below loads the library; a missing library raises ImportError.
"""

__all__ = ["Plan", "BemProblem", "FmbError", "load"]


def __getattr__(name):
    if name in ("Plan", "FmbError", "load"):
        from . import _abi
        return getattr(_abi, name)
    if name == "BemProblem":
        from . import solver
        return solver.BemProblem
    raise AttributeError(name)
