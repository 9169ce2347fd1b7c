"""MI355X-native 3-D Laplace fast multipole method.

The computation lives in the HIP library built from ``csrc/`` (C ABI in
``include/fmm.h``); ``binding`` is its ctypes front end.  Importing this package
does not load the library: the first plan does, and raises if it is missing.
"""
__all__ = ["FMM", "FMMFunction", "fmm_apply", "FMMTargets", "FMMTargetsFunction", "fmm_apply_targets", "FMMError",
           "load_library"]


def __getattr__(name):
    if name in __all__:
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
