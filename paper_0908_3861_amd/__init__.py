"""Constant-cost space-variant elliptical filtering with four-direction box splines on MI355X.

The compute path is the HIP library ``libbsf.so`` (hand-written gfx950 kernels behind a
C ABI, declared in ``include/bsf.h``); this package holds its thin ctypes binding, the
seeded input generators (``synth``) and the serving loop.  Importing the package does not
load the library; the first call of a filter entry point does, and fails loudly if the
library is missing.
"""
__all__ = ["filter", "filter_batched", "preintegrate", "Context"]


def __getattr__(name):
    if name in ("filter", "filter_batched", "preintegrate", "Context", "lib_path"):
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
