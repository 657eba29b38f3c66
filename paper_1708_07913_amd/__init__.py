"""MI355X-native spectral-quadrature (SQ) density/energy step of SQDFT.

The compute path is ``libsq.so`` (hand-written HIP kernels for gfx950 behind
the C ABI declared in ``include/sq.h``); :mod:`paper_1708_07913_amd.sq` is the
thin Python binding over it, and :mod:`paper_1708_07913_amd.workloads` builds
seeded synthetic inputs.  Importing the package loads nothing: the binding
loads the library on first use and raises if it is missing.
"""

__all__ = ["sq", "workloads"]
