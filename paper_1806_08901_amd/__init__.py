"""MI355X-native sampling-based SZ-vs-ZFP rate-distortion selector.

The estimator of arXiv:1806.08901 (Algorithm 1) runs in hand-written HIP
kernels for gfx950 behind the C ABI declared in ``include/szsel.h``; the
``szsel`` submodule is the thin ctypes binding, ``synth`` makes seeded
synthetic fields.  Importing the package loads nothing; the HIP library is
loaded on first use and its absence is an error, never a fallback.
"""
__all__ = ["szsel", "synth"]
