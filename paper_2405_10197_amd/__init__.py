"""MI355X-native string-based CASCI: sigma = H.C and Davidson-Liu on HIP.

The compute path lives in ``libcasci.so`` (hand-written HIP for gfx950,
C ABI declared in ``include/casci.h``); :mod:`.casci` is the thin ctypes
binding over it. Importing this package does not load the library; the
first call into :mod:`.casci` does, and raises if it is not built.
"""
__all__ = ["casci", "synth"]
