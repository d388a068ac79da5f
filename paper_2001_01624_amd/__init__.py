"""MI355X-native multiscale restricted-smoothing (MsRSB) pressure solver.

The solver itself is the HIP library ``libmsrsb.so`` (C ABI in
``include/msrsb.h``); ``capi`` is its ctypes binding and ``serve`` the
continuous-batching request loop built on it.  Nothing here computes on the
CPU: a missing library raises at import of ``capi``.
"""

__all__ = ["capi", "build"]
