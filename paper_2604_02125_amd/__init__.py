"""MI355X-native compact Runge-Kutta flux reconstruction (cRKFR) with
entropy-conservative / kinetic-energy-preserving two-point volume fluxes.

The compute path is the HIP library ``libcrk.so`` (gfx950) behind the C ABI
declared in ``include/crk.h``; ``paper_2604_02125_amd.crk`` is a thin ctypes
binding with the same names.  Importing this package loads nothing; the
binding loads the library on first use and raises if it is missing.
"""
__all__ = ["crk", "inputs"]
