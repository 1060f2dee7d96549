"""MI355X-native fitter of 2D Gaussians to video frames.

The computation lives in the HIP library ``libgs2d.so`` (C ABI in
``include/gs2d.h``); ``_lib`` is its ctypes binding.  ``synth`` generates
seeded synthetic inputs.  Importing the package loads nothing; the library is
loaded on the first call into ``_lib``.
"""
__all__ = ["_lib", "synth"]
