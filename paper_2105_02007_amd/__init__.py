"""MI355X-native batched space-time solves of the parametric monodomain equation.

The HIP library ``libmlq.so`` (C ABI in ``include/mlq.h``) holds every step of
the path; ``paper_2105_02007_amd.mlq`` is its ctypes binding.  The package is
imported lazily so that ``build`` works before the library exists.
"""
__all__ = ["mlq", "build"]
