"""MI355X-native finite-frequency traveltime tomography operators.

The hot path (the traveltime Jacobian J and its adjoint, the regularised
solvers and point-spread functions built on them) lives in the HIP library
``libfftt.so``; ``fftt`` is its thin ctypes binding.  Importing this package
does not load the library: ``paper_1908_03302_amd.fftt`` does, and raises if
the built library is missing.
"""
__all__ = ["inputs"]
