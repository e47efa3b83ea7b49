"""MI355X-native per-Runge-Kutta-substage residual of the explicit
compressible Navier-Stokes method of OpenSBLI (arXiv 2007.14933).

The compute path is the HIP library ``libosbli.so`` behind the C ABI declared
in ``include/osbli.h``; :mod:`.binding` marshals arguments to it and
:mod:`.solver` drives it with device buffers owned by PyTorch.
"""
__all__ = ["inputs"]
