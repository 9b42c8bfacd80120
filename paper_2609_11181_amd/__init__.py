"""MI355X-native spherical shear-based aperture-mass maps.

The compute path is the HIP library ``libsmartap.so`` (C ABI declared in
include/smartap.h), built for gfx950 by ``python -m paper_2609_11181_amd.build``.
This package holds the thin ctypes binding (:mod:`.lib`) and torch-tensor
wrappers (:mod:`.api`); PyTorch only supplies device memory and streams.
Importing :mod:`.api` without the built library raises immediately.
"""
__all__ = ["lib", "api"]
