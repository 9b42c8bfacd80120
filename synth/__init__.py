"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module produces catalogues and pixel maps only. It holds none of the
aperture-mass arithmetic: it never selects apertures, evaluates a filter,
rotates shear into tangential components or normalises a map. Both the FP64
oracle and the GPU library consume the arrays it returns.
"""
from .generators import (  # noqa: F401
    ARCMIN,
    DEG,
    CatalogueSpec,
    PixelMapSpec,
    config1_catalogue,
    config2_catalogue,
    config3_pixelmap,
    config4_catalogue,
    config5_instances,
    galaxy_catalogue,
    noise_angles,
    pixel_level_map,
    small_catalogue,
)
