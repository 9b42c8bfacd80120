"""FP64 CPU oracle for the spherical shear-based aperture mass.

TEST INFRASTRUCTURE ONLY. Nothing in the product library imports, links or
calls this package; only the test suite, the smoke check and the CPU
baseline leg of the benchmark do. It is a plain, slow, obviously correct
restatement of the method in numpy FP64, sharing no code with the HIP path.

Modules
-------
healpix_ref  HEALPix RING geometry (Gorski et al. 2005), the paper's pixel
             scheme (Sect. 3): pixel centres, point -> pixel, ring tables,
             brute-force disc membership.
filters      the two aperture filters q(x) of the workloads, in FP64.
aperture     the aperture sums and maps: galaxy brute-force variant
             (Sect. 3.1), pixel-based variant (Sect. 3.2), summed
             normalisation (Sect. 2.4), noise (Eq. map_noise), shape-noise
             realisations.
binning      catalogue partition by pixel with offset table (Sect. 3.4) and
             per-pixel shear sums (Sect. 3.2, step 2).

Pins: every function is checked in tests/test_oracle_*.py against values
fixed by something other than itself (mpmath brute force, closed-form SIS
aperture masses, symmetry identities, HEALPix invariants). See each module's
header for its pins.
"""
from . import aperture, binning, filters, healpix_ref  # noqa: F401
