"""Plain, slow, FP64 CPU oracle for disk-integrated spectrum synthesis.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this package: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use it, to check and to time the HIP library against an
independent implementation.  It shares no code with the HIP library; both sides
read the same seeded inputs from ``workloads``.

Modules, each citing the passage of Zhao & Dumusque (2023), "SOAP-GPU", that
it follows:

  disk      stellar disk grid, limb darkening, rotation velocity, mu bins,
            active-region membership and the InfoMap owner rule
            (section 2.1, Fig. 1 caption; section 3.3)
  spectrum  relativistic Doppler factor (Eq. 6), bracketing index and linear
            interpolation (Eqs. 9-11), per-cell integration (Algorithms 1
            and 5), the three effects and the final spectrum (Eqs. 1-4),
            wavelength-dependent Planck contrast (section 4.3.1)
  ccf       cross-correlation with a line mask (section 4.1)
  fit       Gaussian fit of the CCF, RV = fitted mean (section 4.1)

Every function is pinned by the CPU tests against something other than
itself: closed forms, brute force on tiny grids, invariants, and the numbers
the paper prints.
"""
from . import disk, spectrum, ccf, fit  # noqa: F401
