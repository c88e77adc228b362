"""FP64 CPU oracle for polyline-array near-field imaging (arXiv 2109.02842).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path (the
HIP library and its Python binding) never does, and shares no code with it.

Everything here is plain numpy in float64/complex128 and follows the paper's
equations directly, with no blocking, fusion or reordering beyond what the
equations state:

  geometry  -- the polyline array, scan grid and frequency grid (Sec. II-A/B,
               Table 1).
  simulate  -- the point-scatterer echo model, eqs. (1) and (10)-(11).
  hybrid    -- the exact discrete form of the hybrid time-domain /
               spatial-frequency inversion, eqs. (2)-(9) and (12)-(19).
  bp        -- brute-force back-projection, the paper's comparison method.
  nudft     -- the direct nonuniform DFT that the NUFFT of eq. (8a)
               approximates, for step-level checks.
  omegak    -- the variant without NUFFT: the range transform by resampling
               onto a uniform wavenumber grid and an inverse FFT.

Every function is pinned by tests under ``tests/`` against facts that do not
come from the oracle itself (closed forms, symmetries, brute force, focusing
at known target positions, the paper's resolution formulas).
"""
from . import geometry, simulate, hybrid, bp, nudft, omegak  # noqa: F401
