"""FP64 CPU oracle for the Defrise-Clack shift-variant FBP path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 NumPy
statement of what the reconstruction computes, written from the paper
(Ye et al., "DRACO: Differentiable Reconstruction for Arbitrary CBCT Orbits",
Sec. 2, eqs. 5-12) and used only by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The GPU library never imports it and it
never imports the GPU library; the two share only the seeded input generators
in ``synth``.

Modules
  pipeline  -- every stage of eq. 12 and its exact transpose
  siddon    -- Siddon ray-driven projector (data generation / cross-checks)
  fdk       -- textbook Feldkamp (FDK) reconstruction for circular orbits
  crofton   -- the smooth Crofton redundancy weight M of eq. 9
  smooth    -- the Gaussian smoothing layer of the learned weight (Sec. 3.1) and its transpose
  ssim      -- the 3D structural similarity of eq. 13's loss and its gradient
  noise     -- Poisson noise on projections (Sec. 3.3) from the counter-based Philox4x64-10 generator
  adam      -- the Adam / AdamW update of the learned weight (Sec. 3.1)

Every function here is pinned by a test against something other than itself
(closed forms, invariants, the FDK equivalence on a circle, exact ball
reconstruction, brute force); see the docstrings for what pins each one.
"""
from . import pipeline, siddon, fdk, crofton  # noqa: F401
