"""FP64 CPU oracle of SPDHG for Poisson PET with non-smooth priors.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU-baseline leg
of the benchmark, never by the HIP library or its Python binding.  It shares no code
with the library: the projector is plain C (projector.c, built with gcc), everything
else is NumPy in float64.

Modules:
  projector  ray-driven Joseph projector G and its ray-driven scatter adjoint
  prox       Poisson distance, its conjugate, KL-dual prox, l2-ball / box projections
  priors     grad, its adjoint, dTV operator D grad, TGV symmetrised gradient, norms
  sampling   SplitMix64 block draws, uniform and balanced probabilities
  spdhg      problem setup, step sizes (Theorem 2), SPDHG (Alg. 2), PDHG (Alg. 1),
             objective, duality gap, KKT residual, MLEM step, metrics

Pins: the paper prints no reconstructed image, objective or iteration count to compare
against (its figures are not in the text and its data are clinical), so the functions
the parity tests rest on are pinned by closed forms, invariants and brute force in
tests/test_oracle_*; the reporting metrics (relative_objective, psnr_paper) are plain
formulas with no pin of their own.
"""
from . import priors, projector, prox, sampling, spdhg  # noqa: F401
