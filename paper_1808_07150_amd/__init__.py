"""MI355X-native SPDHG for Poisson PET with non-smooth priors (arXiv:1808.07150).

The computation lives in libspdhg.so (hand-written HIP kernels for gfx950, C ABI in
include/spdhg.h); this package is its thin Python binding.
"""
from .spdhg import (CGeom, CParams, EpochGraph, Reconstruction, SpdhgError,  # noqa: F401
                    aligned_workspace,
                    batch_epoch, cgeom, cparams, load_library, normalised_backprojection,
                    op_workspace, op_workspace_bytes, spdhg_backproject, spdhg_nnz,
                    spdhg_project, subset_bins)
