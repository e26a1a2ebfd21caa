"""MI355X-native SPDHG for Poisson PET with non-smooth priors (arXiv:1808.07150).

The computation lives in libspdhg.so (hand-written HIP kernels for gfx950, C ABI in
include/spdhg.h); this package is its thin Python binding.
"""
from .spdhg import (CGeom, CParams, Reconstruction, SpdhgError, batch_epoch,  # noqa: F401
                    cgeom, cparams, load_library, spdhg_backproject, spdhg_nnz,
                    spdhg_project, subset_bins)
