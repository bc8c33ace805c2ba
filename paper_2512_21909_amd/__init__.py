"""MI355X-native particle-particle ladder of Cholesky-decomposed CCSD
(T2 and Lambda residual terms, Abelian point-group symmetry), the vvvv
two-body-density contraction with Cholesky vectors, and the O(O^3 V^3)
contraction of the partial symmetric-antisymmetric scheme, and the
symmetry-adapted two-step Cholesky decomposition.

The computation lives in ``libcdcc.so`` (HIP, gfx950) behind the C ABI of
``include/cdcc.h``; this package only marshals arguments.
"""
from ._lib import CdccError, LIB_PATH  # noqa: F401
from .layout import Layout  # noqa: F401
from .ladder import (cd_basis, cd_vectors, ladder_lambda, ladder_t2, ladder_t2_noalloc, lambda_dress,  # noqa: F401
                     partial_contract, release, require_gpu, timing_enable, timing_read, vvvv_density,
                     workspace_bytes)
