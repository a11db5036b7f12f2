"""MI355X (gfx950) SA-AMG preconditioned CG Poisson solver for beam-pipe domains.

The numerical work lives in the HIP library ``libsaamg.so`` (sources in ``csrc/``,
C interface in ``include/saamg.h``); this package is its Python binding plus a
small serving loop built on the incremental-solve entry points.
"""
from . import capi  # noqa: F401
from .capi import (  # noqa: F401
    COARSE_DIRECT, COARSE_GS, FP64, MIXED, VARIANT_CONST, VARIANT_LIN, VARIANT_QUAD, HostDomain,
    SaamgError, TorchAllocator, batch_advance, batch_step, default_options, destroy, domain_for,
    domain_from_shape, footprint_bytes, hierarchy_info, level_apply, level_coefficients,
    operator_apply, pic_create, pic_deposit, pic_destroy, pic_gather, precond_apply, refresh,
    set_operator,
    coarse_inverse, scaling, setup, solve, solve_noalloc, state_create, state_destroy,
    state_finish, state_query,
)
