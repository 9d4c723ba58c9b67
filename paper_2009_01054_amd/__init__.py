"""MI355X (gfx950) generalized vec trick for pairwise kernel learning.

Thin Python binding over the C ABI in ``include/gvt.h`` (``libgvt.so``, built
in-tree by ``paper_2009_01054_amd.build``).  The functions keep the C names
and only marshal arguments: torch tensors provide device memory and the
current HIP stream; every step of the computation runs in the library's HIP
kernels.  There is no fallback: if the library is missing or the device is
not available, calls raise.
"""
from __future__ import annotations

from ._binding import (  # noqa: F401
    BF16X3,
    BF16X6,
    F32,
    F64,
    FLAG_DENSE_TILES,
    FLAG_NO_DENSE_TILES,
    FLAG_ORDER_A,
    FLAG_ORDER_B,
    FLAG_SYMMETRIC_BASES,
    KINDS,
    GvtError,
    Plan,
    gvt_base_kernel,
    gvt_dense_matvec,
    gvt_dense_matvec_checked,
    gvt_dense_matvec_noalloc,
    gvt_empty_cache,
    gvt_erm_newton,
    gvt_erm_objective,
    gvt_krr_cg,
    gvt_krr_cg_batched,
    gvt_krr_minres,
    gvt_last_error,
    gvt_matvec,
    gvt_pairwise_matvec,
    gvt_tanimoto_kernel,
    gvt_plan_create,
    gvt_plan_destroy,
    gvt_plan_execute,
    gvt_plan_info,
    gvt_plan_profile,
    gvt_plan_uses_tiles,
    gvt_version,
    library_path,
    load_library,
)
