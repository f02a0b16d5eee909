"""MI355X-native GLS map-making hot path (arXiv 1408.3048): A = P^T N^-1 P
inside preconditioned CG with block-Jacobi and two-level (A-DEF1) preconditioners.

The compute path is the HIP library ``libmm.so`` (C-ABI in ``include/mm.h``);
this package only binds it (``_lib``) and builds it (``build``)."""

from ._lib import (  # noqa: F401
    EXPORTED, MMError, Plan, gemm_tn_f64, lanczos_ritz, last_error, load,
    MM_OK, MM_ERR_ARG, MM_ERR_DEVICE, MM_ERR_RANK, MM_ERR_NOT_SPD, MM_ERR_BREAKDOWN,
    MM_ERR_NOCONV, MM_ERR_STATE,
)
