"""MI355X (gfx950) Nystrom-Schur solver: HIP kernels behind a C ABI plus a thin ctypes binding.

Two-level Nystrom-Schur preconditioner for sparse SPD systems in doubly
bordered block diagonal form (Al Daas, Rees & Scott, arXiv:2101.12164).
"""

from .nystrom_schur import (  # noqa: F401
    EXPORTED,
    KERNEL_FAMILIES,
    NS_APPLY_ADEF2,
    NS_APPLY_M2,
    NS_ERR_INVALID_ARG,
    NS_ERR_NOT_CONVERGED,
    NS_ERR_NOT_SPD,
    NS_FP32,
    NS_FP64,
    NS_SCHUR_AUTO,
    NS_SCHUR_LOCAL,
    NS_SCHUR_TRIANGULAR,
    NsError,
    NystromSchur,
    library_path,
    load_library,
    nystrom_schur_apply,
    nystrom_schur_destroy,
    nystrom_schur_export_factor,
    nystrom_schur_get_lowrank,
    nystrom_schur_get_sizes,
    nystrom_schur_interface_solve,
    nystrom_schur_interior_solve,
    nystrom_schur_kernel_stats,
    nystrom_schur_kernel_timing,
    nystrom_schur_last_error,
    nystrom_schur_pcg_solve,
    nystrom_schur_pcg_solve_batched,
    nystrom_schur_schur_apply,
    nystrom_schur_setup,
    nystrom_schur_setup_batched,
)
