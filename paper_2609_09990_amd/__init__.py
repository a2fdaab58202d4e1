"""Thin Python binding of libdmrg_mi355x (the two-site DMRG sigma path on MI355X).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch (when used) provides device memory and the stream; it is
imported before the library so both share one HIP runtime.  There is no CPU
fallback: if the shared library is missing, importing this package raises.
"""
from ._lib import (  # noqa: F401
    DMRGError,
    LIB_PATH,
    MLP,
    Problem,
    Solver,
    dmrg_block_gemm,
    dmrg_block_gemm_noalloc,
    dmrg_measure_peaks,
    measure_peaks,
    dmrg_deflate_add,
    dmrg_deflate_clear,
    dmrg_deflate_project,
    dmrg_diag,
    dmrg_energy,
    dmrg_export_mps,
    dmrg_get_bonds,
    dmrg_get_env,
    dmrg_get_stats,
    dmrg_grad,
    dmrg_last_error,
    dmrg_mpo_dims,
    dmrg_mpo_site,
    dmrg_mpo_site_nnz,
    dmrg_options,
    dmrg_overlap,
    dmrg_s_squared,
    dmrg_options_default,
    dmrg_prepare,
    dmrg_problem_create,
    dmrg_problem_destroy,
    dmrg_set_mps,
    dmrg_sigma,
    dmrg_solver_create,
    dmrg_solver_destroy,
    dmrg_step,
    dmrg_sweep,
    dmrg_truncate,
    dmrg_workspace_attach,
    dmrg_workspace_query,
    dmrg_ci_dims,
    dmrg_ci_apply_v,
    dmrg_ci_rdm12,
    dmrg_ci_rdm3,
    dmrg_correction,
    dmrg_fiedler_order,
    dmrg_mps_orbital_rdm2,
    dmrg_mps_to_ci,
    dmrg_mutual_information,
    dmrg_orbital_rdm2,
    dmrg_rdm12,
    dmrg_stationarize,
    fiedler_order,
    lib,
    reorder_integrals,
)

from .autograd import DMRGEnergy, dmrg_energy  # noqa: F401,E402
from .excited import excited_states  # noqa: F401,E402

FP64, FP32, BF16 = 0, 1, 2
PRECOND_DIAG, PRECOND_LEARNED, PRECOND_OLSEN, PRECOND_SHIFT_INVERT = 0, 1, 2, 3
