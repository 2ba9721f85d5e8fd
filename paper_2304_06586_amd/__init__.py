"""MI355X-native generalized FDTD for electromagnetic scattering in moving
structures (Deck-Leger, Bahrami, Li, Caloz, arXiv 2304.06586).

The hot path -- leapfrog stepping of the generalized Yee cell with the
moving-boundary sampling, source, absorbing ends and probes -- runs in HIP
kernels for gfx950 behind the C-ABI of include/gfdtd.h (libgfdtd.so, built
in-tree), and the same scheme in 2D (TE / TM, a stratified moving
modulation) behind include/gfdtd2d.h.  This package is its thin Python
binding.
"""
from .gfdtd import (  # noqa: F401
    Batch, GfdtdError, Run2D, Server, gfdtd2d_check, gfdtd2d_solve,
    gfdtd2d_workspace_bytes, gfdtd_batch_workspace_bytes, gfdtd_check,
    gfdtd_result_sizes, gfdtd_solve, gfdtd_solve_batch, gfdtd_solve_static,
    gfdtd_status_str,
    gfdtd_tmm, gfdtd_tmm_kernel_ms, gfdtd_workspace_bytes, load_library,
)
