"""MI355X (gfx950) implementation of the APR compressible-SPH hot path.

A thin ctypes binding over libapr.so (see include/apr.h).  Every step of the
path runs in the library's HIP kernels; this module only marshals arguments
(torch tensors are used for device memory and the current stream).  There is
no CPU fallback: if libapr.so is missing, importing the binding fails.
"""
from ._abi import (  # noqa: F401
    APR_OK, APR_ERR_INVALID, APR_ERR_CAPACITY, APR_ERR_NOCONVERGE, APR_ERR_HIP,
    APR_ERR_OVERFLOW, APR_ERR_RANGE, APR_FP64, APR_FP32, APR_EOS_ISOTHERMAL, APR_EOS_LOCALLY_ISOTHERMAL,
    APR_EOS_ADIABATIC, APR_SPLIT_TANGENTIAL, APR_SPLIT_RANDOM, APR_KERNEL_M4, APR_KERNEL_WC2,
    APR_ZONE_SPHERE, APR_ZONE_CYLINDER,
    APR_PROF_DENSITY,
    APR_PROF_FORCES, APR_PROF_CELLS, APR_PROF_SPLITMERGE, APR_PROF_VJP, APR_PROF_CAND, AprError, lib, lib_path,
    Params, Zone, Sink, CState, apr_default_params)
from .api import (  # noqa: F401
    Context, DeviceState, apr_ctx_create, apr_ctx_destroy, apr_set_cell_grid, apr_build_cells,
    apr_density,
    apr_forces, apr_vjp, apr_relax, apr_bins_init, apr_step_bins, apr_neighbours, apr_split_merge, apr_step, apr_accel, apr_timestep, apr_timestep_noalloc,
    apr_sync_status, apr_profile_enable, apr_profile_select, apr_profile_read, apr_counters, make_params, make_zones,
    make_sinks)
from .autograd import apr_sums  # noqa: F401,E402
