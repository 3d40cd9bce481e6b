"""MI355X (gfx950) SPH + octree hot path of FleCSPH (arXiv:2007.03097).

The compute path is libsph_gfx950.so (hand-written HIP kernels behind the C ABI declared in
include/sph.h).  ``api`` exposes the same entry points for torch tensors; PyTorch only
provides device memory and streams.
"""
from .api import (  # noqa: F401
    TUNING_CACHE,
    SPHError,
    Context,
    ParticleArrays,
    sph_config_default,
    sph_create,
    sph_destroy,
    sph_workspace_size,
    sph_set_workspace,
    sph_build_tree,
    sph_tree_nodes,
    sph_find_neighbors,
    sph_compute_density,
    sph_compute_forces,
    sph_compute_gravity,
    sph_step,
    sph_step_noalloc,
    sph_autotune,
    sph_get_tuning,
    sph_sync,
    sph_last_error,
    sph_peak_probe,
    sph_timestep,
    sph_key_order,
    sph_gravity_counts,
)
from ._abi import (SPH_CURVE_HILBERT, SPH_CURVE_MORTON, SPH_ENERGY_THERMAL, SPH_ENERGY_THERMOKINETIC, SPH_FP32C, SPH_FP64, SPH_STEP_PRIMED,  # noqa: F401
                   SPH_GRAVITY_FMM, SPH_GRAVITY_QUADRUPOLE, SPH_STEP_RESUME)
