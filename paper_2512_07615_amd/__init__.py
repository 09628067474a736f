"""MI355X (gfx950) matrix-product-state lattice Boltzmann library.

The compute path is the HIP shared library built from csrc/ (C ABI in
include/mps_lbm.h); `mps_lbm` is its ctypes binding.
"""
from .mps_lbm import (  # noqa: F401
    Config, Obs, Simulation, config_from_case, load, mps_lbm_default_config,
    mps_lbm_destroy, mps_lbm_init_from_field, mps_lbm_observables, mps_lbm_step,
    mps_lbm_to_dense,
)
