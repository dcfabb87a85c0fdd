"""MI355X (gfx950) implementation of the voxel-parallel second-order fit of
model-based multi-parameter mapping (Balbastre et al., arXiv 2102.01604).

The compute path is the HIP library ``libmpm.so`` (C ABI in ``include/mpm.h``);
``_lib`` is its thin ctypes binding and ``synth`` draws seeded synthetic inputs.
Importing the package does not load the library.
"""
from ._lib import (MpmError, mpm_fit, mpm_footprint_bytes, mpm_profile_enable, mpm_profile_read,  # noqa: F401
                   mpm_profile_reset, mpm_simulate, mpm_uncertainty, mpm_version)

__all__ = ["MpmError", "mpm_fit", "mpm_uncertainty", "mpm_simulate", "mpm_footprint_bytes", "mpm_version",
           "mpm_profile_enable", "mpm_profile_reset", "mpm_profile_read"]
