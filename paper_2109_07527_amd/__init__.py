"""MI355X-native charge-regulation Monte Carlo (CR-MC).

The hot path (shifted-cell binning, checkerboard trial phases, pair sums,
Metropolis acceptance, Philox random numbers) runs in the HIP library
libcrmc.so behind the C ABI of include/crmc.h; ``crmc`` is its ctypes binding.
"""
from .crmc import (ACID, BASE, NEUTRAL, XNEG, XPOS, CrmcError, System, crmc_build_cells,  # noqa: F401
                   crmc_create, crmc_destroy, crmc_energy, crmc_enable_log, crmc_export_state, crmc_get_group_hist,
                   crmc_get_occupancy, crmc_get_particles, crmc_get_series, crmc_observe, crmc_philox,
                   crmc_import_state, crmc_pIX_from_salt, crmc_read_log, crmc_sweep, crmc_sweep_ex, load)
