"""MI355X-native coupled lattice-Boltzmann PEM-fuel-cell cathode solver.

The solver is the HIP library ``liblbmpem.so`` (C ABI: ``include/lbm_pem.h``);
``paper_2103_01444_amd.lbm`` is its thin Python binding.
"""
from .lbm import (LBM_BODY_FORCE, LBM_KINETICS_BUTLER_VOLMER, LBM_KINETICS_TAFEL, LBM_NO_REACTION, LBM_PERIODIC_X,
                  LBM_PERIODIC_Y, LBM_PERIODIC_Z, LBM_PRESSURE_INLET, LBM_THIN_CL, LBM_BUOYANCY, LBM_SIGMA_ENERGY,
                  LBM_PHYSICAL_HEAT, LBM_CELL_FIELDS, BatchedSweep, Cathode, Cathode3D, CurrentDensity,
                  LbmError, Params, default_params, grad_wrt_permeability, load_library, params_from_workload)

__all__ = ["BatchedSweep", "Cathode", "Cathode3D", "CurrentDensity", "LbmError", "Params", "default_params",
           "load_library", "params_from_workload", "LBM_PERIODIC_X", "LBM_PERIODIC_Y", "LBM_PERIODIC_Z",
           "LBM_PRESSURE_INLET", "LBM_THIN_CL", "LBM_BUOYANCY", "LBM_SIGMA_ENERGY",
           "LBM_PHYSICAL_HEAT", "LBM_CELL_FIELDS", "LBM_BODY_FORCE", "LBM_NO_REACTION", "LBM_KINETICS_TAFEL",
           "LBM_KINETICS_BUTLER_VOLMER", "grad_wrt_permeability"]
