"""libpimc for AMD MI355X: path-integral Monte Carlo data assimilation.

Red-black Metropolis sweeps over the whole state history of a
Hodgkin-Huxley neuron plus its parameters, after Quinn & Abarbanel,
"Data Assimilation using a GPU Accelerated Path Integral Monte Carlo
Approach" (arXiv:1103.4887).  The compute path is the HIP library
libpimc.so (C ABI in include/pimc.h); this package only binds it.
"""

from . import _lib
from .autograd import PimcAction, action
from .api import (Context, HmcStats, InitPhase, PackedBatch, SweepDebug, SweepStats, Window, model_struct, pimc_action,
                  pimc_action_noalloc, pimc_forecast, pimc_grad, pimc_hmc, pimc_model_errors, pimc_param_update,
                  pimc_run_batch, pimc_sweep, pimc_sweep_init, widths_tensor)

__all__ = ["PimcAction", "action", "Context", "HmcStats", "InitPhase", "pimc_sweep_init", "pimc_hmc", "pimc_action_noalloc",
           "pimc_forecast", "pimc_model_errors", "PackedBatch", "SweepDebug", "SweepStats", "Window", "model_struct", "pimc_action",
           "pimc_grad", "pimc_param_update", "pimc_run_batch", "pimc_sweep", "widths_tensor", "_lib"]
