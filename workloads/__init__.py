"""Seeded synthetic inputs for the path-integral Monte Carlo sampler.

This package only *produces inputs*: a model description (constants, noise
precisions, boxes), a drive current I_n, noisy voltage observations y_n, an
initial path X and initial parameters p.  It holds none of the sampler's
arithmetic (no action, no acceptance test, no random stream of the sampler);
both the CPU oracle and the HIP library consume what it returns.

The twin experiment follows the paper's example (Section 5.1): a
Hodgkin-Huxley neuron is integrated at known parameters, only V is observed
with additive Gaussian noise, and every state plus the parameters are then
estimated.  The paper's own drive was a Lorenz-generated current whose scale it
does not state, so a step + sine + Ornstein-Uhlenbeck current of a stated scale
stands in for it.
"""

from .problem import Problem, ModelSpec, P_STAR, GATES_MHN, default_model
from .hh_data import make_hh_problem, hh_stimulus, hh_truth
from .lin1_data import make_lin1_problem
from .configs import CONFIGS, MASK_ALL, MASK_C1, batch_sizes, batch_true_params, config_batch, config_problem

__all__ = [
    "Problem", "ModelSpec", "P_STAR", "GATES_MHN", "default_model",
    "make_hh_problem", "hh_stimulus", "hh_truth", "make_lin1_problem",
    "CONFIGS", "MASK_ALL", "MASK_C1", "batch_sizes", "batch_true_params", "config_batch", "config_problem",
]
