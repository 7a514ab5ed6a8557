"""Plain data containers describing one data-assimilation window.

Conventions shared by every consumer of these inputs:

* sites n = 0..M; the path X has shape (M+1, D) with the state order
  (V, m, h, n) for the Hodgkin-Huxley model (Section 5.1 of the paper);
* y has shape (M+1,): y[0] is unused because observations start at n = 1
  (the observation sum of the action runs over n = 1..M, Section 2.1);
* I has shape (M+1,): the drive sampled at t_n = n * dt;
* the seven HH parameters are p = (p1..p7) of the voltage equation
  (dV/dt equation, Section 5.1); gating constants come from Table 1 and are
  stored in the order (m, h, n).
"""

from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

# Table 2 "Actual" column: the parameter values used to make the data.
P_STAR: Tuple[float, ...] = (1.0, 120.0, 115.0, 20.0, -12.0, 0.3, 10.6)

# Table 1, re-ordered as (m, h, n); each entry is (V_a, dV_a, tau_a0, tau_a1)
# in mV and ms.
GATES_MHN: Tuple[Tuple[float, float, float, float], ...] = (
    (25.0, 15.0, 0.1, 0.4),    # m, Na activation
    (5.0, -15.0, 1.0, 7.0),    # h, Na inactivation
    (10.0, 30.0, 1.0, 5.0),    # n, K activation
)


@dataclass(frozen=True)
class ModelSpec:
    """Model, noise precisions and box prior of one window.

    kind      "hh" (D=4, seven parameters) or "lin1" (D=1 linear-Gaussian
              test model dx/dt = -p1 x + I(t), one parameter).
    dt        time step in ms.
    Ro        observation precision (scalar; L=1, the observed component is V).
    Rd        diagonal model-error precision, one entry per state component.
    beta      multiplier of the dynamical term of the action (annealing
              factor of Section 4.2; 1 means the target posterior).
    gates     Table 1 constants as ((V_a, dV_a, tau0, tau1) for m, h, n).
    x_lo/x_hi state box, applied at every site (uniform prior, Section 2.1).
    p_lo/p_hi parameter box.
    p_mask    bit l set means parameter l+1 is sampled.
    proposal  "gauss" (default) or "uniform" (Fig. 1 step 1a).
    k_lo/k_hi box of the twelve Table 1 constants, flattened in the order
              (m, h, n) x (V_a, dV_a, tau0, tau1).
    k_mask    bit 4 g + c set means constant c of gate g is sampled.
    """

    kind: str = "hh"
    dt: float = 0.02
    Ro: float = 1.0
    Rd: Tuple[float, ...] = (100.0, 1e6, 1e6, 1e6)
    beta: float = 1.0
    gates: Tuple[Tuple[float, float, float, float], ...] = GATES_MHN
    x_lo: Tuple[float, ...] = (-100.0, 0.0, 0.0, 0.0)
    x_hi: Tuple[float, ...] = (200.0, 1.0, 1.0, 1.0)
    p_lo: Tuple[float, ...] = tuple(sorted((0.5 * v, 1.5 * v))[0] for v in P_STAR)
    p_hi: Tuple[float, ...] = tuple(sorted((0.5 * v, 1.5 * v))[1] for v in P_STAR)
    p_mask: int = 0x7F
    proposal: str = "gauss"
    k_lo: Tuple[float, ...] = tuple(sorted((0.5 * v, 1.5 * v))[0] for g in GATES_MHN for v in g)
    k_hi: Tuple[float, ...] = tuple(sorted((0.5 * v, 1.5 * v))[1] for g in GATES_MHN for v in g)
    k_mask: int = 0

    @property
    def D(self) -> int:
        return 4 if self.kind == "hh" else 1

    @property
    def Np(self) -> int:
        return 7 if self.kind == "hh" else 1

    def with_(self, **kw) -> "ModelSpec":
        return replace(self, **kw)


def default_model(**kw) -> ModelSpec:
    return ModelSpec(**kw)


@dataclass
class Problem:
    """One window: model + data + initial state + proposal widths + seeds."""

    model: ModelSpec
    M: int
    y: np.ndarray            # (M+1,) float64, y[0] unused
    I: np.ndarray            # (M+1,) float64
    X0: np.ndarray           # (M+1, D) float64 initial path
    p0: np.ndarray           # (Np,) float64 initial parameters
    w_state: np.ndarray      # (D,) proposal widths of the state components
    w_param: np.ndarray      # (Np,) proposal widths of the parameters
    seed: int = 1
    chain: int = 0
    X_true: Optional[np.ndarray] = None
    p_true: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    def widths(self) -> np.ndarray:
        """Widths packed as [w_state(4) | w_param(7)] for the HH model."""
        return np.concatenate([self.w_state, self.w_param]).astype(np.float64)
