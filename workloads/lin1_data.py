"""Linear-Gaussian D=1 test window ("LIN1").

Model dx/dt = -p1 x + I(t), x observed with Gaussian noise.  With the
trapezoid model error of Section 2.1 the whole path posterior is Gaussian, so
its mean and variance have a closed form (the Kalman smoother, Section 1);
that makes this window a statistical check of a sampler.

Data are drawn from the generative model the action encodes: x_0 from a wide
Gaussian, then eps_n ~ N(0, 1/Rd) solved for x_n through the trapezoid
relation, and y_n = x_n + N(0, 1/Ro).
"""

from __future__ import annotations

import numpy as np

from .problem import ModelSpec, Problem


def make_lin1_problem(M: int = 16, dt: float = 0.1, lam: float = 0.5, Rd: float = 100.0,
                      Ro: float = 4.0, data_seed: int = 7, w: float = 0.2,
                      sampler_seed: int = 3, chain: int = 0) -> Problem:
    rng = np.random.default_rng(data_seed)
    t = np.arange(M + 1) * dt
    I = np.sin(t) + 0.3 * rng.standard_normal(M + 1)
    a = 1.0 + lam * dt / 2.0
    b = 1.0 - lam * dt / 2.0
    x = np.empty(M + 1)
    x[0] = 1.0 + rng.standard_normal()
    for n in range(1, M + 1):
        k = 0.5 * dt * (I[n] + I[n - 1])
        x[n] = (b * x[n - 1] + k + rng.standard_normal() / np.sqrt(Rd)) / a
    y = np.zeros(M + 1)
    y[1:] = x[1:] + rng.standard_normal(M) / np.sqrt(Ro)
    big = 1e300
    model = ModelSpec(kind="lin1", dt=dt, Ro=Ro, Rd=(Rd,), beta=1.0, gates=(),
                      x_lo=(-big,), x_hi=(big,), p_lo=(0.0,), p_hi=(10.0,),
                      p_mask=0, proposal="gauss")
    X0 = np.zeros((M + 1, 1))
    X0[1:, 0] = y[1:]
    X0[0, 0] = y[1]
    return Problem(model=model, M=M, y=y, I=I, X0=X0, p0=np.array([lam]),
                   w_state=np.array([w]), w_param=np.array([0.0]),
                   seed=sampler_seed, chain=chain, X_true=x[:, None],
                   p_true=np.array([lam]), meta={"lam": lam})
