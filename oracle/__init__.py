"""Plain FP64 CPU oracle of the path-integral Monte Carlo sampler.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
link anything in this package: only the test suite, the smoke check of the
package entry point and the CPU-baseline leg of the benchmark use it.  It
shares no code with the HIP library (no kernels, headers, helpers, tables or
constant generators); the only common code is the seeded input generator in
`workloads`, which holds none of the sampler's arithmetic.

Every function cites the passage of Quinn & Abarbanel, "Data Assimilation
using a GPU Accelerated Path Integral Monte Carlo Approach" (arXiv:1103.4887)
that it follows.  Where the paper is silent the reading taken is stated in
the function's docstring.

Modules
  philox   Philox4x32-10 counter-based generator (Salmon et al., SC'11), the
           sampler's random-number contract and the uniform/normal mappings
  models   HH vector field F, Jacobian J and dF/dp (Section 5.1, Table 1);
           the D=1 linear test model
  action   model error eps_n, action A = A_o + beta*A_d (Section 2.1), the
           local change of A under one site move, the analytic gradient
  sampler  red-black Metropolis sweep + sequential parameter moves
           (Fig. 1, Sections 4.1-4.2), statistics
  hmc      leapfrog / Hybrid Monte Carlo proposal on the same action
  kalman   closed-form posterior of the D=1 linear-Gaussian window
  mp       50-digit mpmath evaluation of A for tiny windows (a pin)

Parity status: every function here is pinned by a test in tests/test_oracle_*.
The HH posterior itself has no closed form: beyond the pins of its parts
(local dA = brute-force dA, detailed balance on a lattice, the linear-Gaussian
closed form, gradient = finite differences) it is parity unpinned.
"""
