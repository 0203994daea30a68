"""Plain FP64 CPU oracle of the SMC-MPC hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls, links
or runs this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the HIP path; both are fed from
the seeded input generators in ``synth``.

Modules:
  philox   -- Philox4x32-10 counter-based generator, uniform and normal draws
  wind     -- grid, Kronecker Cholesky factor, field samples, trilinear lookup
  rollout  -- dynamics, constraints, landing, cost terms, pairwise separation
  smc      -- Alg. 1: initialisation, weights, resampling, moves, selection
  grad     -- FP64 autograd transcription of the fuel + time cost (Langevin move)
  mpc      -- receding-horizon loop: plant step, rolling window

Each function cites the passage of the paper it follows.  Functions without an
independent pin say "parity unpinned" in their docstring.
"""
from . import philox, wind, rollout, smc, mpc  # noqa: F401
