"""Plain FP64 CPU oracle for the SGLD + ULISSE hot path (Filippone & Engler, ICML 2015).

This package is test infrastructure. Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the GPU library never calls into it and
it imports nothing from the GPU package.

Everything here is deliberately slow and direct: dense covariance matrices, Cholesky
factorisations and the paper's algorithms taken step by step in double precision.

Modules
  gp          covariance function, its derivatives, log marginal likelihood, exact gradient
  cg          the Conjugate Gradient algorithm (Alg. 1)
  ulisse      randomly truncated CG series (Sec. 4) and its exact moments
  rng         Philox4x64-10 counter layout and the uniform / normal / sign mappings
  stoch_grad  the unbiased stochastic gradient (Sec. 2.1 and Sec. 4.1)
  sgld        the preconditioned SGLD update, step-size schedule, Langevin monitor, priors
  precond     Galerkin targets, MLP forward/backward and Adam for the learned preconditioner
  diagnostics PSRF, effective sample size, subset MAP and the SGLD preconditioner M

Parity status: every function listed above is pinned by a CPU test against a library
routine, a closed form, a published test vector or brute force; no function here is
"parity unpinned".
"""
from . import gp, cg, ulisse, rng, stoch_grad, sgld, precond, diagnostics  # noqa: F401
