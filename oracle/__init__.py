"""CPU FP64 oracle for one implicit radiation / ionization / gas-energy step.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, NumPy (FP64)
statement of what the method computes.  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path
(the HIP library and its Python binding) never does.  It shares no code with
the HIP path: the only common module is `synth`, which holds seeded inputs and
none of the method's arithmetic.

Paper: D. R. Reynolds, J. C. Hayes, P. Paschos, M. L. Norman, "Self-Consistent
Solution of Cosmological Radiation-Hydrodynamics and Chemical Ionization".

Module map
  model     parameters, physical constants, spectrum constants (Sec. 2.2, 3.2.5)
  physics   temperature, rates, local operators L_e, L_n, L_E (Sec. 2.1, Eqs. 26-28)
  fld       flux limiter and the diffusion operator D_E (Eq. 12, Eq. 25)
  residual  theta-scheme time level g^n and residual f(U), RMS norm (Eqs. 22-30)
  jacobian  local blocks by complex-step differentiation, Schur pieces,
            dense Jacobian for brute force (Eqs. 31-35)
  mg        geometric multigrid V-cycle and preconditioned CG (Sec. 3.2.1)
  newton    globalised inexact Newton step (Sec. 3.2), algorithm and
            definition (direct linear solve) modes

Parity status: every function is pinned by CPU tests (heat kernel, Stromgren
radius, single-cell equilibrium, dense-LU brute force, invariants) except the
rate coefficients' temperature dependence away from 1e4 K, the helium
chemistry constants and the cosmological a-factors, which the paper does not
print: those are "parity unpinned" (checked only for internal consistency).
"""
from .model import Model, model_from_workload  # noqa: F401
