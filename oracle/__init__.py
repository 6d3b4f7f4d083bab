"""Plain FP64 CPU oracle for the implicit photochemical column step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import or run anything in this
package; the HIP library never does, and it shares no code with it.

It computes, slowly and plainly, what the GPU path computes:

  thermo      NASA-7 G/RT and Cp/R (Appendix A)
  grid        number densities, half levels, heights, optical depth
              (Section 2.1, Eq. transportflux / discrete_continuity;
              Section 2.3.3 optical depth)
  rates       two-body (Kooij / modified Arrhenius), three-body
              (Lindemann), photolysis, reverse rates from Gibbs energies
              (Section 2.3.1-2.3.4)
  rhs         P - L - d(phi)/dz (Eq. continuity, Eq. transportflux)
  jacobian    analytic dF/dn, block-tridiagonal blocks
  linalg      dense LU solve and block Thomas with partial pivoting
  integrate   linearly implicit backward Euler (Section 2.1, integrator
              list), fixed schedule and adaptive steady-state driver
  equilibrium element-potential equilibrium (independent check)

Functions with no independent pin say "parity unpinned" in their docstring.
"""

from .constants import KB, AMU, P_STD
from . import thermo, grid, rates, rhs, jacobian, linalg, integrate, equilibrium

__all__ = ["KB", "AMU", "P_STD", "thermo", "grid", "rates", "rhs", "jacobian",
           "linalg", "integrate", "equilibrium"]
