"""Plain FP64 CPU oracle for the matrix-free DG residual, Jacobian-vector
product, element block-Jacobi preconditioner and flexible GMRES.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product library
never calls it and shares no code with it.

The oracle follows the paper's statement of the discretisation:

* broken polynomial spaces, hierarchical orthonormal modal basis (Sec. 2.1,
  2.4.1: restriction = keeping the low modes);
* residual f_h of eq. (NSdiscrRes): volume term with the BR2 corrected
  gradient, face term with the numerical flux against the jump of the test
  function;
* BR1/BR2 local and elemental lifting operators (Sec. 2.1, definition of the
  consistent gradient and eq. (vflux));
* Jacobian-vector product j_h = directional derivative of f_h (Sec. 2.2),
  evaluated here by complex-step differentiation (exact to round-off), and
  the finite-difference form of eqs. (matrix-free)/(epsdef) (Sec. 2.3);
* the global operator G = M/(gamma*dt) + J of eq. (rosSysOp) with M = I;
* element-wise block Jacobi = LU of the diagonal blocks (Sec. 2.3, EWBJ);
* flexible GMRES with right preconditioning (Sec. 2.5);
* the p-multigrid V-cycle with inherited coarse operators and GMRES[EWBJ]
  smoothers (Sec. 2.4, Alg. vcic, eq. GalProj) in ``oracle.pmg``.

Compressible Navier-Stokes fluxes (perfect gas, Stokes stress as in the
paper's viscous flux, Fourier heat flux, Lax-Friedrichs or Roe convective
flux) are textbook definitions.  The paper's own incompressible equations
(eq. ns, velocity and pressure, the mass form of eq. massBil) are in
IncompressibleNS, with a Lax-Friedrichs flux of the artificial
compressibility system standing in for the exact Riemann solver the paper
cites.
"""
from .quadrature import gauss_legendre, tensor_rule
from .basis import multi_indices, legendre_orthonormal, eval_basis, basis_size
from .physics import NavierStokes, Diffusion, IncompressibleNS
from .dg import DGOracle
from .solvers import fgmres, block_solve, backward_euler_dt

__all__ = [
    "gauss_legendre", "tensor_rule", "multi_indices", "legendre_orthonormal", "eval_basis",
    "basis_size", "NavierStokes", "Diffusion", "IncompressibleNS", "DGOracle", "fgmres", "block_solve",
    "backward_euler_dt",
]
