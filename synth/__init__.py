"""Seeded synthetic inputs shared by the oracle and the HIP library.

This module holds no discretisation arithmetic: no quadrature, no basis, no
flux, no projection.  It only builds

* periodic structured lattices of quadrilaterals / hexahedra (vertex
  coordinates per element, face-neighbour table, optional seeded vertex
  perturbation that moves periodic images together),
* analytic initial fields, given as plain numpy functions of physical
  coordinates returning conserved variables (rho, rho*u_1..d, rho*E), or
  velocity and pressure (u_1..u_d, p) for the incompressible equations,
* seeded random vectors (element-fastest flat layout),
* the named workload presets (cfg1..cfg5) with their physical constants,
* seeded initial weights of the learned preconditioner's network.

Each consumer (the oracle and the product library) projects the analytic
fields onto its own basis with its own quadrature.
"""
from .lattice import lattice_mesh, mesh_neighbors
from .fields import (FreeStreamPlusModes, TaylorGreenStandIn, UniformState,
                     TrigSum, primitive_to_conserved, IncompressibleStandIn)
from .presets import PRESETS, preset, random_vector
from .mlp_init import mlp_init_weights

__all__ = [
    "lattice_mesh", "mesh_neighbors", "FreeStreamPlusModes", "TaylorGreenStandIn",
    "UniformState", "TrigSum", "primitive_to_conserved", "IncompressibleStandIn", "PRESETS", "preset",
    "random_vector", "mlp_init_weights",
]
