"""Named workload presets (sizes, physical constants, seeds).

cfg1  2D compressible NS, periodic unit square, 16x16 quads, Q2, 4x4 Gauss,
      free stream Mach 0.2 (c_inf = 1) + seeded sinusoids, Re = 100.
cfg2  3D compressible NS, periodic [0, 2pi]^3, 32^3 hexes, P3, 4^3 Gauss,
      Taylor-Green stand-in at Mach 0.1, Re = 1600.
cfg3  cfg2 field at P4 on 24^3 hexes (5^3 Gauss), backward Euler at CFL 100.
cfg4  cfg3 with every lattice vertex moved by seeded U(-0.1h, 0.1h).
cfg5  cfg2 discretisation, learned element preconditioner workload, backward
      Euler at CFL 30 (block-Jacobi FGMRES converges at every snapshot).
"""
import numpy as np

from .fields import FreeStreamPlusModes, TaylorGreenStandIn, IncompressibleStandIn
from .lattice import lattice_mesh

GAMMA = 1.4
PRANDTL = 0.72

PRESETS = {
    "cfg1": dict(dim=2, N=(16, 16), L=1.0, space="Q", order=2, nq1d=4, mu=0.2 / 100.0,
                 field="freestream_modes", field_seed=1809, v_seed=866, perturb=0.0, mesh_seed=None),
    "cfg2": dict(dim=3, N=(32, 32, 32), L=2 * np.pi, space="P", order=3, nq1d=4, mu=1.0 / 1600.0,
                 field="taylor_green", field_seed=1600, v_seed=866, perturb=0.0, mesh_seed=None),
    "cfg3": dict(dim=3, N=(24, 24, 24), L=2 * np.pi, space="P", order=4, nq1d=5, mu=1.0 / 1600.0,
                 field="taylor_green", field_seed=1600, v_seed=866, perturb=0.0, mesh_seed=None,
                 cfl=100.0, mg_orders=(4, 2, 1), mg_smooth=(8, 8, 40), restart=30, rtol=1e-8),
    "cfg4": dict(dim=3, N=(24, 24, 24), L=2 * np.pi, space="P", order=4, nq1d=5, mu=1.0 / 1600.0,
                 field="taylor_green", field_seed=1600, v_seed=866, perturb=0.1, mesh_seed=2403,
                 cfl=100.0, mg_orders=(4, 2, 1), mg_smooth=(8, 8, 40), restart=30, rtol=1e-8),
    "cfg5": dict(dim=3, N=(32, 32, 32), L=2 * np.pi, space="P", order=3, nq1d=4, mu=1.0 / 1600.0,
                 field="taylor_green", field_seed=1600, v_seed=866, perturb=0.0, mesh_seed=None,
                 cfl=30.0, restart=30, rtol=1e-8),
}


def preset(name, N=None, order=None, nq1d=None):
    """Return (config dict, mesh dict, field callable) for a named preset.

    N / order / nq1d override the preset's lattice size and polynomial degree
    (used for small parity cases with the same physics and field).
    """
    cfg = dict(PRESETS[name])
    cfg["name"] = name
    cfg["gamma"] = GAMMA
    cfg["prandtl"] = PRANDTL
    if N is not None:
        cfg["N"] = tuple(N) if not np.isscalar(N) else (int(N),) * cfg["dim"]
    if order is not None:
        cfg["order"] = int(order)
        if nq1d is None:
            nq1d = int(order) + 1 if cfg["dim"] == 3 else max(int(order) + 2, 2)
    if nq1d is not None:
        cfg["nq1d"] = int(nq1d)
    mesh = lattice_mesh(cfg["N"], L=cfg["L"], perturb=cfg["perturb"], seed=cfg["mesh_seed"])
    if cfg["field"] == "freestream_modes":
        field = FreeStreamPlusModes(seed=cfg["field_seed"], gamma=GAMMA)
    else:
        field = TaylorGreenStandIn(seed=cfg["field_seed"], gamma=GAMMA, L=float(np.max(cfg["L"])))
    return cfg, mesh, field


def random_vector(n, seed=866):
    """Seeded N(0,1) vector of length n (layout-agnostic: entries are i.i.d.)."""
    return np.random.default_rng(seed).standard_normal(n)
