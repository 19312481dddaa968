"""GPU parity of the incompressible equations (Sec. 2.1, eq. ns: unknowns
(u, p), divergence constraint, mass form of eq. massBil on the velocities
only) against the FP64 oracle, through the C ABI.

Tolerances as for the compressible operator: residual 1e-12 of
max(|R|, |R_volume|), exact Jv 1e-12 (with the shift on the velocities only),
FD Jv 1e-6, block apply 1e-11, V-cycle 1e-9, a Rosenbrock step 1e-10 of its
increment; solves re-checked on the true residual with the oracle operator.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import DGOracle, IncompressibleNS, block_solve
from oracle import rosenbrock as ros
from oracle.pmg import PMultigrid

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NU = 1e-2


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_case(N, k, nq, seed=5):
    from paper_1809_00866_amd import DG
    mesh = synth.lattice_mesh(N, L=1.0)
    d = len(N)
    o = DGOracle(mesh, k, "P", nq, IncompressibleNS(d, nu=NU))
    U = o.project(synth.IncompressibleStandIn(d, seed=seed))
    U = U + 1e-2 * np.random.default_rng(seed).standard_normal(U.shape)
    g = DG(mesh, k, nq1d=nq, mu=NU, physics="incompressible")
    w = torch.tensor(o.to_flat(U), device="cuda")
    return o, g, U, w


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300)


CASES = [((4, 3), 2, 4), ((5, 2), 3, 5), ((2, 3, 2), 1, 2), ((3, 2, 2), 2, 3), ((2, 2, 3), 3, 4)]
IDS = [f"{len(c[0])}d-N{'x'.join(map(str, c[0]))}-P{c[1]}" for c in CASES]


@pytest.mark.parametrize("N,k,nq", CASES, ids=IDS)
def test_residual_and_jvp_parity(N, k, nq):
    _say(f"incompressible residual/jvp {N} P{k}")
    o, g, U, w = make_case(N, k, nq)
    assert g.nv == len(N) + 1
    R, Rv = o.residual(U, return_parts=True)
    err = np.linalg.norm(g.residual(w).cpu().numpy() - o.to_flat(R)) / max(np.linalg.norm(R), np.linalg.norm(Rv))
    assert err <= 1e-12, err
    V = np.random.default_rng(8).standard_normal(U.shape)
    v = torch.tensor(o.to_flat(V), device="cuda")
    for shift in (0.0, 12.5):
        ref = o.to_flat(o.operator(U, V, shift))
        assert rel(g.jvp(w, v, shift=shift).cpu().numpy(), ref) <= 1e-12
        assert rel(g.jvp_noalloc(w, v, shift=shift).cpu().numpy(), ref) <= 1e-12
    fd = g.jvp(w, v, shift=12.5, mode="fd").cpu().numpy()
    assert rel(fd, o.to_flat(o.jvp_fd(U, V) + 12.5 * o.mass()[None, :, None] * V)) <= 1e-6
    g.close()


@pytest.mark.parametrize("N,k,nq", [CASES[0], CASES[3]], ids=[IDS[0], IDS[3]])
def test_block_jacobi_and_fgmres_on_the_dae_system(N, k, nq):
    """Blocks D_K = shift M_K + dR_K/dU_K (zero mass on the pressure) against
    the oracle, and FGMRES[EWBJ] on G dw = b (b in the range of G) to 1e-10,
    re-checked with the oracle operator."""
    _say(f"incompressible blocks and FGMRES {N} P{k}")
    o, g, U, w = make_case(N, k, nq)
    shift = 20.0
    D = o.block_diagonal(U, shift=shift)
    r = np.random.default_rng(4).standard_normal(U.shape)
    z_o = block_solve(D, r.reshape(o.ne, -1)).reshape(U.shape)
    g.block_setup(w, shift)
    z_g = g.block_apply(torch.tensor(o.to_flat(r), device="cuda")).cpu().numpy()
    assert rel(z_g, o.to_flat(z_o)) <= 1e-11
    # on the periodic mesh a constant pressure is in the kernel of the DAE
    # operator (no mass, no pressure gradient, no pressure jump), so the
    # right-hand side is taken in its range: b = G x* for a random x*
    B = o.operator(U, np.random.default_rng(6).standard_normal(U.shape), shift)
    b = torch.tensor(o.to_flat(B), device="cuda")
    x, st = g.fgmres(w, shift, b, restart=30, rtol=1e-10, max_iter=3000, precond="bj")
    assert st["converged"] == 1 and st["rel_res_true"] <= 1e-10
    X = o.from_flat(x.cpu().numpy())
    res = np.linalg.norm(o.to_flat(o.operator(U, X, shift)) - o.to_flat(B)) / np.linalg.norm(B)
    assert res <= 1e-9
    # the wave speed of the interface flux's artificial compressibility system
    et = o.elem_tables(np.arange(o.ne))
    smax = o.phys.max_wave_speed(np.einsum("eqb,ecb->eqc", et["phi"], U)).max()
    assert abs(g.max_wave_speed(w) - smax) <= 1e-12 * smax
    g.close()


def test_vcycle_matches_the_oracle():
    """p-multigrid P2/P1 on the incompressible operator (inherited coarse
    operators of the DAE system): coarse operators 1e-12, one V-cycle 1e-9."""
    _say("incompressible p-multigrid")
    o, g, U, w = make_case((4, 3), 2, 4)
    shift, orders, iters = 15.0, (2, 1), (3, 10)
    mg = PMultigrid(o, U, shift, orders, iters)
    g.mg_setup(w, shift, orders, iters, storage="fp64", use_graph=True)
    X = np.random.default_rng(1).standard_normal((o.ne, o.nvar, mg.nbs[1]))
    y_o = (mg.A[1] @ X.reshape(-1)).reshape(X.shape)
    Xf = torch.tensor(np.ascontiguousarray(np.transpose(X, (1, 2, 0))).reshape(-1), device="cuda")
    y_g = g.mg_level_apply(1, Xf).cpu().numpy().reshape(o.nvar, mg.nbs[1], o.ne).transpose(2, 0, 1)
    assert np.linalg.norm(y_g - y_o) <= 1e-12 * np.linalg.norm(y_o)
    R = np.random.default_rng(2).standard_normal(U.shape)
    z_o = o.to_flat(mg.apply(R))
    z_g = g.mg_apply(torch.tensor(o.to_flat(R), device="cuda")).cpu().numpy()
    assert np.linalg.norm(z_g - z_o) <= 1e-9 * np.linalg.norm(z_o)
    g.close()


@pytest.mark.parametrize("scheme", ["lie", "ros2"])
def test_rosenbrock_step_with_the_mass_form(scheme):
    """Alg. ros with M acting on the velocities only (also in the stages'
    M dq/dt term) against the oracle's dense step."""
    from paper_1809_00866_amd import DG
    _say(f"incompressible rosenbrock {scheme}")
    coeffs = ros.ros2() if scheme == "ros2" else ros.linear_implicit_euler()
    mesh = synth.lattice_mesh((3, 2), L=1.0)
    o = DGOracle(mesh, 2, "P", 4, IncompressibleNS(2, nu=NU))
    U = o.project(synth.IncompressibleStandIn(2, seed=3))
    dt = 0.02
    U1 = ros.dg_step(o, U, dt, coeffs, lstsq=True)
    g = DG(mesh, 2, nq1d=4, mu=NU, physics="incompressible")
    w = torch.tensor(o.to_flat(U), device="cuda")
    g.block_setup(w, 1.0 / (coeffs["gamma"] * dt))
    w1, st = g.rosenbrock_step(w, dt, coeffs, rtol=1e-12, max_iter=1000, precond="bj")
    assert st["converged"] == 1
    # a constant pressure (mode 0 of the pressure, equal on the uniform
    # elements) is free on the periodic mesh: compare without it
    def drop_level(d):
        D = o.from_flat(d)
        D[:, -1, 0] -= D[:, -1, 0].mean()
        return o.to_flat(D)
    d_o = drop_level(o.to_flat(U1) - o.to_flat(U))
    d_g = drop_level(w1.cpu().numpy() - o.to_flat(U))
    assert np.linalg.norm(d_g - d_o) <= 1e-10 * np.linalg.norm(d_o), np.linalg.norm(d_g - d_o) / np.linalg.norm(d_o)
    g.close()


def test_incompressible_configurations_that_are_refused():
    from paper_1809_00866_amd import DG
    from paper_1809_00866_amd._lib import DGError
    with pytest.raises(DGError) as ei:
        DG(synth.lattice_mesh((2, 2, 2), L=1.0, perturb=0.1, seed=1), 2, nq1d=3, physics="incompressible")
    assert ei.value.status == -1
    o, g, U, w = make_case((2, 2, 2), 2, 3)
    with pytest.raises(DGError) as ei:
        g.residual(w, precision="fp32")
    assert ei.value.status == -1
    g.close()
