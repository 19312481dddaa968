"""Pins of the incompressible oracle (Sec. 2.1, eq. ns; mass form of eq.
massBil): free-stream preservation and discrete conservation (divergence
theorem), the artificial-compressibility Lax-Friedrichs interface flux at a
state pair computed by hand, the differential-algebraic operator (the shift
acts on the velocities only), the exact Jv against a central difference, and
convergence on a manufactured solution (velocity at p+1, pressure at p)."""
import numpy as np
import pytest

import synth
from oracle import DGOracle, IncompressibleNS
from oracle.mms import solve_mms
from oracle.quadrature import tensor_rule
from synth.fields import TrigSum

CASES = [((3, 4), 2, 4, 0.0), ((3, 4), 2, 4, 0.1), ((2, 2, 3), 2, 3, 0.1), ((2, 3, 2), 1, 2, 0.0)]


def _oracle(N, k, nq, pert, nu=1e-2, seed=3):
    mesh = synth.lattice_mesh(N, L=1.0, perturb=pert, seed=seed if pert else None)
    return DGOracle(mesh, k, "P", nq, IncompressibleNS(len(N), nu=nu))


@pytest.mark.parametrize("N,k,nq,pert", CASES)
def test_free_stream_and_conservation(N, k, nq, pert):
    o = _oracle(N, k, nq, pert)
    d = len(N)
    w0 = np.array([0.3, -0.2, 0.1][:d] + [0.7])
    U = o.project(lambda x: np.broadcast_to(w0, x.shape[:-1] + (d + 1,)))
    R, Rv = o.residual(U, return_parts=True)
    assert np.abs(R).max() <= 1e-13 * np.abs(Rv).max()
    # conservation: the residual tested with 1 sums to zero for every equation
    U = o.project(synth.IncompressibleStandIn(d, seed=5))
    R = o.residual(U)
    vol = o.element_volumes()
    sums = np.einsum("e,ec->c", np.sqrt(vol), R[:, :, 0])
    assert np.abs(sums).max() <= 1e-13 * np.abs(R).max()


def test_artificial_compressibility_flux_hand_computed():
    # L: u (0.3, -0.2), p 0.5; R: u (0.1, 0.4), p 0.7; n (0.6, 0.8), beta 1
    #   u.n: 0.02 and 0.38; lambda = max(0.02 + sqrt(1.0004), 0.38 + sqrt(1.1444)) = 1.44976633 (R side)
    #   F.n(L) = (0.306, 0.396, 0.02), F.n(R) = (0.458, 0.712, 0.38), w_R - w_L = (-0.2, 0.6, 0.2)
    ns = IncompressibleNS(2, nu=0.0)
    H = ns.conv_numflux(np.array([0.3, -0.2, 0.5]), np.array([0.1, 0.4, 0.7]), np.array([0.6, 0.8]))
    assert np.allclose(H, [0.5269766329625307, 0.11907010111240796, 0.05502336703746938], rtol=0, atol=1e-14)
    # beta scales the pressure dissipation by 1/beta^2 and enters lambda
    ns2 = IncompressibleNS(2, nu=0.0, beta=2.0)
    H2 = ns2.conv_numflux(np.array([0.3, -0.2, 0.5]), np.array([0.1, 0.4, 0.7]), np.array([0.6, 0.8]))
    lam2 = 0.38 + np.sqrt(0.38 ** 2 + 4.0)
    assert abs(H2[2] - (0.2 - 0.5 * lam2 * 0.2 / 4.0)) <= 1e-14
    assert abs(H2[0] - (0.382 + 0.5 * lam2 * 0.2)) <= 1e-14


def test_operator_is_differential_algebraic():
    o = _oracle((2, 3), 2, 4, 0.0)
    U = o.project(synth.IncompressibleStandIn(2, seed=9))
    V = np.random.default_rng(1).standard_normal(U.shape)
    diff = o.operator(U, V, 7.0) - o.operator(U, V, 0.0)
    assert np.allclose(diff[:, :2], 7.0 * V[:, :2], rtol=1e-13, atol=1e-13)
    assert np.abs(diff[:, 2]).max() <= 1e-13
    D = o.block_diagonal(U, shift=7.0) - o.block_diagonal(U, shift=0.0)
    assert np.allclose(np.diagonal(D, axis1=1, axis2=2), np.repeat([7.0, 7.0, 0.0], o.nb)[None], atol=1e-12)


@pytest.mark.parametrize("N,k,nq,pert", [CASES[1], CASES[2]])
def test_jvp_matches_central_difference(N, k, nq, pert):
    o = _oracle(N, k, nq, pert)
    U = o.project(synth.IncompressibleStandIn(len(N), seed=5))
    V = np.random.default_rng(2).standard_normal(U.shape)
    h = 1e-6 * np.linalg.norm(U) / np.linalg.norm(V)
    fd = (o.residual(U + h * V) - o.residual(U - h * V)) / (2 * h)
    J = o.jvp(U, V)
    assert np.linalg.norm(J - fd) <= 1e-7 * np.linalg.norm(J)


@pytest.mark.slow
@pytest.mark.parametrize("k", [1, 2])
def test_manufactured_solution_rates(k):
    """sigma w + div F(w) = s with sigma = 0.01 on every variable (which fixes
    the pressure level on the periodic square): velocity L2 errors at rate
    >= p+1-0.3, pressure at >= p (equal-order pressure)."""
    rng = np.random.default_rng(0)
    fld = TrigSum(a=[0.3, -0.2, 0.5], b=0.1 * rng.standard_normal((3, 3)),
                  k=2 * np.pi * np.array([[1, 0], [0, 1], [1, 1]]), phi=rng.uniform(0, 6, 3))
    xi, w = tensor_rule(k + 5, 2)
    errs = []
    for N in (4, 8, 16):
        o = DGOracle(synth.lattice_mesh((N, N), L=1.0), k, "P", k + 2, IncompressibleNS(2, nu=1e-2))
        U = solve_mms(o, fld, sigma=0.01)
        x, uh, det = o.evaluate(U, xi)
        e = uh - fld.value(x)
        errs.append(np.sqrt(np.einsum("q,eq,eqc->c", w, det, e * e)))
    errs = np.array(errs)
    rates = np.log2(errs[1] / errs[2])
    assert rates[0] >= k + 1 - 0.3 and rates[1] >= k + 1 - 0.3, rates
    assert rates[2] >= k, rates
