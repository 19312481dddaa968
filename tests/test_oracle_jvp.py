"""Pins for the oracle's Jacobian-vector products and diagonal blocks."""
import numpy as np
import pytest

import synth
from oracle import DGOracle, NavierStokes

GAMMA = 1.4


def _state(o, seed=2, noise=1e-2):
    d = o.d
    fld = synth.FreeStreamPlusModes(seed=seed) if d == 2 else synth.TaylorGreenStandIn(seed=seed, L=1.0)
    U = o.project(fld)
    rng = np.random.default_rng(seed)
    return U + noise * rng.standard_normal(U.shape) * np.abs(U[:, :, :1])


CASES = [((4, 4), 2, "Q", 4, 0.0, "roe"), ((3, 3, 3), 3, "P", 4, 0.1, "roe"), ((2, 2, 2), 2, "P", 3, 0.0, "lf")]


@pytest.mark.parametrize("N,k,space,nq,pert,flux", CASES)
def test_jvp_matches_central_difference(N, k, space, nq, pert, flux):
    o = DGOracle(synth.lattice_mesh(N, L=1.0, perturb=pert, seed=1), k, space, nq,
                 NavierStokes(len(N), mu=0.01, flux=flux))
    U = _state(o)
    V = np.random.default_rng(7).standard_normal(U.shape)
    Jv = o.jvp(U, V)
    # LF's max() has kinks; a smaller step keeps the stencil on one branch
    h = (1e-6 if flux == "roe" else 1e-9) * np.linalg.norm(U) / np.linalg.norm(V)
    fd = (o.residual(U + h * V) - o.residual(U - h * V)) / (2 * h)
    assert np.linalg.norm(Jv - fd) <= (1e-7 if flux == "roe" else 1e-6) * np.linalg.norm(Jv)


@pytest.mark.parametrize("N,k,space,nq,pert,flux", CASES)
def test_jvp_linear_and_conservative(N, k, space, nq, pert, flux):
    o = DGOracle(synth.lattice_mesh(N, L=1.0, perturb=pert, seed=1), k, space, nq,
                 NavierStokes(len(N), mu=0.01, flux=flux))
    U = _state(o)
    rng = np.random.default_rng(8)
    V1, V2 = rng.standard_normal(U.shape), rng.standard_normal(U.shape)
    a, b = 0.7, -1.3
    lhs = o.jvp(U, a * V1 + b * V2)
    rhs = a * o.jvp(U, V1) + b * o.jvp(U, V2)
    assert np.linalg.norm(lhs - rhs) <= 1e-14 * np.linalg.norm(lhs) * 10
    tot = np.einsum("e,ec->c", np.sqrt(o.element_volumes()), lhs[:, :, 0])
    assert np.abs(tot).max() <= 1e-12 * np.abs(lhs).max()


def test_paper_fd_jvp_close_to_exact():
    """eq. (epsdef) with eps = 1e-9: the one-sided FD product is within 1e-5."""
    o = DGOracle(synth.lattice_mesh((4, 4), L=1.0), 2, "Q", 4, NavierStokes(2, mu=2e-3))
    U = _state(o, noise=0.0)
    V = np.random.default_rng(9).standard_normal(U.shape)
    ex = o.jvp(U, V)
    fd = o.jvp_fd(U, V)
    assert np.linalg.norm(fd - ex) <= 1e-5 * np.linalg.norm(ex)


def test_block_diagonal_colouring_matches_brute_force():
    o = DGOracle(synth.lattice_mesh((2, 2, 2), L=1.0, perturb=0.1, seed=2), 1, "P", 2, NavierStokes(3, mu=0.01))
    U = _state(o)
    Dc = o.block_diagonal(U, shift=3.0, method="color")
    Db = o.block_diagonal(U, shift=3.0, method="brute")
    assert np.abs(Dc - Db).max() <= 1e-12 * np.abs(Db).max()
    # block K applied to a vector supported on K equals (G v)_K
    V = np.zeros(U.shape)
    V[3] = np.random.default_rng(0).standard_normal(U.shape[1:])
    Gv = o.operator(U, V, 3.0)
    assert np.abs(Gv[3].reshape(-1) - Db[3] @ V[3].reshape(-1)).max() <= 1e-12 * np.abs(Gv).max()


def test_single_element_block_is_whole_jacobian():
    o = DGOracle(synth.lattice_mesh((1, 1, 1), L=1.0), 2, "P", 3, NavierStokes(3, mu=0.01))
    U = _state(o)
    D = o.block_diagonal(U, shift=2.0)[0]
    V = np.random.default_rng(3).standard_normal(U.shape)
    assert np.abs(D @ V.reshape(-1) - o.operator(U, V, 2.0).reshape(-1)).max() < 1e-12 * np.abs(D).max()
