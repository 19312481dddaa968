"""Pins for the oracle's p-multigrid cycles (Sec. 2.4, Algs. vcic and fullvcic, eq. GalProj).

Each pin checks the oracle against something other than itself: the coarse
discretisation built independently at the lower degree, the colour-probed
sparse Jacobian, dense linear algebra, and least squares over an explicitly
built Krylov power basis.
"""
import numpy as np
import pytest

import synth
from oracle import DGOracle, NavierStokes, block_solve
from oracle.mms import sparse_jacobian
from oracle.pmg import (PMultigrid, diagonal_blocks, gmres_fixed, inherited_matrix, prolong,
                        restrict)


def _state(N, order, nq, mu=1e-2, seed=4, coarse_nb=None):
    mesh = synth.lattice_mesh(N, L=1.0)
    o = DGOracle(mesh, order, "P", nq, NavierStokes(3, mu=mu))
    U = o.project(synth.TaylorGreenStandIn(seed=seed, L=1.0))
    U = U + 1e-2 * np.random.default_rng(seed).standard_normal(U.shape) * np.abs(U[:, :, :1])
    if coarse_nb is not None:  # a state that lies in the coarse space
        U = prolong(restrict(U, coarse_nb), o.nb)
    return mesh, o, U


def _dense(o, U, shift):
    n = U.size
    A = np.zeros((n, n))
    for j in range(n):
        V = np.zeros(n)
        V[j] = 1.0
        A[:, j] = o.operator(U, V.reshape(U.shape), shift).reshape(-1)
    return A


def test_restriction_is_l2_projection_and_prolongation_its_right_inverse():
    """Keeping the low modes equals the L2 projection onto the coarse space built
    from the degree-1 basis of its own discretisation; R P = I."""
    mesh, o, U = _state((2, 2, 1), 3, 4)
    oc = DGOracle(mesh, 1, "P", 4, NavierStokes(3))
    et_f = o.elem_tables(np.arange(o.ne))
    et_c = oc.elem_tables(np.arange(o.ne))
    vals = np.einsum("eqb,ecb->eqc", et_f["phi"], U)            # the fine polynomial at the points
    proj = np.einsum("eq,eqc,eqb->ecb", et_c["wdet"], vals, et_c["phi"])
    assert np.abs(restrict(U, oc.nb) - proj).max() <= 1e-13 * np.abs(U).max()
    Xc = np.random.default_rng(0).standard_normal((o.ne, o.nvar, oc.nb))
    assert np.array_equal(restrict(prolong(Xc, o.nb), oc.nb), Xc)


@pytest.mark.parametrize("mu,equal", [(0.0, True), (5e-2, False)], ids=["inviscid", "viscous"])
def test_inherited_vs_rediscretised_coarse_operator(mu, equal):
    """Inherited and non-inherited coarse Jacobians coincide for the inviscid part
    and differ through the lifting operators for the viscous part (Sec. 2.4.2)."""
    shift = 3.0
    mesh, o, U = _state((1, 1, 2), 2, 3, mu=mu, coarse_nb=4)
    A_inh = inherited_matrix(o, U, shift, 4)
    oc = DGOracle(mesh, 1, "P", 3, NavierStokes(3, mu=mu))
    A_re = _dense(oc, restrict(U, 4), shift)
    diff = np.abs(A_inh - A_re).max() / np.abs(A_re).max()
    if equal:
        assert diff <= 1e-12, diff
    else:
        assert diff >= 1e-4, diff


def test_inherited_operator_matches_colour_probed_jacobian_and_nests():
    """G_1 = sub-matrix of the colour-probed assembled Jacobian; G_2 = leading
    sub-blocks of G_1 (eq. GalProj applied recursively)."""
    shift = 7.0
    mesh, o, U = _state((1, 2, 2), 2, 3)
    J = sparse_jacobian(o, U, shift).toarray()
    m = o.nvar * o.nb

    def idx(nbc):
        return np.array([e * m + c * o.nb + b for e in range(o.ne) for c in range(o.nvar) for b in range(nbc)])

    A1 = inherited_matrix(o, U, shift, 4)
    i1 = idx(4)
    assert np.abs(A1 - J[np.ix_(i1, i1)]).max() <= 1e-12 * np.abs(A1).max()
    A0 = inherited_matrix(o, U, shift, 1)
    m1 = o.nvar * 4
    i01 = np.array([e * m1 + c * 4 for e in range(o.ne) for c in range(o.nvar)])
    assert np.abs(A0 - A1[np.ix_(i01, i01)]).max() <= 1e-13 * np.abs(A0).max()
    D = diagonal_blocks(A1, o.ne, m1)
    for e in range(o.ne):
        assert np.array_equal(D[e], A1[e * m1:(e + 1) * m1, e * m1:(e + 1) * m1])


def test_fixed_gmres_is_the_minimal_residual_over_the_krylov_space():
    """Compare with least squares over the explicit power basis of K_k(A M^-1, r0)."""
    rng = np.random.default_rng(2)
    n = 40
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) / np.sqrt(n)
    Mi = np.diag(1.0 / np.diag(A))
    g = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    for k in (1, 3, 5):
        x = gmres_fixed(lambda v: A @ v, lambda v: Mi @ v, g, x0, k)
        r0 = g - A @ x0
        P = [r0]
        for _ in range(k - 1):
            P.append(A @ (Mi @ P[-1]))
        P = np.array(P).T
        y = np.linalg.lstsq(A @ Mi @ P, r0, rcond=None)[0]
        xr = x0 + Mi @ P @ y
        assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)
    assert np.array_equal(gmres_fixed(lambda v: A @ v, lambda v: v, g, x0, 0), x0)


def test_fixed_gmres_with_full_dimension_solves_exactly():
    mesh, o, U = _state((1, 1, 1), 1, 2)
    shift = 5.0
    A = _dense(o, U, shift)
    D = o.block_diagonal(U, shift)
    g = np.random.default_rng(3).standard_normal(A.shape[0])
    x = gmres_fixed(lambda v: A @ v, lambda v: block_solve(D, v.reshape(o.ne, -1)).reshape(-1), g, None,
                    A.shape[0])
    assert np.linalg.norm(x - np.linalg.solve(A, g)) <= 1e-9 * np.linalg.norm(x)


def test_two_grid_without_smoothing_is_the_coarse_galerkin_solve():
    """With no fine smoothing and an exact coarsest solve, Alg. vcic returns
    P (R G P)^-1 R g, with R G P solved by dense LU."""
    mesh, o, U = _state((1, 1, 2), 2, 3)
    shift = 4.0
    nc = o.ne * o.nvar * 4
    mg = PMultigrid(o, U, shift, orders=(2, 1), iters=(0, nc))
    R = np.random.default_rng(5).standard_normal(U.shape)
    z = mg.apply(R)
    A1 = inherited_matrix(o, U, shift, 4)
    zc = np.linalg.solve(A1, restrict(R, 4).reshape(-1)).reshape(o.ne, o.nvar, 4)
    assert np.linalg.norm(z - prolong(zc, o.nb)) <= 1e-9 * np.linalg.norm(zc)


def test_coarse_correction_annihilates_the_restricted_defect():
    """With an exact coarsest solve the Galerkin correction makes the restricted
    defect vanish: R(g - G w_hat) = R d - (R G P) e = 0.  Pre-smoothing and
    post-smoothing each reduce the residual (GMRES minimises it over a space
    that contains the starting point; strictly, unless it stagnates)."""
    mesh, o, U = _state((1, 1, 2), 2, 3)
    shift = 4.0
    nc = o.ne * o.nvar * 4
    mg = PMultigrid(o, U, shift, orders=(2, 1), iters=(2, nc))
    g = np.random.default_rng(8).standard_normal(U.size)
    tr = {}
    z = mg.vcycle(0, g, trace=tr)
    w, w_hat = tr[0]
    res = lambda x: g - mg.apply_G(0, x)
    rd = restrict(res(w_hat).reshape(U.shape), 4)
    assert np.linalg.norm(rd) <= 1e-10 * np.linalg.norm(g)
    assert np.linalg.norm(res(w)) < np.linalg.norm(g)
    assert np.linalg.norm(res(z)) < np.linalg.norm(res(w_hat))


def test_full_cycle_two_grid_is_the_galerkin_solve_and_its_correction_vanishes():
    """Alg. fullvcic on two levels with no fine smoothing and an exact coarsest
    solve: the prolonged coarse solution w_hat = P (R G P)^-1 R g has a defect
    whose restriction is zero, so the V-cycle correction adds nothing and the
    cycle returns w_hat (a wrong sign of the defect would double it)."""
    mesh, o, U = _state((1, 1, 2), 2, 3)
    shift = 4.0
    nc = o.ne * o.nvar * 4
    mg = PMultigrid(o, U, shift, orders=(2, 1), iters=(0, nc), cycle="full")
    R = np.random.default_rng(11).standard_normal(U.shape)
    z = mg.apply(R)
    A1 = inherited_matrix(o, U, shift, 4)
    zc = np.linalg.solve(A1, restrict(R, 4).reshape(-1)).reshape(o.ne, o.nvar, 4)
    assert np.linalg.norm(z - prolong(zc, o.nb)) <= 1e-9 * np.linalg.norm(zc)


def test_full_cycle_three_levels_with_exact_middle_smoothing():
    """Three levels (P2/P1/P0), exact GMRES on the two coarse levels and no fine
    smoothing: the level-1 full cycle ends with an exact post-smoothing, so the
    result is again P (R G P)^-1 R g with the level-1 inherited operator."""
    mesh, o, U = _state((1, 1, 2), 2, 3)
    shift = 4.0
    n1, n2 = o.ne * o.nvar * 4, o.ne * o.nvar
    R = np.random.default_rng(12).standard_normal(U.shape)
    A1 = inherited_matrix(o, U, shift, 4)
    zc = np.linalg.solve(A1, restrict(R, 4).reshape(-1)).reshape(o.ne, o.nvar, 4)
    mg = PMultigrid(o, U, shift, orders=(2, 1, 0), iters=(0, n1, n2), cycle="full")
    z = mg.apply(R)
    assert np.linalg.norm(z - prolong(zc, o.nb)) <= 1e-9 * np.linalg.norm(zc)


def test_lagged_hierarchy_keeps_the_coarse_solve_and_follows_the_fine_operator():
    """Preconditioner lagging: built at state U1, updated to (U2, shift2).
    Without fine smoothing and with an exact coarse solve the cycle is still
    P (R G(U1) P)^-1 R g (the coarse level is frozen); with a fine smoothing
    count equal to the fine dimension the post-smoothing is an exact solve with
    the new operator G(U2), so the cycle returns G(U2)^-1 g (dense LU)."""
    mesh, o, U1 = _state((1, 1, 2), 2, 3, seed=4)
    _, _, U2 = _state((1, 1, 2), 2, 3, seed=9)
    s1, s2 = 4.0, 6.0
    nc, nf = o.ne * o.nvar * 4, U1.size
    g = np.random.default_rng(13).standard_normal(U1.shape)
    mg = PMultigrid(o, U1, s1, orders=(2, 1), iters=(0, nc))
    mg.update_fine(U2, s2)
    A1 = inherited_matrix(o, U1, s1, 4)
    zc = np.linalg.solve(A1, restrict(g, 4).reshape(-1)).reshape(o.ne, o.nvar, 4)
    assert np.linalg.norm(mg.apply(g) - prolong(zc, o.nb)) <= 1e-9 * np.linalg.norm(zc)
    mg = PMultigrid(o, U1, s1, orders=(2, 1), iters=(nf, nc))
    mg.update_fine(U2, s2)
    z = mg.apply(g).reshape(-1)
    z_ex = np.linalg.solve(_dense(o, U2, s2), g.reshape(-1))
    assert np.linalg.norm(z - z_ex) <= 1e-8 * np.linalg.norm(z_ex)


def test_block_ilu0_reproduces_the_operator_on_its_pattern():
    """ILU(0): L U agrees with A on every block of the pattern (element and
    face neighbours) and differs only by the dropped fill; on two elements the
    pattern is closed under elimination, so the factorisation is exact."""
    from oracle.pmg import BlockILU0, greedy_colouring
    mesh, o, U = _state((3, 3, 2), 1, 2)
    shift = 4.0
    A = inherited_matrix(o, U, shift, 1)                        # P0 level: m = 5
    m = o.nvar
    ilu = BlockILU0(A, o.ne, m, o.nbr, greedy_colouring(o.nbr))
    L, Uf = ilu.factors()
    M = L @ Uf
    mask = np.kron(ilu.pat, np.ones((m, m), dtype=bool))
    assert np.abs((M - A)[mask]).max() <= 1e-12 * np.abs(A).max()
    assert np.abs((M - A)[~mask]).max() > 1e-8 * np.abs(A).max()      # fill was dropped
    r = np.random.default_rng(9).standard_normal(A.shape[0])
    assert np.allclose(M @ ilu.solve(r), r, rtol=0, atol=1e-10 * np.abs(r).max())
    mesh2, o2, U2 = _state((2, 1, 1), 1, 2)
    A2 = inherited_matrix(o2, U2, shift, 4)
    ilu2 = BlockILU0(A2, o2.ne, o2.nvar * 4, o2.nbr, greedy_colouring(o2.nbr))
    r2 = np.random.default_rng(10).standard_normal(A2.shape[0])
    assert np.allclose(ilu2.solve(r2), np.linalg.solve(A2, r2), rtol=1e-10, atol=1e-12)


def test_greedy_colouring_is_proper():
    from oracle.pmg import greedy_colouring
    mesh, o, U = _state((3, 4, 2), 1, 2)
    col = greedy_colouring(o.nbr)
    for e in range(o.ne):
        assert all(col[n] != col[e] for n in o.nbr[e] if n != e)


@pytest.mark.slow
def test_mg_preconditioned_fgmres_beats_block_jacobi():
    from oracle import fgmres
    mesh, o, U = _state((3, 3, 2), 2, 3)
    shift = 2.0
    mg = PMultigrid(o, U, shift, orders=(2, 1, 0), iters=(4, 4, 20))
    D = mg.D[0]
    B = np.random.default_rng(6).standard_normal(U.shape).reshape(-1)
    A = lambda v: o.operator(U, v.reshape(U.shape), shift).reshape(-1)
    _, i_bj = fgmres(A, B, apply_M=lambda v: block_solve(D, v.reshape(o.ne, -1)).reshape(-1), rtol=1e-10,
                     max_iter=600)
    x, i_mg = fgmres(A, B, apply_M=lambda v: mg.apply(v.reshape(U.shape)).reshape(-1), rtol=1e-10,
                     max_iter=600)
    assert i_mg["converged"] and i_bj["converged"]
    assert np.linalg.norm(A(x) - B) <= 1e-10 * np.linalg.norm(B) * 1.01
    assert i_mg["iters"] < i_bj["iters"]
