"""Pins for the oracle's FGMRES and block-Jacobi solve (dense linear algebra)."""
import numpy as np

import synth
from oracle import DGOracle, NavierStokes, block_solve, fgmres


def _dense_G(shift=50.0):
    o = DGOracle(synth.lattice_mesh((4, 4), L=1.0), 2, "Q", 4, NavierStokes(2, mu=2e-3))
    U = o.project(synth.FreeStreamPlusModes(seed=1))
    n = U.size
    A = np.zeros((n, n))
    for j in range(n):
        V = np.zeros(n)
        V[j] = 1.0
        A[:, j] = o.operator(U, V.reshape(U.shape), shift).reshape(-1)
    return o, U, A


def test_fgmres_matches_dense_solve_and_is_monotone():
    o, U, A = _dense_G()
    b = np.random.default_rng(0).standard_normal(A.shape[0])
    x, info = fgmres(lambda v: A @ v, b, restart=30, rtol=1e-10, max_iter=2000)
    xd = np.linalg.solve(A, b)
    assert info["converged"]
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd) * np.linalg.cond(A) ** 0.5
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    h = np.array(info["history"][:30])  # inside the first cycle the estimate is monotone
    assert np.all(np.diff(h) <= 1e-12 * h[0])


def test_fgmres_modified_gram_schmidt_matches_the_dense_solve_and_cgs2():
    """Both orthogonalisations span the same Krylov spaces: the same iteration
    count and solution (to the tolerance), and the dense solution."""
    o, U, A = _dense_G()
    b = np.random.default_rng(2).standard_normal(A.shape[0])
    x1, i1 = fgmres(lambda v: A @ v, b, restart=20, rtol=1e-10, max_iter=2000, orth="mgs")
    x2, i2 = fgmres(lambda v: A @ v, b, restart=20, rtol=1e-10, max_iter=2000, orth="cgs2")
    assert i1["converged"] and i2["converged"] and abs(i1["iters"] - i2["iters"]) <= 1
    assert np.linalg.norm(b - A @ x1) <= 1e-10 * np.linalg.norm(b)
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x1 - xd) <= 1e-8 * np.linalg.norm(xd) * np.linalg.cond(A) ** 0.5
    h1, h2 = np.array(i1["history"][:20]), np.array(i2["history"][:20])
    assert np.allclose(h1, h2, rtol=1e-8, atol=1e-12 * h1[0])


def test_fgmres_exact_preconditioner_one_iteration():
    _, _, A = _dense_G()
    Ainv = np.linalg.inv(A)
    b = np.random.default_rng(1).standard_normal(A.shape[0])
    x, info = fgmres(lambda v: A @ v, b, apply_M=lambda v: Ainv @ v, rtol=1e-10)
    assert info["converged"] and info["iters"] == 1


def test_fgmres_edge_cases():
    A = np.diag(np.arange(1.0, 11.0))
    x, info = fgmres(lambda v: A @ v, np.zeros(10))
    assert info["converged"] and info["iters"] == 0 and not np.any(x)
    b = np.ones(10)
    x, info = fgmres(lambda v: A @ v, b, max_iter=1, rtol=1e-12)
    assert not info["converged"] and info["iters"] == 1


def test_block_jacobi_of_dg_operator():
    """EWBJ: block_solve with the diagonal blocks equals solving each diagonal block;
    with the diagonal-block preconditioner FGMRES converges faster than without."""
    o, U, A = _dense_G(shift=20.0)
    m = o.nvar * o.nb
    # oracle flat order here is (e, c, b): diagonal blocks are contiguous
    D = np.stack([A[e * m:(e + 1) * m, e * m:(e + 1) * m] for e in range(o.ne)])
    D2 = o.block_diagonal(U, shift=20.0)
    assert np.abs(D - D2).max() < 1e-11 * np.abs(D).max()
    r = np.random.default_rng(2).standard_normal((o.ne, m))
    z = block_solve(D, r)
    assert np.abs(np.einsum("eij,ej->ei", D, z) - r).max() < 1e-11
    b = np.random.default_rng(3).standard_normal(A.shape[0])
    M = lambda v: block_solve(D, v.reshape(o.ne, m)).reshape(-1)
    _, i0 = fgmres(lambda v: A @ v, b, rtol=1e-8, max_iter=3000)
    _, i1 = fgmres(lambda v: A @ v, b, apply_M=M, rtol=1e-8, max_iter=3000)
    assert i1["converged"] and i1["iters"] < i0["iters"]
