"""Pins for the oracle residual: free stream, conservation, flux identities,
BR2 symmetry/sign, projection exactness and manufactured-solution convergence."""
import numpy as np
import pytest

import synth
from oracle import DGOracle, Diffusion, NavierStokes
from oracle.mms import l2_error, solve_mms

GAMMA = 1.4


def _case(N, k, space, nq, perturb=0.0, flux="roe", mu=0.01, seed=5, L=1.0):
    mesh = synth.lattice_mesh(N, L=L, perturb=perturb, seed=seed)
    return DGOracle(mesh, k, space, nq, NavierStokes(len(N), mu=mu, flux=flux))


CASES = [((4, 4), 2, "Q", 4), ((3, 3, 3), 2, "P", 3), ((2, 2, 2), 3, "P", 4), ((2, 3, 2), 4, "P", 5)]


@pytest.mark.parametrize("N,k,space,nq", CASES)
@pytest.mark.parametrize("perturb", [0.0, 0.1])
@pytest.mark.parametrize("flux", ["roe", "lf"])
def test_free_stream_preservation(N, k, space, nq, perturb, flux):
    o = _case(N, k, space, nq, perturb, flux)
    d = len(N)
    U = o.project(synth.UniformState(1.0, [0.3, -0.2, 0.1][:d], 1.0 / GAMMA, GAMMA))
    R, Rvol = o.residual(U, return_parts=True)
    assert np.abs(Rvol).max() > 0.1
    assert np.abs(R).max() <= 1e-12 * np.abs(Rvol).max() * 10


@pytest.mark.parametrize("N,k,space,nq", CASES)
@pytest.mark.parametrize("perturb", [0.0, 0.1])
def test_discrete_conservation(N, k, space, nq, perturb):
    """Testing with z = 1: sum_K sqrt|K| R_K,0,c = 0 (faces single valued, grad 1 = 0)."""
    o = _case(N, k, space, nq, perturb)
    d = len(N)
    fld = synth.FreeStreamPlusModes(seed=3) if d == 2 else synth.TaylorGreenStandIn(seed=3, L=1.0)
    U = o.project(fld)
    U = U + 1e-2 * np.random.default_rng(1).standard_normal(U.shape) * np.abs(U).max(axis=2, keepdims=True)
    R, Rvol = o.residual(U, return_parts=True)
    tot = np.einsum("e,ec->c", np.sqrt(o.element_volumes()), R[:, :, 0])
    assert np.abs(tot).max() <= 1e-12 * np.abs(Rvol).max()


def test_physical_orthonormality_curved():
    o = _case((3, 3, 3), 3, "P", 4, perturb=0.1)
    et = o.elem_tables(np.arange(o.ne))
    M = np.einsum("eq,eqa,eqb->eab", et["wdet"], et["phi"], et["phi"])
    assert np.abs(M - np.eye(o.nb)[None]).max() < 1e-13
    # affine element: phi = psi / sqrt|J|
    o2 = _case((3, 3, 3), 3, "P", 4)
    et2 = o2.elem_tables([0])
    assert np.allclose(et2["phi"][0], o2.psi_v / np.sqrt(et2["det"][0][:, None]), atol=1e-13)


def test_subset_evaluation_matches_full():
    o = _case((3, 3, 3), 2, "P", 3, perturb=0.1)
    U = o.project(synth.TaylorGreenStandIn(seed=4, L=1.0))
    R, Rvol = o.residual(U, return_parts=True)
    for sub in ([0], [5, 26], [1, 2, 13]):  # same sums in another order: round-off of the volume term
        assert np.abs(o.residual(U, elems=sub) - R[sub]).max() < 1e-14 * np.abs(Rvol).max()


def test_face_points_conform():
    o = _case((3, 3, 3), 2, "P", 3, perturb=0.1)
    fp = np.repeat(np.arange(3), o.ne)
    fo = np.tile(np.arange(o.ne), 3)
    ft = o.face_tables(fp, fo)
    gap = ft["xL"] - ft["xR"]
    gap -= np.round(gap / 1.0) * 1.0  # periodic images
    assert np.abs(gap).max() < 1e-13


@pytest.mark.parametrize("flux", ["roe", "lf"])
def test_numflux_consistency_and_roe_property(flux):
    ph = NavierStokes(3, flux=flux)
    rng = np.random.default_rng(0)
    n = rng.standard_normal((50, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    prim = lambda: (1 + 0.3 * rng.random(50), 0.5 * rng.standard_normal((50, 3)), 1 + 0.5 * rng.random(50))
    UL = synth.primitive_to_conserved(*prim(), GAMMA)
    UR = synth.primitive_to_conserved(*prim(), GAMMA)
    Fn = lambda U: np.einsum("...pc,...p->...c", ph.conv_flux(U), n)
    assert np.abs(ph.conv_numflux(UL, UL, n) - Fn(UL)).max() < 1e-13
    # Roe property: A_roe (UR - UL) = F(UR).n - F(UL).n with signed eigenvalues
    D = NavierStokes(3).roe_dissipation(UL, UR, n, signed=True)
    assert np.abs(D - (Fn(UR) - Fn(UL))).max() < 1e-12
    # conservation of the numerical flux: H(UL,UR,n) = -H(UR,UL,-n)
    assert np.abs(ph.conv_numflux(UL, UR, n) + ph.conv_numflux(UR, UL, -n)).max() < 1e-12


def test_viscous_flux_closed_forms():
    mu, Pr = 0.3, 0.72
    ph = NavierStokes(3, mu=mu, prandtl=Pr)
    rho, u, p = 1.3, np.array([0.2, -0.1, 0.4]), 2.0
    U = synth.primitive_to_conserved(np.array(rho), u, np.array(p), GAMMA)
    # velocity gradient A (du_i/dx_j) and p/rho gradient b, converted to conservative gradients
    A = np.array([[0.1, 0.7, 0.0], [-0.2, 0.3, 0.5], [0.4, 0.0, -0.6]])
    b = np.array([0.05, -0.02, 0.03])
    grho = np.array([0.11, -0.07, 0.02])
    G = np.zeros((5, 3))
    G[0] = grho
    for i in range(3):
        G[1 + i] = rho * A[i] + u[i] * grho
    # rho*E = p/(g-1) + rho|u|^2/2 with p = rho*(p/rho)
    ppr = p / rho
    gp = rho * b + ppr * grho
    G[4] = gp / (GAMMA - 1) + 0.5 * (np.sum(u * u)) * grho + rho * (A.T @ u)
    F = ph.visc_flux(U, G)
    tau = mu * (A + A.T - 2.0 / 3.0 * np.trace(A) * np.eye(3))
    kap = mu * GAMMA / (Pr * (GAMMA - 1))
    assert np.allclose(F[:, 0], 0)
    assert np.allclose(F[:, 1:4], tau, atol=1e-14)
    assert np.allclose(F[:, 4], tau @ u + kap * b, atol=1e-14)


def _assemble(o, U):
    n = U.size
    A = np.zeros((n, n))
    for j in range(n):
        V = np.zeros(n)
        V[j] = 1.0
        A[:, j] = o.jvp(U, V.reshape(U.shape)).reshape(-1)
    return A


@pytest.mark.parametrize("N,k,space,nq", [((4, 4), 2, "Q", 4), ((2, 2, 2), 2, "P", 3)])
def test_br2_laplacian_sign(N, k, space, nq):
    """Adopted lifting sign: symmetric PSD with only constants in the kernel.
    The sign printed in eq. (vflux) gives a non-symmetric indefinite operator."""
    mesh = synth.lattice_mesh(N, L=1.0)
    for sign in (+1, -1):
        o = DGOracle(mesh, k, space, nq, Diffusion(len(N), mu=1.0), lifting_sign=sign)
        A = _assemble(o, np.zeros((o.ne, 1, o.nb)))
        asym = np.abs(A - A.T).max() / np.abs(A).max()
        ev = np.linalg.eigvalsh(0.5 * (A + A.T))
        if sign > 0:
            assert asym < 1e-13
            assert ev[0] > -1e-10 * ev[-1]
            assert np.sum(np.abs(ev) < 1e-10 * ev[-1]) == 1
        else:
            assert asym > 1e-3
            assert ev[0] < -0.1 * ev[-1]


def test_projection_reproduces_polynomials():
    """On affine elements P_k contains every polynomial of total degree <= k in x."""
    o = DGOracle(synth.lattice_mesh((2, 2, 2), L=1.0), 3, "P", 4, NavierStokes(3))
    f = lambda x: np.stack([1 + x[..., 0] ** 3 - 2 * x[..., 1] * x[..., 2] + x[..., 0] * x[..., 1] * x[..., 2]] * 5, -1)
    U = o.project(f)
    xi = np.random.default_rng(0).uniform(-1, 1, (7, 3))
    x, uh, _ = o.evaluate(U, xi)
    assert np.abs(uh - f(x)).max() < 1e-12


def _mms_rate(o_of_N, field, Ns, sigma):
    errs = []
    for N in Ns:
        o = o_of_N(N)
        errs.append(l2_error(o, solve_mms(o, field, sigma=sigma), field))
    return np.log2(np.array(errs[:-1]) / np.array(errs[1:]))


@pytest.mark.slow
def test_mms_navier_stokes_q2_rate():
    """Q2 compressible NS (Roe + BR2, Re ~ 500): L2 error rate >= p+1-0.3."""
    fld = synth.TrigSum(a=[1.0, 0.5, 0.3, 1 / (GAMMA * (GAMMA - 1)) + 0.5 * 0.34],
                        b=[[0.1, 0.05, 0], [0.02, 0, 0.03], [0, 0.03, 0.02], [0.1, 0.05, 0.05]],
                        k=[[2 * np.pi, 0], [0, 2 * np.pi], [2 * np.pi, 2 * np.pi]], phi=[0.3, 1.1, 2.0])
    mk = lambda N: DGOracle(synth.lattice_mesh((N, N), L=1.0), 2, "Q", 4, NavierStokes(2, mu=1e-3, flux="roe"))
    rates = _mms_rate(mk, fld, (4, 8, 16), sigma=0.01)
    assert rates[-1] >= 2.7, rates


@pytest.mark.slow
def test_mms_br2_diffusion_p2_3d_rate():
    """P2 (total degree) BR2 diffusion in 3D, u + div(-grad u) = s: rate >= p+1-0.3."""
    fld = synth.TrigSum(a=[1.0], b=[[0.3, 0.2]], k=[[2 * np.pi, 0, 2 * np.pi], [0, 2 * np.pi, 2 * np.pi]],
                        phi=[0.3, 1.1])
    mk = lambda N: DGOracle(synth.lattice_mesh((N, N, N), L=1.0), 2, "P", 3, Diffusion(3, mu=0.05))
    rates = _mms_rate(mk, fld, (4, 8), sigma=1.0)
    assert rates[-1] >= 2.7, rates


def test_mms_br2_diffusion_q2_rate():
    fld = synth.TrigSum(a=[1.0], b=[[0.3, 0.2, 0.1]], k=[[2 * np.pi, 0], [0, 2 * np.pi], [2 * np.pi, 2 * np.pi]],
                        phi=[0.3, 1.1, 2.0])
    mk = lambda N: DGOracle(synth.lattice_mesh((N, N), L=1.0), 2, "Q", 4, Diffusion(2, mu=0.1))
    rates = _mms_rate(mk, fld, (4, 8, 16), sigma=1.0)
    assert rates[-1] >= 2.7, rates
