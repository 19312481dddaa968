"""Pins for the oracle's BR2 stabilisation Jacobian (DGOracle.stab_jvp, the last
term of eq. jacTrilFNURef) and the rescaled-inherited coarse operators of
App. A (oracle/pmg.py, eq. GalProjResc).

For the linear BR2 Laplacian the stabilisation part is exactly the difference
of the operators with and without the penalty eta, and it is symmetric
positive semi-definite (it is eta times a sum of products of liftings).
Without viscosity it vanishes, and the rescaled hierarchy is the inherited
one."""
import numpy as np

import synth
from oracle import DGOracle, Diffusion, NavierStokes
from oracle.pmg import PMultigrid, stab_scale


def _dense(f, shape):
    n = int(np.prod(shape))
    A = np.zeros((n, n))
    for j in range(n):
        V = np.zeros(n)
        V[j] = 1.0
        A[:, j] = f(V.reshape(shape)).reshape(-1)
    return A


def _laplacian(eta):
    mesh = synth.lattice_mesh((3, 3), L=1.0)
    o = DGOracle(mesh, 2, "P", 3, Diffusion(2, mu=0.7, eta=eta))
    U = np.zeros((o.ne, 1, o.nb))
    return o, U


def test_laplacian_stabilisation_is_the_penalty_difference_and_spd():
    o, U = _laplacian(5.0)
    o0, _ = _laplacian(0.0)
    S = _dense(lambda V: o.stab_jvp(U, V), U.shape)
    J = _dense(lambda V: o.jvp(U, V), U.shape)
    J0 = _dense(lambda V: o0.jvp(U, V), U.shape)
    assert np.abs(S - (J - J0)).max() <= 1e-12 * np.abs(J).max()
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert ev.min() >= -1e-12 * ev.max() and ev.max() > 0


def test_inviscid_stabilisation_vanishes_and_rescaling_changes_nothing():
    mesh = synth.lattice_mesh((1, 1, 2), L=1.0)
    o = DGOracle(mesh, 2, "P", 3, NavierStokes(3, mu=0.0))
    U = o.project(synth.TaylorGreenStandIn(seed=4, L=1.0))
    V = np.random.default_rng(1).standard_normal(U.shape)
    assert np.abs(o.stab_jvp(U, V)).max() == 0.0
    a = PMultigrid(o, U, 3.0, orders=(2, 1, 0), iters=(1, 1, 2))
    b = PMultigrid(o, U, 3.0, orders=(2, 1, 0), iters=(1, 1, 2), rescale=True)
    for l in (1, 2):
        assert np.array_equal(a.A[l], b.A[l])


def test_scale_factors_and_viscous_rescaling_changes_the_coarse_operator():
    """The scale factors of App. A (S = k1 (k1 + d) / (k0 (k0 + d))), and with
    viscosity the rescaled level-1 operator differs from the inherited one."""
    assert stab_scale(2, 1, 3) == 4 / 10 and stab_scale(4, 2, 3) == 10 / 28 and stab_scale(1, 0, 3) == 0.0
    mesh = synth.lattice_mesh((1, 1, 2), L=1.0)
    o = DGOracle(mesh, 2, "P", 3, NavierStokes(3, mu=5e-2))
    U = o.project(synth.TaylorGreenStandIn(seed=4, L=1.0))
    a = PMultigrid(o, U, 3.0, orders=(2, 1), iters=(1, 2))
    b = PMultigrid(o, U, 3.0, orders=(2, 1), iters=(1, 2), rescale=True)
    D = a.A[1] - b.A[1]
    assert np.abs(D).max() > 1e-8 * np.abs(a.A[1]).max()
