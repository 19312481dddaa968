"""Pins of oracle parts that the convergence and consistency tests cannot see.

* Lax-Friedrichs flux: consistency, conservation and MMS convergence hold for
  any wave speed lambda >= 0, so the flux is checked against values computed
  by hand from the primitive variables (two state pairs, oblique normals,
  negative normal velocity, either side giving the maximum).
* Roe flux: the characteristic-wave sum with Harten's entropy fix equals the
  matrix function |A|_delta (A) dU of the Roe matrix A = dF.n/dU at the
  Roe-averaged state, built here by eigendecomposition (fix inactive, and
  active on the contact/shear waves and on an acoustic wave).
* Time step rule dt = CFL h / ((2p+1) max(|u| + c)) and the wave speed at a
  fixed state, by hand.
* Finite-difference step of eq. (epsdef): Delta = 1e-9 sqrt(1 + ||w||)/||v||
  with ||w|| = 8 and ||v|| = 2, i.e. Delta = 1.5e-9, both as the exposed step
  and as the step jvp_fd really takes (read back through a quadratic residual
  for which the one-sided quotient is exactly Delta v^2).
"""
import numpy as np
import pytest

from oracle import DGOracle, NavierStokes, backward_euler_dt
import synth

GAMMA = 1.4


def conserved(rho, u, p):
    u = np.asarray(u, dtype=np.float64)
    return np.concatenate([[rho], rho * u, [p / (GAMMA - 1.0) + 0.5 * rho * u @ u]])


# Hand computation, pair 1 (3D), n = (0.6, 0.8, 0):
#   L: rho 1,   u (0.3,-0.2,0.1), p 1   -> rhoE 2.57,  u.n 0.02, c sqrt(1.4)
#   R: rho 1.2, u (0.1,0.4,-0.2), p 0.8 -> rhoE 2.126, u.n 0.38, c sqrt(1.4*0.8/1.2)
#   lambda = max(0.02 + 1.18321596, 0.38 + 0.96609178) = 1.34609178 (R side)
#   F.n(L) = (0.02, 0.606, 0.796, 0.002, 0.0714)
#   F.n(R) = (0.456, 0.5256, 0.8224, -0.0912, 1.11188)
#   U_R - U_L = (0.2, -0.18, 0.68, -0.34, -0.444)
#   H = mean(F.n) - lambda/2 (U_R - U_L)
PAIR1 = dict(L=(1.0, (0.3, -0.2, 0.1), 1.0), R=(1.2, (0.1, 0.4, -0.2), 0.8), n=(0.6, 0.8, 0.0),
             lam=1.346091783079296,
             H=(0.10339082169207041, 0.68694826047713663, 0.35152879375303939, 0.1842356031234803,
                0.89047237584360369))
# Pair 2 (2D), n = (0.28, -0.96): negative normal velocities, the L side gives lambda
#   L: rho 0.9, u (-0.5,0.6), p 1.1 -> rhoE 3.0245, u.n -0.716, c sqrt(1.4*1.1/0.9)
#   R: rho 1,   u (0.2,0.1),  p 1   -> rhoE 2.525,  u.n -0.04,  c sqrt(1.4)
#   lambda = max(0.716 + 1.30809446, 0.04 + 1.18321596) = 2.02409446 (L side)
#   F.n(L) = (-0.6444, 0.6302, -1.44264, -2.953142)
#   F.n(R) = (-0.04, 0.272, -0.964, -0.141)
#   U_R - U_L = (0.1, 0.65, -0.44, -0.4995)
PAIR2 = dict(L=(0.9, (-0.5, 0.6), 1.1), R=(1.0, (0.2, 0.1), 1.0), n=(0.28, -0.96),
             lam=2.0240944580232387,
             H=(-0.44340472290116195, -0.20673069885755258, -0.7580192192348874, -1.0415534091086958))


@pytest.mark.parametrize("pair", [PAIR1, PAIR2], ids=["3d", "2d"])
def test_lax_friedrichs_flux_hand_computed(pair):
    d = len(pair["n"])
    ns = NavierStokes(d, gamma=GAMMA, flux="lf")
    UL, UR = conserved(*pair["L"]), conserved(*pair["R"])
    n = np.array(pair["n"])
    H = ns.conv_numflux(UL, UR, n)
    assert np.allclose(H, pair["H"], rtol=0, atol=1e-14)
    # the wave speed alone: the flux of a pair with equal fluxes but different
    # states isolates lambda/2 (U_R - U_L)
    Fn = 0.5 * (np.einsum("pc,p->c", ns.conv_flux(UL), n) + np.einsum("pc,p->c", ns.conv_flux(UR), n))
    lam = (Fn - H) / (0.5 * (UR - UL))
    assert np.allclose(lam, pair["lam"], rtol=1e-13, atol=0)


def _roe_matrix(ns, UL, UR, n):
    """A = d(F^c(U).n)/dU at the Roe-averaged state (complex step), with the
    Roe averages of u and H; also returns u~.n and c~."""
    g = ns.gamma
    d = ns.d
    rL, rR = UL[0], UR[0]
    uL, uR = UL[1:1 + d] / rL, UR[1:1 + d] / rR
    pL = (g - 1) * (UL[-1] - 0.5 * rL * uL @ uL)
    pR = (g - 1) * (UR[-1] - 0.5 * rR * uR @ uR)
    HL, HR = (UL[-1] + pL) / rL, (UR[-1] + pR) / rR
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    ut = (sL * uL + sR * uR) / (sL + sR)
    Ht = (sL * HL + sR * HR) / (sL + sR)
    rt = sL * sR
    Et = (Ht + (g - 1) * 0.5 * ut @ ut) / g     # total energy per mass giving enthalpy Ht
    Ut = np.concatenate([[rt], rt * ut, [rt * Et]])
    A = np.empty((d + 2, d + 2))
    for j in range(d + 2):
        e = np.zeros(d + 2, dtype=np.complex128)
        e[j] = 1e-100j
        A[:, j] = np.imag(np.einsum("pc,p->c", ns.conv_flux(Ut + e), n)) / 1e-100
    ct = np.sqrt((g - 1) * (Ht - 0.5 * ut @ ut))
    return A, ut @ n, ct


ROE_CASES = {
    "fix-inactive": ((1.0, (0.3, -0.2, 0.1), 1.0), (1.2, (0.1, 0.4, -0.2), 0.8), (0.6, 0.8, 0.0)),
    "fix-on-contact": ((1.0, (0.01, 0.5, -0.3), 1.0), (1.05, (0.02, 0.45, -0.2), 1.02), (1.0, 0.0, 0.0)),
    "fix-on-acoustic": ((1.0, (1.15, 0.1, 0.0), 0.95), (1.01, (1.2, 0.12, 0.05), 0.97), (1.0, 0.0, 0.0)),
}


@pytest.mark.parametrize("name", list(ROE_CASES))
def test_roe_dissipation_is_the_matrix_function_of_the_roe_matrix(name):
    L, R, n = ROE_CASES[name]
    ns = NavierStokes(3, gamma=GAMMA, flux="roe", entropy_fix=0.1)
    UL, UR = conserved(*L), conserved(*R)
    n = np.array(n)
    A, unt, ct = _roe_matrix(ns, UL, UR, n)
    lam, X = np.linalg.eig(A)
    lam = np.real(lam)
    delta = 0.1 * (abs(unt) + ct)
    f = np.where(np.abs(lam) < delta, (lam ** 2 + delta ** 2) / (2 * delta), np.abs(lam))
    if name != "fix-inactive":
        assert np.any(np.abs(lam) < delta)
    else:
        assert not np.any(np.abs(lam) < delta)
    D_ref = np.real(X @ np.diag(f) @ np.linalg.inv(X)) @ (UR - UL)
    D = ns.roe_dissipation(UL, UR, n)
    assert np.linalg.norm(D - D_ref) <= 1e-12 * np.linalg.norm(D_ref)
    # and the flux is the average minus half of it
    Fn = 0.5 * (np.einsum("pc,p->c", ns.conv_flux(UL), n) + np.einsum("pc,p->c", ns.conv_flux(UR), n))
    assert np.allclose(ns.conv_numflux(UL, UR, n), Fn - 0.5 * D_ref, rtol=0, atol=1e-13)


def test_time_step_rule_and_wave_speed_hand_computed():
    # rho 1, u (3, 4, 0), p 1/1.4: |u| = 5, c = sqrt(1.4 p / rho) = 1, |u| + c = 6
    ns = NavierStokes(3, gamma=GAMMA)
    U = conserved(1.0, (3.0, 4.0, 0.0), 1.0 / 1.4)
    assert abs(ns.max_wave_speed(U) - 6.0) <= 1e-14
    # h 0.25, p = 4, CFL 100: dt = 100 * 0.25 / (9 * 6) = 25/54
    assert abs(backward_euler_dt(6.0, 0.25, 4, 100.0) - 25.0 / 54.0) <= 1e-15


def test_fd_step_of_eq_epsdef():
    # ||w|| = 8, ||v|| = 2: Delta = 1e-9 * sqrt(9) / 2 = 1.5e-9
    w = np.zeros((2, 1, 3))
    w[0, 0, 0] = 8.0
    v = np.zeros((2, 1, 3))
    v[1, 0, 2] = 2.0
    assert abs(DGOracle.fd_step(w, v) - 1.5e-9) <= 1e-24
    # the step jvp_fd takes: with R(U) = U^2 entrywise, w and v of disjoint
    # support, (R(w + D v) - R(w))/D = D v^2 exactly up to one rounding
    mesh = synth.lattice_mesh((1, 2), L=1.0)
    o = DGOracle(mesh, 0, "P", 1, NavierStokes(2))
    o.residual = lambda U, elems=None: U * U
    fd = o.jvp_fd(w, v)
    assert abs(fd[1, 0, 2] / 4.0 - 1.5e-9) <= 1e-22
    assert np.count_nonzero(fd) == 1
