"""Rosenbrock (linearly implicit Runge-Kutta) time step (Sec. 2.2, Alg. ros)
-- FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For M dw/dt + R(w) = 0 (M = I with the orthonormal modal basis, restricted
to the velocities for the incompressible equations), one step from w^n of
size dt with n_s stages:

    for s = 1..n_s:
        dp = sum_{o<s} a[s][o] dw_o,   dq = sum_{o<s} c[s][o] dw_o
        (M/(gamma dt) + J(w^n)) dw_s = -R(w^n + dp) - M dq/dt
    w^{n+1} = w^n + sum_s m[s] dw_s

The Jacobian (and any preconditioner) is that of w^n for every stage.  The
last loop of the printed algorithm assigns inside a loop over the stages; the
sum above is the reading taken.  The scheme the paper uses (ROSI2PW) is
cited but its coefficients are not in the text, so the coefficient sets here
are the one-stage linearly implicit Euler method and ROS2 (Verwer, Spee,
Blom, Hundsdorfer 1999), rewritten in the form above.
"""
import numpy as np


def step(residual, solve, w, dt, gamma, a, c, m, mass=None):
    """One step.  residual(x) -> R(x); solve(rhs) -> (M/(gamma dt) + J(w^n))^-1 rhs.
    a, c: n_s x n_s (strictly lower parts used), m: n_s.  Flat FP64 arrays.
    mass: the diagonal of M (flat, default identity); the dq/dt term of the
    stage right-hand side is M dq / dt (eq. rossys)."""
    w = np.asarray(w, dtype=np.float64)
    dws = []
    for s in range(len(m)):
        dp = np.zeros_like(w)
        dq = np.zeros_like(w)
        for o in range(s):
            dp += a[s][o] * dws[o]
            dq += c[s][o] * dws[o]
        dws.append(solve(-residual(w + dp) - (dq if mass is None else mass * dq) / dt))
    out = w.copy()
    for s in range(len(m)):
        out += m[s] * dws[s]
    return out


def linear_implicit_euler():
    """One stage, gamma = 1: (I/dt + J) dw = -R(w^n), w^{n+1} = w^n + dw."""
    return dict(gamma=1.0, a=[[0.0]], c=[[0.0]], m=[1.0])


def ros2():
    """ROS2: with k-stages (I - gamma h J_f) k1 = f(y), (I - gamma h J_f) k2 =
    f(y + h k1) - 2 k1, y+ = y + 3/2 h k1 + 1/2 h k2, gamma = 1 + 1/sqrt(2)
    (f = -R, J_f = -J).  With dw_s = gamma h k_s the stages become the form
    of Alg. ros with a21 = 1/gamma, c21 = 2/gamma, m = (3/(2 gamma), 1/(2 gamma))."""
    g = 1.0 + 1.0 / np.sqrt(2.0)
    return dict(gamma=g, a=[[0.0, 0.0], [1.0 / g, 0.0]], c=[[0.0, 0.0], [2.0 / g, 0.0]],
                m=[1.5 / g, 0.5 / g])


def dg_step(o, U, dt, coeffs, lstsq=False):
    """One step of the oracle DG discretisation (U[e, c, b]) with dense solves
    of the stage systems (small meshes only).  lstsq: minimum-norm solutions
    (for singular consistent stage systems, e.g. the incompressible equations
    on a periodic mesh, whose pressure level is free)."""
    shift = 1.0 / (coeffs["gamma"] * dt)
    n = U.size
    G = np.zeros((n, n))
    for j in range(n):
        V = np.zeros(n)
        V[j] = 1.0
        G[:, j] = o.operator(U, V.reshape(U.shape), shift).reshape(-1)
    res = lambda x: o.residual(x.reshape(U.shape)).reshape(-1)
    mass = np.broadcast_to(o.mass()[None, :, None], U.shape).reshape(-1)
    solve = (lambda r: np.linalg.lstsq(G, r, rcond=None)[0]) if lstsq else (lambda r: np.linalg.solve(G, r))
    out = step(res, solve, U.reshape(-1), dt, coeffs["gamma"], coeffs["a"], coeffs["c"], coeffs["m"], mass=mass)
    return out.reshape(U.shape)
