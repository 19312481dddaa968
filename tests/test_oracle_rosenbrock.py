"""Pins for the oracle's Rosenbrock step (oracle/rosenbrock.py, Sec. 2.2 Alg. ros):
the transformed ROS2 coefficients against an independent k-stage
implementation of ROS2, the orders of accuracy of ROS2 and of the linearly
implicit Euler method on a nonlinear ODE with a fine reference solution, and
conservation of the element means by a DG step on a periodic mesh."""
import numpy as np

import synth
from oracle import DGOracle, NavierStokes
from oracle import rosenbrock as ros

F = lambda y: np.array([-y[0] ** 2 + np.sin(y[1]), -0.5 * y[1] * y[0]])
JF = lambda y: np.array([[-2 * y[0], np.cos(y[1])], [-0.5 * y[1], -0.5 * y[0]]])
Y0 = np.array([1.0, 0.5])


def _ros_step(y, h, coeffs):
    # dy/dt = F(y) is M dy/dt + R(y) = 0 with R = -F, J = -JF
    A = np.eye(2) / (coeffs["gamma"] * h) - JF(y)
    return ros.step(lambda x: -F(x), lambda r: np.linalg.solve(A, r), y, h, coeffs["gamma"], coeffs["a"],
                    coeffs["c"], coeffs["m"])


def _ros2_kform(y, h):
    g = 1 + 1 / np.sqrt(2)
    A = np.eye(2) - g * h * JF(y)
    k1 = np.linalg.solve(A, F(y))
    k2 = np.linalg.solve(A, F(y + h * k1) - 2 * k1)
    return y + 1.5 * h * k1 + 0.5 * h * k2


def _rk4(y, T, n):
    h = T / n
    for _ in range(n):
        a = F(y)
        b = F(y + h / 2 * a)
        c = F(y + h / 2 * b)
        d = F(y + h * c)
        y = y + h / 6 * (a + 2 * b + 2 * c + d)
    return y


def test_transformed_ros2_equals_the_k_stage_form():
    y = Y0.copy()
    for h in (0.3, 0.05, 1e-3):
        assert np.allclose(_ros_step(y, h, ros.ros2()), _ros2_kform(y, h), rtol=1e-13, atol=1e-15)


def test_orders_of_accuracy():
    ref = _rk4(Y0, 1.0, 20000)
    for coeffs, order in ((ros.ros2(), 2), (ros.linear_implicit_euler(), 1)):
        errs = []
        for n in (20, 40, 80):
            y = Y0.copy()
            for _ in range(n):
                y = _ros_step(y, 1.0 / n, coeffs)
            errs.append(np.linalg.norm(y - ref))
        ratios = [errs[i] / errs[i + 1] for i in range(2)]
        assert all(abs(np.log2(r) - order) < 0.2 for r in ratios), (order, ratios)


def test_dg_step_conserves_the_element_means_on_a_periodic_mesh():
    mesh = synth.lattice_mesh((2, 1, 2), L=1.0)
    o = DGOracle(mesh, 1, "P", 2, NavierStokes(3, mu=1e-2))
    U = o.project(synth.TaylorGreenStandIn(seed=3, L=1.0))
    for coeffs in (ros.linear_implicit_euler(), ros.ros2()):
        U1 = ros.dg_step(o, U, 0.05, coeffs)
        assert np.linalg.norm(U1 - U) > 1e-6 * np.linalg.norm(U)
        tot0, tot1 = U[:, :, 0].sum(axis=0), U1[:, :, 0].sum(axis=0)
        assert np.allclose(tot1, tot0, rtol=1e-12, atol=1e-12 * np.abs(tot0).max())
