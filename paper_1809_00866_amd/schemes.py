"""Rosenbrock coefficient sets in the form of Alg. ros (Sec. 2.2):
(I/(gamma dt) + J) dw_s = -R(w + sum a[s][o] dw_o) - (1/dt) sum c[s][o] dw_o,
w_next = w + sum m[s] dw_s.  The paper's scheme (ROSI2PW) is cited without
its coefficients."""
import math

# one stage: the linearised backward Euler step
LINEAR_IMPLICIT_EULER = {"gamma": 1.0, "a": [[0.0]], "c": [[0.0]], "m": [1.0]}

# ROS2 (second order, L-stable; Verwer, Spee, Blom and Hundsdorfer 1999), whose
# stages k_1, k_2 with (I - g h J_f) k_1 = f(y), (I - g h J_f) k_2 = f(y + h k_1) - 2 k_1
# and y_next = y + h (3 k_1 + k_2) / 2 become dw_s = g h k_s in the form above
_G = 1.0 + 1.0 / math.sqrt(2.0)
ROS2 = {"gamma": _G, "a": [[0.0, 0.0], [1.0 / _G, 0.0]], "c": [[0.0, 0.0], [2.0 / _G, 0.0]],
        "m": [1.5 / _G, 0.5 / _G]}
