"""The instrumented pointwise flop count (oracle.flops) behind the roofline
figures: the counting type counts by its stated cost table (hand-counted
expressions and the 3D convective flux counted by hand), its tangent is the
exact directional derivative (equal to the complex-step derivative of the
same physics), and the stored table tests/golden/pointwise_flops.json is the
one the script writes from the oracle."""
import json
import os

import numpy as np

from oracle.flops import Num, Tally, _count, _nums, pointwise_flops
from oracle.physics import NavierStokes

HERE = os.path.dirname(os.path.abspath(__file__))


def test_cost_table_on_hand_counted_expressions():
    a, b, c, d = Num(1.5, 0.1), Num(2.0, -0.3), Num(0.5, 0.2), Num(3.0, 0.7)
    assert _count(lambda: (a * b + c) / d) == 4 + 2 + 4
    av, bv, cv, dv = Num(1.5), Num(2.0), Num(0.5), Num(3.0)
    assert _count(lambda: (av * bv + cv) / dv) == 3
    assert _count(lambda: a * 2.0 + 0.0) == 2          # product with a constant; adding 0 is free
    assert _count(lambda: 1.0 * a - a * -1.0) == 2      # products with +-1 are free, the sum is not
    assert _count(lambda: a.sqrt()) == 3 and _count(lambda: av.sqrt()) == 1


def test_convective_flux_counted_by_hand():
    # primitives: u = m/rho (3), |m.u| (3 mul + 2 add), p = (g-1)(rE - 0.5 .) (3): 11;
    # per direction P: rho u_P (1), rho u_P u_j (2 x 3), + p (1), u_P (rE + p) (2): 10
    ns = NavierStokes(3)
    u = _nums(np.array([1.1, 0.2, -0.3, 0.1, 2.6]), None)
    assert _count(lambda: ns.conv_flux(u)) == 11 + 3 * 10


def test_counted_tangent_is_the_exact_derivative():
    ns = NavierStokes(3, mu=1e-2)
    rng = np.random.default_rng(3)
    u0 = np.array([1.1, 0.2, -0.3, 0.1, 2.6])
    G0 = 0.1 * rng.standard_normal((5, 3))
    du, dG = rng.standard_normal(5), rng.standard_normal((5, 3))
    F = ns.conv_flux(_nums(u0, du)) - ns.visc_flux(_nums(u0, du), _nums(G0, dG))
    tan = np.vectorize(lambda x: x.t)(F)[0]
    h = 1e-100
    ref = np.imag(ns.conv_flux((u0 + 1j * h * du)[None]) - ns.visc_flux((u0 + 1j * h * du)[None],
                                                                         (G0 + 1j * h * dG)[None]))[0] / h
    assert np.allclose(tan, ref, rtol=1e-13, atol=1e-15)


def test_stored_table_matches_the_oracle():
    stored = json.load(open(os.path.join(HERE, "golden", "pointwise_flops.json")))["counts"]
    for flux in ("roe", "lf"):
        for d in (2, 3):
            assert stored[flux][str(d)] == pointwise_flops(d, flux)
