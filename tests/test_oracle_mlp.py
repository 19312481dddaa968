"""Pins for the oracle's learned preconditioner (oracle/mlp.py): BF16 rounding
against torch's own conversion and hand-checked ties, gradients against
central finite differences of the FP64 loss, Adam's closed-form first step,
positive homogeneity, and cell means against closed forms."""
import numpy as np
import pytest

import synth
from oracle import DGOracle, NavierStokes
from oracle.mlp import adam_step, apply, bf16_round, cell_means, features, forward, loss_and_grad, n_params, sizes
from synth import mlp_init_weights


def init_params(n_in, n_out, seed):
    return mlp_init_weights(n_in, n_out, seed).astype(np.float64)


def test_bf16_rounding_ties_to_even_and_matches_torch():
    torch = pytest.importorskip("torch")
    assert bf16_round(1.0 + 2.0 ** -8) == 1.0                      # tie -> even (1.0)
    assert bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6      # tie -> even (mantissa 2)
    assert bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert bf16_round(-3.0) == -3.0 and bf16_round(0.0) == 0.0
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32) * 10.0 ** np.random.default_rng(1).integers(
        -8, 8, 10000)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(bf16_round(x), ref)


def test_parameter_count_of_the_p3_network():
    n_in, _, n_out = sizes(5, 20, 6)
    assert (n_in, n_out) == (130, 100)
    assert n_params(n_in, n_out) == 125028


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    n_in, n_out, B = 14, 6, 9
    # a narrower network is enough to pin the formulas; HIDDEN layers are fixed at 256
    theta = init_params(n_in, n_out, seed=4) + 0.01 * rng.standard_normal(n_params(n_in, n_out))
    X = rng.standard_normal((B, n_in))
    T = rng.standard_normal((B, n_out))
    L, g = loss_and_grad(theta, X, T, rounding=False)
    idx = rng.choice(theta.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (loss_and_grad(theta + e, X, T, rounding=False)[0] - loss_and_grad(theta - e, X, T, rounding=False)[0]) / (
            2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, np.abs(g).max()), (i, fd, g[i])


def test_adam_first_step_is_a_signed_learning_rate_step():
    g = np.array([3.0, -2e-3, 0.5])
    th, m, v = adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), t=1, lr=1e-3, eps=1e-8)
    assert np.allclose(th, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_training_reduces_the_loss_on_a_fixed_batch():
    rng = np.random.default_rng(5)
    n_in, n_out = 10, 4
    theta = init_params(n_in, n_out, seed=6)
    X = rng.standard_normal((64, n_in))
    T = np.tanh(X[:, :n_out])
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    L0 = loss_and_grad(theta, X, T)[0]
    for t in range(1, 51):
        L, g = loss_and_grad(theta, X, T)
        theta, m, v = adam_step(theta, g, m, v, t)
    assert L < 0.5 * L0


def _case():
    mesh = synth.lattice_mesh((2, 3, 2), L=1.0)
    o = DGOracle(mesh, 2, "P", 3, NavierStokes(3, mu=1e-2))
    U = o.project(synth.TaylorGreenStandIn(seed=9, L=1.0))
    return o, U


def test_cell_means_equal_the_first_mode_over_sqrt_volume_and_a_linear_field_centroid():
    o, U = _case()
    mean = cell_means(o, U)
    vol = o.element_volumes()
    assert np.allclose(mean, U[:, :, 0] / np.sqrt(vol)[:, None], rtol=1e-13, atol=1e-13)
    # the mean of a linear field is its value at the centroid
    lin = lambda x: np.stack([1.0 + x[..., 0] + 2 * x[..., 1] - x[..., 2]] * o.nvar, axis=-1)
    Ul = o.project(lin)
    cen = np.asarray(synth.lattice_mesh((2, 3, 2), L=1.0)["elem_xyz"]).mean(axis=1)
    assert np.allclose(cell_means(o, Ul)[:, 0], 1.0 + cen[:, 0] + 2 * cen[:, 1] - cen[:, 2], rtol=0, atol=1e-13)


def test_features_layout_and_positive_homogeneity():
    o, U = _case()
    R = np.random.default_rng(7).standard_normal(U.shape)
    X, s = features(o, U, R)
    n_in, _, n_out = sizes(o.nvar, o.nb, 2 * o.d)
    assert X.shape == (o.ne, n_in)
    assert np.allclose(X[:, :n_out] * s[:, None], R.reshape(o.ne, -1), rtol=1e-15, atol=0)
    Uc = np.zeros_like(U)
    Uc[:, :, 0] = np.array([1.0, 0.5, -0.25, 2.0, 7.0]) * np.sqrt(o.element_volumes())[:, None]
    Xc, _ = features(o, Uc, R)
    assert np.allclose(Xc[:, n_out:].reshape(o.ne, 2 * o.d, o.nvar), np.sign([1.0, 0.5, -0.25, 2.0, 7.0]),
                       rtol=1e-13, atol=0)
    theta = init_params(n_in, n_out, seed=8)
    z1 = apply(o, theta, U, R)
    z4 = apply(o, theta, U, 4.0 * R)
    assert np.array_equal(z4, 4.0 * z1)
    y, _ = forward(theta, X, n_out)
    assert np.allclose(z1.reshape(o.ne, -1), s[:, None] * y, rtol=1e-15, atol=0)
