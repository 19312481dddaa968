"""Seeded initial weights of the learned preconditioner's network (an input,
like the other seeded data; no preconditioner arithmetic here).

Flat FP32 layout: W1 [256 x n_in], b1 [256], W2 [256 x 256], b2 [256],
W3 [n_out x 256], b3 [n_out]; He-uniform weights U(-sqrt(6/fan_in),
sqrt(6/fan_in)), zero biases.
"""
import numpy as np

HIDDEN = 256


def mlp_init_weights(n_in, n_out, seed):
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in [(HIDDEN, n_in), (HIDDEN, HIDDEN), (n_out, HIDDEN)]:
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)
