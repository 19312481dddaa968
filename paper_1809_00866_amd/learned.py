"""Training workflow of the learned element-local preconditioner.

Every numerical step runs in the library (backward-Euler steps, target
solves, features, Adam steps); this module only sequences the calls and
samples minibatch rows.

Data (one linearisation per snapshot of a backward-Euler trajectory): input
vectors r = R(w) and the next terms of the block-Jacobi-preconditioned
Krylov sequence (G D^-1)^k r, which span the Arnoldi vectors that FGMRES with
block Jacobi hands to its preconditioner; targets z solve G z = r to a
relative 1e-6 (p-multigrid FGMRES); every element of every (r, z) pair is
one training pair.  In the block-Jacobi correction mode the target of
element K is (z_K - D_K^-1 r_K) / s_K.  Features and targets are normalised
per element, so the vectors need no scaling.
"""
import numpy as np
import torch


def time_step(g, w, cfl, order, h):
    """shift = 1/dt with dt = CFL h / ((2p+1) max(|u| + c))."""
    dt = cfl * h / ((2 * order + 1) * g.max_wave_speed(w))
    return 1.0 / dt


def mg_levels(order):
    """Degrees and smoothing counts of the V-cycle used for data generation."""
    orders = [order] + [k for k in (2, 1) if k < order]
    if len(orders) == 1:
        orders.append(0)
    return orders, [8] * (len(orders) - 1) + [40]


def _setup(g, w, shift):
    orders, its = mg_levels(g.order)
    g.mg_setup(w, shift, orders, its)


def trajectory(g, w0, n_steps, cfl, order, h, rtol=1e-8):
    """States after 0..n_steps linearised backward-Euler steps (one-stage
    Rosenbrock steps of the library, p-multigrid preconditioned)."""
    from .schemes import LINEAR_IMPLICIT_EULER
    states = [w0.clone()]
    w = w0.clone()
    for _ in range(n_steps):
        shift = time_step(g, w, cfl, order, h)
        _setup(g, w, shift)
        w, st = g.rosenbrock_step(w, 1.0 / shift, LINEAR_IMPLICIT_EULER, rtol=rtol, max_iter=500, precond="mg")
        if not st["converged"]:
            raise RuntimeError(f"trajectory step did not converge: {st}")
        states.append(w.clone())
    return states


def pairs(g, w, shift, rtol=1e-6, n_krylov=2, n_random=0, seed=0):
    """(X, T) training pairs of one linearisation: r = -R(w), n_krylov terms
    (G D^-1)^k r of the block-Jacobi-preconditioned Krylov sequence and
    optionally n_random seeded Gaussian vectors."""
    r0 = g.residual(w)                   # the sign of a pair (r, G^-1 r) is immaterial
    _setup(g, w, shift)                  # also the fine block-Jacobi factors at (w, shift)
    vecs = [r0]
    v = r0
    for _ in range(n_krylov):
        v = g.jvp(w, g.block_apply(v), shift=shift)
        vecs.append(v)
    gen = torch.Generator(device=r0.device)
    gen.manual_seed(seed)
    for _ in range(n_random):
        vecs.append(torch.randn(r0.shape, generator=gen, device=r0.device, dtype=r0.dtype))
    Xs, Ts = [], []
    for r in vecs:
        z, _ = g.fgmres(w, shift, r, rtol=rtol, max_iter=500, precond="mg")
        X, T, _ = g.mlp_features(w, r, z)
        Xs.append(X)
        Ts.append(T)
    return torch.cat(Xs), torch.cat(Ts)


def train(g, X, T, steps, batch=1024, lr=1e-3, seed=0):
    """Adam steps on random minibatches (rows drawn with a seeded generator);
    returns the loss history (one value per step, read back at the end)."""
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    losses = torch.empty(steps, dtype=torch.float32, device=X.device)
    n = X.shape[0]
    for k in range(steps):
        rows = torch.randint(0, n, (batch,), generator=gen, device=X.device, dtype=torch.int64)
        g.mlp_train_step(X, T, rows, lr=lr, loss=losses[k:k + 1])
    return losses.cpu().numpy()


def validation_loss(g, X, T, chunk=65536):
    """Mean squared error of the current network over (X, T) (the library's
    loss, chunk by chunk)."""
    tot, n = 0.0, X.shape[0]
    for s in range(0, n, chunk):
        _, loss = g.mlp_grad(X[s:s + chunk].contiguous(), T[s:s + chunk].contiguous())
        tot += loss.item() * min(chunk, n - s)
    return tot / n
