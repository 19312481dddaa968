"""Krylov solver, block-Jacobi solve and time-step helpers (FP64 oracle).

fgmres: flexible GMRES(m) with right preconditioning (the outer solver of
Sec. 2.5, which needs the preconditioned vectors z_j stored because the
preconditioner may change between iterations).  Classical Gram-Schmidt with
re-orthogonalisation (two passes), Givens rotations on the Hessenberg matrix,
restart from the true residual, x0 = 0 by default.  Convergence is declared on
the true unpreconditioned residual ||b - A x|| <= rtol ||b||.  Also reports the
convergence factor rho = exp(ln(||d_N||/||d_0||)/N) of App. B.
"""
import numpy as np


def fgmres(apply_A, b, apply_M=None, x0=None, restart=30, rtol=1e-8, max_iter=1000,
           breakdown_tol=1e-14, orth="cgs2"):
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    M = (lambda v: v.copy()) if apply_M is None else apply_M
    bnorm = np.linalg.norm(b)
    info = dict(iters=0, restarts=0, converged=False, history=[], rel_res_true=0.0, rho=0.0)
    if bnorm == 0.0:
        x[:] = 0.0
        info["converged"] = True
        return x, info
    r = b - apply_A(x) if np.any(x) else b.copy()
    beta = np.linalg.norm(r)
    d0 = beta
    while True:
        if beta <= rtol * bnorm:
            info["converged"] = True
            break
        if info["iters"] >= max_iter:
            break
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = M(V[j])
            w = apply_A(Z[j])
            w0 = np.linalg.norm(w)
            if orth == "mgs":                 # modified Gram-Schmidt: one vector at a time
                h = np.zeros(j + 1)
                for i in range(j + 1):
                    h[i] = V[i] @ w
                    w = w - h[i] * V[i]
            else:                             # classical Gram-Schmidt, one re-orthogonalisation
                h = V[:j + 1] @ w
                w = w - V[:j + 1].T @ h
                h2 = V[:j + 1] @ w
                w = w - V[:j + 1].T @ h2
                h = h + h2
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):  # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            info["iters"] += 1
            info["history"].append(abs(g[j + 1]))
            if abs(g[j + 1]) <= rtol * bnorm or hn <= breakdown_tol * w0 or info["iters"] >= max_iter:
                break
            V[j + 1] = w / hn
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + Z[:k].T @ y
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        info["restarts"] += 1
    info["rel_res_true"] = beta / bnorm
    if info["iters"] > 0 and beta > 0:
        info["rho"] = float(np.exp(np.log(beta / d0) / info["iters"]))
    return x, info


def block_solve(D, r):
    """z_K = D_K^{-1} r_K for stacked blocks D[E, m, m], r[E, m] (LU, partial pivoting)."""
    return np.linalg.solve(D, r[..., None])[..., 0]


def backward_euler_dt(max_speed, h, order, cfl):
    """dt = CFL * h / ((2p+1) * max(|u| + c)) (the step rule used for the implicit workloads)."""
    return cfl * h / ((2 * order + 1) * max_speed)
