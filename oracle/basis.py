"""Hierarchical modal basis on the reference hypercube.

psi_alpha(xi) = prod_i Lt_{alpha_i}(xi_i) with Lt_n = sqrt((2n+1)/2) P_n the
orthonormal Legendre polynomials.  P_k = {|alpha|_1 <= k} (total degree, the
paper's broken space of Sec. 2.1); Q_k = {max alpha_i <= k}.

Ordering: ascending total degree; inside one degree, descending alpha_1, then
descending alpha_2.  The first dim(P_k') functions then span P_k' for every
k' <= k, so restriction to a coarser p-level keeps leading modes (Sec. 2.4.1).
"""
from math import comb

import numpy as np


def basis_size(k, d, space="P"):
    return comb(k + d, d) if space == "P" else (k + 1) ** d


def multi_indices(k, d, space="P"):
    import itertools
    alphas = [a for a in itertools.product(range(k + 1), repeat=d)
              if (sum(a) <= k if space == "P" else max(a) <= k)]
    alphas.sort(key=lambda a: (sum(a),) + tuple(-ai for ai in a))
    return np.array(alphas, dtype=np.int64).reshape(-1, d)


def legendre_orthonormal(kmax, x):
    """Values and derivatives of Lt_0..Lt_kmax at x: arrays [kmax+1, *x.shape]."""
    x = np.asarray(x, dtype=np.float64)
    P = np.zeros((kmax + 1,) + x.shape)
    dP = np.zeros_like(P)
    P[0] = 1.0
    if kmax >= 1:
        P[1] = x
        dP[1] = 1.0
    for n in range(1, kmax):
        # Bonnet recursion and P'_{n+1} = P'_{n-1} + (2n+1) P_n
        P[n + 1] = ((2 * n + 1) * x * P[n] - n * P[n - 1]) / (n + 1)
        dP[n + 1] = dP[n - 1] + (2 * n + 1) * P[n]
    s = np.sqrt((2 * np.arange(kmax + 1) + 1) / 2.0).reshape((-1,) + (1,) * x.ndim)
    return s * P, s * dP


def eval_basis(alphas, xi):
    """psi [Q, Nb] and reference gradient dpsi [Q, Nb, d] at points xi [Q, d]."""
    xi = np.atleast_2d(np.asarray(xi, dtype=np.float64))
    q, d = xi.shape
    kmax = int(alphas.max()) if alphas.size else 0
    L = np.empty((d, kmax + 1, q))
    dL = np.empty((d, kmax + 1, q))
    for i in range(d):
        L[i], dL[i] = legendre_orthonormal(kmax, xi[:, i])
    nb = len(alphas)
    psi = np.ones((q, nb))
    dpsi = np.ones((q, nb, d))
    for b, a in enumerate(alphas):
        for i in range(d):
            psi[:, b] *= L[i, a[i]]
            for j in range(d):
                dpsi[:, b, j] *= dL[i, a[i]] if i == j else L[i, a[i]]
    return psi, dpsi
