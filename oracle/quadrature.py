"""Gauss-Legendre rules (parity pinned: exactness on monomials, weight sums).

The paper integrates with Gauss rules and ignores the mapping degree when
choosing them (Sec. 3.2, sphere case); one tensor rule of nq points per
direction is used on volumes and the (d-1)-dimensional tensor rule on faces.
"""
import numpy as np


def gauss_legendre(nq):
    """Nodes and weights of the nq-point Gauss-Legendre rule on [-1, 1]."""
    x, w = np.polynomial.legendre.leggauss(int(nq))
    return x.astype(np.float64), w.astype(np.float64)


def tensor_rule(nq, d):
    """Tensor Gauss rule on [-1,1]^d; the first coordinate varies fastest.

    Returns points [nq^d, d] and weights [nq^d].  d = 0 gives one point of
    weight 1 (the face rule of a 1D element).
    """
    x, w = gauss_legendre(nq)
    if d == 0:
        return np.zeros((1, 0)), np.ones(1)
    grids = np.meshgrid(*([np.arange(nq)] * d), indexing="ij")
    idx = [g.reshape(-1) for g in grids[::-1]]  # idx[0] fastest
    pts = np.stack([x[i] for i in idx], axis=-1)
    wts = np.prod(np.stack([w[i] for i in idx], axis=-1), axis=-1)
    return pts, wts
