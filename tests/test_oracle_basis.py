"""Pins for the oracle's quadrature and modal basis (closed forms, printed counts)."""
import json
import os
from math import comb

import numpy as np
import pytest

from oracle import basis_size, eval_basis, gauss_legendre, legendre_orthonormal, multi_indices, tensor_rule

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")


@pytest.mark.parametrize("nq", [1, 2, 3, 4, 5, 6])
def test_gauss_rule_exact_to_degree_2nq_minus_1(nq):
    x, w = gauss_legendre(nq)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(2 * nq):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-14
    # and not exact one degree higher (nq >= 1): x^(2nq) integrates wrongly
    k = 2 * nq
    assert abs(np.sum(w * x ** k) - 2.0 / (k + 1)) > 1e-6


@pytest.mark.parametrize("d,nq", [(2, 4), (3, 4), (3, 5), (3, 2)])
def test_tensor_rule_monomials(d, nq):
    pts, w = tensor_rule(nq, d)
    assert abs(w.sum() - 2.0 ** d) < 1e-13
    rng = np.random.default_rng(0)
    for _ in range(20):
        a = rng.integers(0, 2 * nq, size=d)
        exact = np.prod([0.0 if ai % 2 else 2.0 / (ai + 1) for ai in a])
        got = np.sum(w * np.prod(pts ** a, axis=1))
        assert abs(got - exact) < 1e-13


def test_legendre_closed_forms():
    x = np.linspace(-1, 1, 11)
    L, dL = legendre_orthonormal(3, x)
    P = [np.ones_like(x), x, 0.5 * (3 * x ** 2 - 1), 0.5 * (5 * x ** 3 - 3 * x)]
    dP = [np.zeros_like(x), np.ones_like(x), 3 * x, 0.5 * (15 * x ** 2 - 3)]
    for n in range(4):
        s = np.sqrt((2 * n + 1) / 2)
        assert np.allclose(L[n], s * P[n], atol=1e-15)
        assert np.allclose(dL[n], s * dP[n], atol=1e-14)


@pytest.mark.parametrize("k,d,space,n", [(3, 3, "P", 20), (4, 3, "P", 35), (2, 3, "P", 10), (1, 3, "P", 4),
                                         (6, 3, "P", 84), (2, 2, "Q", 9), (2, 2, "P", 6)])
def test_basis_sizes(k, d, space, n):
    assert basis_size(k, d, space) == n
    assert len(multi_indices(k, d, space)) == n


def test_paper_printed_counts():
    items = json.load(open(GOLDEN))["items"]
    rlg = items[0]
    assert rlg["elements"] * basis_size(rlg["order"], rlg["dim"]) == rlg["dofs_per_variable"]
    for it in items[1:]:
        ratio = (basis_size(it["k_fine"], it["dim"]) / basis_size(it["k_coarse"], it["dim"])) ** 2
        assert abs(ratio - it["printed_ratio"]) / it["printed_ratio"] < 0.01


@pytest.mark.parametrize("d", [2, 3])
def test_hierarchical_ordering(d):
    """The leading dim P_k' functions of P_k are exactly P_k' (restriction = truncation)."""
    for k in range(1, 5):
        full = [tuple(a) for a in multi_indices(k, d)]
        for kc in range(k):
            lead = full[:comb(kc + d, d)]
            assert sorted(lead) == sorted(tuple(a) for a in multi_indices(kc, d))
            assert all(sum(a) <= kc for a in lead)
    # ordering inside one degree: descending alpha_1, then alpha_2
    a = [tuple(x) for x in multi_indices(2, 3)]
    assert a == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0), (1, 0, 1),
                 (0, 2, 0), (0, 1, 1), (0, 0, 2)]


@pytest.mark.parametrize("k,d,space,nq", [(3, 3, "P", 4), (4, 3, "P", 5), (2, 2, "Q", 4), (1, 3, "P", 2)])
def test_discrete_orthonormality_degree_2p(k, d, space, nq):
    """Products psi_a*psi_b have degree <= 2p per direction: integrated exactly -> identity."""
    al = multi_indices(k, d, space)
    pts, w = tensor_rule(nq, d)
    psi, dpsi = eval_basis(al, pts)
    G = psi.T @ (w[:, None] * psi)
    assert np.abs(G - np.eye(len(al))).max() < 1e-13
    # reference gradients against a finite difference of psi
    h = 1e-6
    for j in range(d):
        e = np.zeros(d)
        e[j] = h
        fd = (eval_basis(al, pts + e)[0] - eval_basis(al, pts - e)[0]) / (2 * h)
        assert np.abs(fd - dpsi[:, :, j]).max() < 1e-7
