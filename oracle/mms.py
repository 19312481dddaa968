"""Manufactured solutions for the oracle's convergence pin.

For a smooth periodic field U*(x) the steady problem
    sigma*U + div(F^c(U) - F^v(U, grad U)) = s,
    s = sigma*U* + sum_p d/dx_p F_p(U*(x), grad U*(x))
has U* as exact solution.  The source is evaluated pointwise: the x_p
derivative of F_p along (dU*/dx_p, d(grad U*)/dx_p) is a directional
derivative of the flux function, taken by complex step (exact to round-off).
The discrete problem sigma*U_h + R(U_h) = S_h (S_h the L2 projection of s) is
solved by Newton's method with a sparse Jacobian assembled column by column
by complex-step probing with a distance-2 colouring of the element graph.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def source(phys, field, x, sigma=0.0, h=1e-100):
    U = field.value(x)
    dU = field.grad(x)       # [..., n, d]
    H = field.hess(x)        # [..., n, d, d]
    s = sigma * U
    for p in range(phys.d):
        Uc = U + 1j * h * dU[..., p]
        Gc = dU + 1j * h * H[..., p]
        F = phys.conv_flux(Uc) - phys.visc_flux(Uc, Gc)
        s = s + np.imag(F[..., p, :]) / h
    return s


def distance2_coloring(o):
    nbhd = [set([e]) | set(o.nbr[e].tolist()) for e in range(o.ne)]
    color = np.full(o.ne, -1)
    for e in range(o.ne):
        ring = set()
        for k in nbhd[e]:
            ring |= nbhd[k]
        used = {color[k] for k in ring if color[k] >= 0}
        c = 0
        while c in used:
            c += 1
        color[e] = c
    return color, nbhd


def sparse_jacobian(o, U, shift=0.0, h=1e-100):
    """Assembled (shift*I + dR/dU) in the oracle's flat element-major order (e, c, b)."""
    color, nbhd = distance2_coloring(o)
    m = o.nvar * o.nb
    rows, cols, vals = [], [], []
    for c in range(color.max() + 1):
        members = np.nonzero(color == c)[0]
        for l in range(m):
            V = np.zeros(U.shape)
            V[members, l // o.nb, l % o.nb] = 1.0
            Jv = np.imag(o.residual(U.astype(np.complex128) + 1j * h * V)) / h
            for j in members:
                col = j * m + l
                for i in nbhd[j]:
                    blk = Jv[i].reshape(-1)
                    nz = np.nonzero(blk)[0]
                    rows.append(i * m + nz)
                    cols.append(np.full(len(nz), col))
                    vals.append(blk[nz])
    n = o.ne * m
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    if shift:
        A = A + shift * sp.identity(n, format="csr")
    return A


def solve_mms(o, field, sigma=0.0, newton_tol=1e-11, max_newton=8):
    """Newton solve of sigma*U + R(U) = S_h from the projection of U*."""
    S = o.project(lambda x: source(o.phys, field, x, sigma))
    U = o.project(field.value)
    for _ in range(max_newton):
        F = sigma * U + o.residual(U) - S
        fn = np.linalg.norm(F)
        if fn <= newton_tol * max(1.0, np.linalg.norm(S)):
            break
        A = sparse_jacobian(o, U, shift=sigma)
        dU = spla.spsolve(A.tocsc(), -F.reshape(-1))
        U = U + dU.reshape(U.shape)
    return U


def l2_error(o, U, field, nq_fine=None):
    """||u_h - U*||_{L2} with a (finer) tensor Gauss rule on every element."""
    from .quadrature import tensor_rule
    nqf = nq_fine or (o.nq1d + 3)
    xi, w = tensor_rule(nqf, o.d)
    x, uh, det = o.evaluate(U, xi)
    err = uh - field.value(x)
    return float(np.sqrt(np.einsum("q,eq,eqc->", w, det, err * err)))
