"""p-multigrid V-cycle preconditioner (Sec. 2.4) -- FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Levels l = 0 (fine, degree k_0), 1, ..., L (coarsest), k_0 > k_1 > ... > k_L.
With the hierarchical orthonormal modal basis of the fine discretisation
(Sec. 2.4.1, 2.4.2):

* restriction I_l^{l+1} (the L2 projection onto P^{k_{l+1}}) keeps the first
  N_b(k_{l+1}) modes of every variable and discards the rest;
* prolongation I_{l+1}^l (the injection) pads the missing modes with zeros;
* the inherited coarse operator G_l = I_0^l G_0 I_l^0 (eq. GalProj; the
  projection matrices are unit-diagonal rectangular) keeps the leading
  sub-block of every diagonal and off-diagonal block of the fine operator;
  it is formed here column by column from the fine operator itself;
* SMOOTH(G_l, g, x0) is a fixed number of GMRES iterations (one cycle, no
  restart), right-preconditioned by element-wise block Jacobi of G_l; the
  coarsest-level SOLVE is the same smoother from x0 = 0 with its own count;
* Alg. vcic: pre-smoothing, coarse-grid correction of the defect,
  post-smoothing; called on the fine level with a zero initial guess, it is
  the (nonlinear, hence flexible-GMRES) preconditioner of the outer solve;
* Alg. fullvcic (the full cycle): the right-hand side is restricted to the
  next level, solved there by the full cycle, prolonged as the initial
  iterate, and corrected by one V-cycle on the defect.  The full cycle runs as
  the algorithm lists it: its V-cycle correction smooths the level twice (the
  text's count of one fine smoothing per full cycle is not what the listing
  does).

Arrays use the oracle layout X[e, c, b]; level l has N_b(k_l) modes.
"""
import numpy as np

from .basis import basis_size
from .solvers import block_solve


def restrict(X, nb_coarse):
    """Keep the first nb_coarse modes of every variable (L2 projection)."""
    return np.ascontiguousarray(X[..., :nb_coarse])


def prolong(Xc, nb_fine):
    """Zero-pad the modes above Xc's degree (injection)."""
    out = np.zeros(Xc.shape[:-1] + (nb_fine,), dtype=Xc.dtype)
    out[..., :Xc.shape[-1]] = Xc
    return out


def inherited_matrix(o, U, shift, nb_coarse):
    """Dense G_l = R G_0 P for the level with nb_coarse modes, in the flat
    order of X[e, c, b].reshape(-1).  Column j is the fine operator applied to
    the zero-padded j-th coarse unit vector, restricted to the coarse modes."""
    mc = o.nvar * nb_coarse
    n = o.ne * mc
    A = np.zeros((n, n))
    for col in range(n):
        e, l = divmod(col, mc)
        c, b = divmod(l, nb_coarse)
        V = np.zeros(U.shape)
        V[e, c, b] = 1.0
        A[:, col] = restrict(o.operator(U, V, shift), nb_coarse).reshape(-1)
    return A


def stab_matrix(o, U, nb_coarse):
    """Dense R STB_0 P for the level with nb_coarse modes (STB_0: the BR2
    stabilisation part of the fine Jacobian, DGOracle.stab_jvp)."""
    mc = o.nvar * nb_coarse
    n = o.ne * mc
    A = np.zeros((n, n))
    for col in range(n):
        e, l = divmod(col, mc)
        c, b = divmod(l, nb_coarse)
        V = np.zeros(U.shape)
        V[e, c, b] = 1.0
        A[:, col] = restrict(o.stab_jvp(U, V), nb_coarse).reshape(-1)
    return A


def truncate_matrix(A, ne, nv, nb_from, nb_to):
    """Keep the rows and columns of the first nb_to modes of every variable
    (the Galerkin projection between two coarse levels)."""
    keep = (np.arange(ne * nv * nb_from).reshape(ne, nv, nb_from)[:, :, :nb_to]).reshape(-1)
    return A[np.ix_(keep, keep)]


def stab_scale(k_from, k_to, d):
    """S = k_to (k_to + d) / (k_from (k_from + d)) (App. A)."""
    return k_to * (k_to + d) / (k_from * (k_from + d))


def greedy_colouring(nbr):
    """Colour of every element: the smallest colour not used by an earlier
    face neighbour (elements in index order, self-neighbours ignored)."""
    ne = nbr.shape[0]
    col = -np.ones(ne, dtype=np.int64)
    for e in range(ne):
        used = {int(col[n]) for n in nbr[e] if n != e and col[n] >= 0}
        c = 0
        while c in used:
            c += 1
        col[e] = c
    return col


class BlockILU0:
    """Block ILU(0) of a level operator (dense, element-major blocks of size m)
    in the multicolour order of the face-neighbour graph (colour, then element
    index): the textbook elimination restricted to the block pattern of the
    operator (element K couples to itself and to its face neighbours), fill
    outside the pattern dropped.  Stands in for the ILU-based coarse smoother
    preconditioner of the paper (ASM(1,ILU(0)) over subdomains)."""

    def __init__(self, A, ne, m, nbr, colour):
        order = np.lexsort((np.arange(ne), colour))           # colour-major
        pos = np.empty(ne, dtype=np.int64)
        pos[order] = np.arange(ne)
        pat = np.zeros((ne, ne), dtype=bool)
        for e in range(ne):
            pat[e, e] = True
            pat[e, nbr[e]] = True
        blk = lambda X, i, j: X[i * m:(i + 1) * m, j * m:(j + 1) * m]
        LU = A.copy()
        for kk in range(ne):
            k = order[kk]
            Dk_inv = np.linalg.inv(blk(LU, k, k))
            for ii in range(kk + 1, ne):
                i = order[ii]
                if not pat[i, k]:
                    continue
                Lik = blk(LU, i, k) @ Dk_inv
                LU[i * m:(i + 1) * m, k * m:(k + 1) * m] = Lik
                for jj in range(kk + 1, ne):
                    j = order[jj]
                    if pat[k, j] and pat[i, j]:
                        LU[i * m:(i + 1) * m, j * m:(j + 1) * m] -= Lik @ blk(LU, k, j)
        self.LU, self.order, self.pos, self.pat, self.ne, self.m = LU, order, pos, pat, ne, m

    def factors(self):
        """(L, U) as dense matrices in the element ordering: L unit block lower,
        U block upper, with respect to the multicolour order."""
        ne, m = self.ne, self.m
        L = np.eye(ne * m)
        U = np.zeros((ne * m, ne * m))
        for i in range(ne):
            for j in range(ne):
                if not self.pat[i, j]:
                    continue
                B = self.LU[i * m:(i + 1) * m, j * m:(j + 1) * m]
                if self.pos[j] < self.pos[i]:
                    L[i * m:(i + 1) * m, j * m:(j + 1) * m] = B
                else:
                    U[i * m:(i + 1) * m, j * m:(j + 1) * m] = B
        return L, U

    def solve(self, r):
        """(L U)^-1 r by block forward and backward substitution."""
        ne, m = self.ne, self.m
        blk = lambda i, j: self.LU[i * m:(i + 1) * m, j * m:(j + 1) * m]
        y = np.array(r, dtype=np.float64).reshape(ne, m)
        for k in self.order:                                   # forward, unit lower
            for j in range(ne):
                if self.pat[k, j] and self.pos[j] < self.pos[k]:
                    y[k] -= blk(k, j) @ y[j]
        z = y.copy()
        for k in self.order[::-1]:                             # backward, upper
            for j in range(ne):
                if self.pat[k, j] and self.pos[j] > self.pos[k]:
                    z[k] -= blk(k, j) @ z[j]
            z[k] = np.linalg.solve(blk(k, k), z[k])
        return z.reshape(-1)


def diagonal_blocks(A, ne, m):
    """Diagonal m x m blocks of a dense element-major matrix, [ne, m, m]."""
    return np.stack([A[e * m:(e + 1) * m, e * m:(e + 1) * m] for e in range(ne)])


def gmres_fixed(apply_A, apply_Minv, g, x0, iters, breakdown_tol=1e-14):
    """x0 + M^-1 V_k y with y minimising ||g - A(x0 + M^-1 V_k y)||: k = iters
    GMRES steps on A M^-1 (one cycle, no restart), Arnoldi by classical
    Gram-Schmidt with one re-orthogonalisation.  Stops early only on a happy
    breakdown (||w|| <= breakdown_tol ||A M^-1 v_j||).  Flat vectors."""
    x0 = np.zeros_like(g) if x0 is None else x0
    r = g - apply_A(x0) if np.any(x0) else g.copy()
    beta = np.linalg.norm(r)
    if beta == 0.0 or iters == 0:
        return x0.copy()
    V = [r / beta]
    H = np.zeros((iters + 1, iters))
    k = 0
    for j in range(iters):
        w = apply_A(apply_Minv(V[j]))
        w0 = np.linalg.norm(w)
        B = np.array(V)
        h = B @ w
        w = w - B.T @ h
        h2 = B @ w
        w = w - B.T @ h2
        hn = np.linalg.norm(w)
        H[:j + 1, j] = h + h2
        H[j + 1, j] = hn
        k = j + 1
        if hn <= breakdown_tol * w0:
            break
        V.append(w / hn)
    rhs = np.zeros(k + 1)
    rhs[0] = beta
    y = np.linalg.lstsq(H[:k + 1, :k], rhs, rcond=None)[0]
    return x0 + apply_Minv(np.array(V[:k]).T @ y)


class PMultigrid:
    """Alg. vcic (or fullvcic) with inherited (optionally rescaled-inherited,
    App. A) operators and GMRES[EWBJ] smoothers.

    orders: degrees k_0 > ... > k_L (k_0 = o.order); iters: smoothing
    iterations per level, the last one being the coarsest-level solve.
    """

    def __init__(self, o, U, shift, orders, iters, cycle="V", rescale=False, coarse_ilu=False):
        assert orders[0] == o.order and all(a > b for a, b in zip(orders, orders[1:]))
        assert len(iters) == len(orders) and cycle in ("V", "full")
        self.o, self.U, self.shift, self.cycle = o, U, float(shift), cycle
        self.iters = list(iters)
        self.nbs = [basis_size(k, o.d) for k in orders]
        self.L = len(orders) - 1
        if not rescale:
            self.A = [None] + [inherited_matrix(o, U, shift, nb) for nb in self.nbs[1:]]
        else:
            # eq. GalProjResc: G_{l+1} = R (G_l - STB_l) P + S_l^{l+1} R STB_l P,
            # STB_{l+1} = S_l^{l+1} R STB_l P, starting from the fine operator
            self.A = [None]
            G = inherited_matrix(o, U, shift, self.nbs[1])
            S = stab_matrix(o, U, self.nbs[1])
            for l in range(1, self.L + 1):
                if l > 1:
                    G = truncate_matrix(G, o.ne, o.nvar, self.nbs[l - 1], self.nbs[l])
                    S = truncate_matrix(S, o.ne, o.nvar, self.nbs[l - 1], self.nbs[l])
                sc = stab_scale(orders[l - 1], orders[l], o.d)
                G = G - (1.0 - sc) * S
                S = sc * S
                self.A.append(G)
        self.D = [o.block_diagonal(U, shift)] + [
            diagonal_blocks(self.A[l], o.ne, o.nvar * self.nbs[l]) for l in range(1, self.L + 1)]
        # optional block ILU(0) preconditioner of the coarsest level's smoother
        self.ilu = (BlockILU0(self.A[self.L], o.ne, o.nvar * self.nbs[self.L], o.nbr,
                              greedy_colouring(o.nbr)) if coarse_ilu else None)

    def update_fine(self, U, shift, refresh_blocks=True):
        """Preconditioner lagging (Sec. 4, time-step study): the fine level's
        operator (and, with refresh_blocks, its block-Jacobi blocks) follows the
        new state and shift; the coarse operators and their blocks stay those of
        the state the hierarchy was built at."""
        self.U, self.shift = U, float(shift)
        if refresh_blocks:
            self.D[0] = self.o.block_diagonal(U, shift)

    # level operators on flat vectors of X[e, c, b] with N_b(k_l) modes
    def _shape(self, l):
        return (self.o.ne, self.o.nvar, self.nbs[l])

    def apply_G(self, l, x):
        if l == 0:
            return self.o.operator(self.U, x.reshape(self._shape(0)), self.shift).reshape(-1)
        return self.A[l] @ x

    def apply_Minv(self, l, x):
        if l == self.L and self.ilu is not None:
            return self.ilu.solve(x)
        return block_solve(self.D[l], x.reshape(self.o.ne, -1)).reshape(-1)

    def smooth(self, l, g, x0):
        return gmres_fixed(lambda v: self.apply_G(l, v), lambda v: self.apply_Minv(l, v), g, x0, self.iters[l])

    def vcycle(self, l, g, trace=None):
        """MG_V(l, g, 0) on flat level-l vectors.  `trace` (a dict, optional)
        receives the level-l iterates after pre-smoothing and after the
        coarse-grid correction."""
        if l == self.L:
            return self.smooth(l, g, None)
        w = self.smooth(l, g, None)                                       # pre-smoothing
        d = g - self.apply_G(l, w)                                        # defect
        dc = restrict(d.reshape(self._shape(l)), self.nbs[l + 1]).reshape(-1)
        e = self.vcycle(l + 1, dc)                                        # coarse-grid correction
        w_hat = w + prolong(e.reshape(self._shape(l + 1)), self.nbs[l]).reshape(-1)
        if trace is not None:
            trace[l] = (w, w_hat)
        return self.smooth(l, g, w_hat)                                   # post-smoothing

    def full(self, l, g):
        """MG_full(l, g, 0) on flat level-l vectors (Alg. fullvcic)."""
        if l == self.L:
            return self.smooth(l, g, None)
        gc = restrict(g.reshape(self._shape(l)), self.nbs[l + 1]).reshape(-1)
        w_hat = prolong(self.full(l + 1, gc).reshape(self._shape(l + 1)), self.nbs[l]).reshape(-1)
        d = g - self.apply_G(l, w_hat)                                    # defect of the prolonged solution
        return w_hat + self.vcycle(l, d)                                  # V-cycle correction

    def apply(self, R):
        """The preconditioner on the fine level, R[e, c, b] -> Z: MG_V(0, R, 0),
        or MG_full(0, R, 0) for the full cycle."""
        g = np.asarray(R, dtype=np.float64).reshape(-1)
        z = self.vcycle(0, g) if self.cycle == "V" else self.full(0, g)
        return z.reshape(self._shape(0))
