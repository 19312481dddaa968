"""DG residual, Jacobian-vector products and diagonal blocks (FP64 oracle).

State layout inside the oracle: U[e, c, b] (element, variable, mode).

Geometry: every element is the multilinear image of [-1,1]^d through its
2^d corners.  J = dx/dxi, |J| = det J, physical gradients J^{-T} grad_xi.
Face normals and area factors follow Nanson's formula n dA = |J| J^{-T} N dA_ref
evaluated from the owning element.

Physical basis: phi_K = L_K^{-1} psi with L_K L_K^T = sum_q w_q |J_q| psi psi^T
(Cholesky of the discrete reference mass matrix), so that phi_K is orthonormal
in the discrete L2(K) inner product and stays hierarchical (L_K is lower
triangular).  On affine elements phi_K = psi / sqrt|J|.

Faces: face (p, e) is the +p face of its owner e; the neighbour is
e' = nbr[e, 2p+1]; n points from e to e' and [[v]] = v_e - v_e'.

Residual (eq. NSdiscrRes, Sec. 2.2), per element K, mode b, variable c:
  R_Kbc = - sum_q w_q|J_q| sum_p F_pc(U_q, G_q) d_p phi_b(x_q)
          + sum_{faces of K} (+/-) sum_f w_f|J_f| Hn_c(x_f) phi_b(x_f)
with + on the owner side, - on the neighbour side (the jump of the test
function), F = F^c - F^v and
  Hn = H^c(U_e, U_e', n) - F^v({U}, {grad U} + eta {r}) . n.
BR2 lifting (Sec. 2.1): the consistent gradient is G = grad U + R^K with
R^K = sum of the local liftings r^sigma of K's faces, where the local lifting
satisfies  int r^sigma . tau = - int_sigma [[U]] {tau} . n.  With an
orthonormal basis its coefficients on side S of sigma are
  rho^{sigma,S}_{b,c,p} = -1/2 sum_f w_f|J_f| [[U_c]](x_f) n_p(x_f) phi^S_b(x_f).
The face viscous flux is evaluated at the averaged state with the averaged
gradient plus eta times the averaged local lifting.  eq. (vflux) prints the
opposite sign for the lifting terms; that reading makes the BR2 Laplacian
non-symmetric with negative stabilisation, contradicting the coercivity
statement that follows it, so the sign consistent with the definition of the
consistent gradient is used (lifting_sign=+1).  lifting_sign=-1 reproduces
the printed sign for the test that pins this choice.
"""
import numpy as np

from .basis import eval_basis, multi_indices
from .quadrature import tensor_rule


def _ein(*args):
    return np.einsum(*args, optimize=True)


def _shape_functions(xi):
    """Multilinear shape functions N[q, v] and derivatives dN[q, v, j] at xi[q, d]."""
    q, d = xi.shape
    nv = 2 ** d
    N = np.ones((q, nv))
    dN = np.ones((q, nv, d))
    for v in range(nv):
        for i in range(d):
            bit = (v >> i) & 1
            f = 0.5 * (1.0 + xi[:, i]) if bit else 0.5 * (1.0 - xi[:, i])
            df = 0.5 if bit else -0.5
            N[:, v] *= f
            for j in range(d):
                dN[:, v, j] *= df if i == j else f
    return N, dN


class DGOracle:
    def __init__(self, mesh, order, space, nq1d, physics, lifting_sign=+1):
        self.d = int(mesh["dim"])
        self.xyz = np.asarray(mesh["elem_xyz"], dtype=np.float64)
        self.nbr = np.asarray(mesh["elem_nbr"], dtype=np.int64)
        self.ne = self.xyz.shape[0]
        self.order = int(order)
        self.space = space
        self.nq1d = int(nq1d)
        self.phys = physics
        self.nvar = physics.nvar
        self.lifting_sign = float(lifting_sign)
        self.alphas = multi_indices(self.order, self.d, space)
        self.nb = len(self.alphas)
        self.xi_v, self.w_v = tensor_rule(self.nq1d, self.d)
        self.xi_f, self.w_f = tensor_rule(self.nq1d, self.d - 1)
        self.psi_v, self.dpsi_v = eval_basis(self.alphas, self.xi_v)
        self.nq = len(self.w_v)
        self.nfq = len(self.w_f)
        self._full = None

    # ------------------------------------------------------------------ geometry
    def face_ref_points(self, p, side):
        """Reference points of the (p, side) face: xi_p = side, others from the face rule."""
        others = [i for i in range(self.d) if i != p]
        xi = np.empty((self.nfq, self.d))
        xi[:, p] = float(side)
        for k, i in enumerate(others):
            xi[:, i] = self.xi_f[:, k]
        return xi

    def map_points(self, elems, xi):
        """Physical points x[E, Q, d] and Jacobians J[E, Q, d, d] (J_ij = dx_i/dxi_j)."""
        N, dN = _shape_functions(xi)
        X = self.xyz[elems]
        x = _ein("qv,evi->eqi", N, X)
        J = _ein("qvj,evi->eqij", dN, X)
        return x, J

    def cholesky(self, elems):
        _, J = self.map_points(elems, self.xi_v)
        det = np.linalg.det(J)
        M = _ein("q,eq,qa,qb->eab", self.w_v, det, self.psi_v, self.psi_v)
        return np.linalg.cholesky(M)

    def _phys_basis(self, Linv, J, psi, dpsi):
        """phi[E,Q,Nb] and physical gradient gphi[E,Q,Nb,d] from reference tables."""
        Jinv = np.linalg.inv(J)
        phi = _ein("eab,qb->eqa", Linv, psi)
        gref = _ein("eqji,qbj->eqbi", Jinv, dpsi)
        gphi = _ein("eab,eqbi->eqai", Linv, gref)
        return phi, gphi

    def elem_tables(self, elems):
        elems = np.asarray(elems, dtype=np.int64)
        x, J = self.map_points(elems, self.xi_v)
        det = np.linalg.det(J)
        Linv = np.linalg.inv(self.cholesky(elems))
        phi, gphi = self._phys_basis(Linv, J, self.psi_v, self.dpsi_v)
        return dict(x=x, phi=phi, gphi=gphi, wdet=self.w_v[None, :] * det, det=det, Linv=Linv)

    def face_tables(self, fp, fo):
        """Owner (L) and neighbour (R) traces, unit normal and weights of faces (fp, fo)."""
        fp = np.asarray(fp, dtype=np.int64)
        fo = np.asarray(fo, dtype=np.int64)
        fn = self.nbr[fo, 2 * fp + 1]
        nf = len(fp)
        d, nb, nfq = self.d, self.nb, self.nfq
        out = dict(phiL=np.empty((nf, nfq, nb)), gphiL=np.empty((nf, nfq, nb, d)),
                   phiR=np.empty((nf, nfq, nb)), gphiR=np.empty((nf, nfq, nb, d)),
                   n=np.empty((nf, nfq, d)), W=np.empty((nf, nfq)), xL=np.empty((nf, nfq, d)),
                   xR=np.empty((nf, nfq, d)), fn=fn)
        for p in range(d):
            sel = np.nonzero(fp == p)[0]
            if len(sel) == 0:
                continue
            for side, key, elems in ((+1, "L", fo[sel]), (-1, "R", fn[sel])):
                xi = self.face_ref_points(p, side)
                psi, dpsi = eval_basis(self.alphas, xi)
                x, J = self.map_points(elems, xi)
                Linv = np.linalg.inv(self.cholesky(elems))
                phi, gphi = self._phys_basis(Linv, J, psi, dpsi)
                out["phi" + key][sel] = phi
                out["gphi" + key][sel] = gphi
                out["x" + key][sel] = x
                if side == +1:
                    det = np.linalg.det(J)
                    a = det[..., None] * np.linalg.inv(J)[..., p, :]  # Nanson, N = +e_p
                    area = np.sqrt(np.sum(a * a, axis=-1))
                    out["n"][sel] = a / area[..., None]
                    out["W"][sel] = self.w_f[None, :] * area
        return out

    # ----------------------------------------------------------------- residual
    def _faces_of(self, elems):
        d = self.d
        fp = np.concatenate([np.full(2 * len(elems), p) for p in range(d)])
        fo = np.concatenate([np.concatenate([elems, self.nbr[elems, 2 * p]]) for p in range(d)])
        key = np.unique(fp * self.ne + fo)
        return key // self.ne, key % self.ne

    def _setup(self, elems):
        if elems is None:
            if self._full is None:
                el = np.arange(self.ne)
                fp, fo = self._faces_of(el)
                self._full = (el, fp, fo, self.face_tables(fp, fo), self.elem_tables(el))
            return self._full
        el = np.unique(np.asarray(elems, dtype=np.int64))
        fp, fo = self._faces_of(el)
        return el, fp, fo, self.face_tables(fp, fo), self.elem_tables(el)

    def residual(self, U, elems=None, return_parts=False, U_lift=None):
        """R[E, c, b] for the elements `elems` (all elements if None).
        U_lift (optional): state whose jumps feed the face lifting term eta {r}
        of the face viscous flux (only there; the elemental lifting R^K keeps U)."""
        el, fp, fo, ft, et = self._setup(elems)
        fn = ft["fn"]
        phys = self.phys
        s = self.lifting_sign
        dtype = U.dtype
        pos = np.full(self.ne, -1)
        pos[el] = np.arange(len(el))

        # traces on both sides of every face
        uL = _ein("fqb,fcb->fqc", ft["phiL"], U[fo])
        uR = _ein("fqb,fcb->fqc", ft["phiR"], U[fn])
        gL = _ein("fqbp,fcb->fqcp", ft["gphiL"], U[fo])
        gR = _ein("fqbp,fcb->fqcp", ft["gphiR"], U[fn])
        jump = uL - uR
        n = ft["n"]
        W = ft["W"]
        # local lifting coefficients on each side
        rhoL = -0.5 * _ein("fq,fqp,fqc,fqb->fbcp", W, n, jump, ft["phiL"])
        rhoR = -0.5 * _ein("fq,fqp,fqc,fqb->fbcp", W, n, jump, ft["phiR"])
        if U_lift is None:
            rL = _ein("fqb,fbcp->fqcp", ft["phiL"], rhoL)
            rR = _ein("fqb,fbcp->fqcp", ft["phiR"], rhoR)
        else:
            jl = _ein("fqb,fcb->fqc", ft["phiL"], U_lift[fo]) - _ein("fqb,fcb->fqc", ft["phiR"], U_lift[fn])
            rL = _ein("fqb,fbcp->fqcp", ft["phiL"], -0.5 * _ein("fq,fqp,fqc,fqb->fbcp", W, n, jl, ft["phiL"]))
            rR = _ein("fqb,fbcp->fqcp", ft["phiR"], -0.5 * _ein("fq,fqp,fqc,fqb->fbcp", W, n, jl, ft["phiR"]))
        gface = 0.5 * (gL + gR) + s * phys.eta * 0.5 * (rL + rR)
        uavg = 0.5 * (uL + uR)
        Hn = phys.conv_numflux(uL, uR, n) - _ein("fqpc,fqp->fqc", phys.visc_flux(uavg, gface), n)

        # elemental lifting R^K = sum of the local liftings of K's faces
        ne_loc = len(el)
        RK = np.zeros((ne_loc, self.nb, self.nvar, self.d), dtype=dtype)
        mo = pos[fo] >= 0
        mn = pos[fn] >= 0
        np.add.at(RK, pos[fo[mo]], rhoL[mo])
        np.add.at(RK, pos[fn[mn]], rhoR[mn])

        # volume term
        Ue = U[el]
        u = _ein("eqb,ecb->eqc", et["phi"], Ue)
        G = _ein("eqbp,ecb->eqcp", et["gphi"], Ue) + s * _ein("eqb,ebcp->eqcp", et["phi"], RK)
        F = phys.conv_flux(u) - phys.visc_flux(u, G)
        R = -_ein("eq,eqpc,eqbp->ecb", et["wdet"], F, et["gphi"])
        Rvol = R.copy() if return_parts else None

        # face term: + on the owner side, - on the neighbour side
        cL = _ein("fq,fqc,fqb->fcb", W, Hn, ft["phiL"])
        cR = _ein("fq,fqc,fqb->fcb", W, Hn, ft["phiR"])
        np.add.at(R, pos[fo[mo]], cL[mo])
        np.add.at(R, pos[fn[mn]], -cR[mn])
        if return_parts:
            return R, Rvol
        return R

    # ----------------------------------------------------------- linearisation
    def jvp(self, U, V, elems=None, h=1e-100):
        """Exact J(U) V by complex-step differentiation of the residual.

        Im R(U + i h V) / h equals the forward-mode tangent to round-off: every
        product of two imaginary parts is O(h^2) and vanishes against the real
        parts.  This is the linearisation j_h of Sec. 2.2.
        """
        Uc = U.astype(np.complex128) + 1j * h * V
        return np.imag(self.residual(Uc, elems)) / h

    def stab_jvp(self, U, V, elems=None, h=1e-100):
        """The BR2 stabilisation part of J(U) V (the last term of eq.
        jacTrilFNURef): the derivative of the residual through the face lifting
        argument eta {r} of the face viscous flux only, by complex step."""
        Uc = U.astype(np.complex128)
        return np.imag(self.residual(Uc, elems, U_lift=U + 1j * h * V)) / h

    @staticmethod
    def fd_step(U, V, eps=1e-9):
        """Step of the finite-difference Jv, eq. (epsdef) as printed:
        Delta = eps*sqrt(1 + ||U||)/||V||, with L2 norms, which equal the DOF
        2-norms for an orthonormal basis."""
        return eps * np.sqrt(1.0 + np.linalg.norm(U)) / np.linalg.norm(V)

    def jvp_fd(self, U, V, R0=None, eps=1e-9, elems=None):
        """Finite-difference Jv of eqs. (matrix-free), (epsdef): one-sided,
        (R(U + Delta V) - R(U))/Delta with Delta from fd_step."""
        delta = self.fd_step(U, V, eps)
        if R0 is None:
            R0 = self.residual(U, elems)
        return (self.residual(U + delta * V, elems) - R0) / delta

    def mass(self):
        """Per-variable mass weights of eq. massBil (orthonormal basis): 1 for
        every variable with a time derivative, 0 for the incompressible
        pressure."""
        return np.asarray(getattr(self.phys, "mass", np.ones(self.nvar)), dtype=np.float64)

    def operator(self, U, V, shift, elems=None):
        """G V = shift*M V + J(U) V (eq. rosSysOp; M = I on the variables with a
        time derivative, 0 on the incompressible pressure)."""
        out = self.jvp(U, V, elems)
        Vs = V if elems is None else V[np.unique(elems)]
        return shift * self.mass()[None, :, None] * Vs + out

    def coloring(self):
        """Greedy colouring of the face-neighbour graph (self-loops ignored)."""
        color = np.full(self.ne, -1)
        for e in range(self.ne):
            used = {color[k] for k in self.nbr[e] if k != e and color[k] >= 0}
            c = 0
            while c in used:
                c += 1
            color[e] = c
        return color

    def block_diagonal(self, U, shift=0.0, method="color", h=1e-100):
        """D_K = shift*M_K + dR_K/dU_K for every element, as [Ne, n*Nb, n*Nb].

        Local DOF index l = c*Nb + b.  'brute' perturbs one element at a time;
        'color' perturbs one colour class at a time (no two elements of a class
        are face neighbours, so R_K only sees its own perturbation).
        """
        nloc = self.nvar * self.nb
        D = np.zeros((self.ne, nloc, nloc))
        if method == "brute":
            for K in range(self.ne):
                for j in range(nloc):
                    Vc = np.zeros(U.shape)
                    Vc[K, j // self.nb, j % self.nb] = 1.0
                    col = np.imag(self.residual(U.astype(np.complex128) + 1j * h * Vc, elems=[K]))[0] / h
                    D[K, :, j] = col.reshape(-1)
        else:
            color = self.coloring()
            for c in range(color.max() + 1):
                members = np.nonzero(color == c)[0]
                for j in range(nloc):
                    Vc = np.zeros(U.shape)
                    Vc[members, j // self.nb, j % self.nb] = 1.0
                    col = self.jvp(U, Vc)
                    D[members, :, j] = col[members].reshape(len(members), -1)
        D += shift * np.diag(np.repeat(self.mass(), self.nb))[None]
        return D

    # --------------------------------------------------------------- projection
    def project(self, f, elems=None, chunk=4096):
        """L2 projection of f(x)[..., n] onto the physical orthonormal basis
        (elements processed in chunks to bound memory)."""
        el = np.arange(self.ne) if elems is None else np.asarray(elems)
        out = np.empty((len(el), self.nvar, self.nb))
        for s in range(0, len(el), chunk):
            et = self.elem_tables(el[s:s + chunk])
            vals = f(et["x"])  # [E, Q, n]
            out[s:s + chunk] = _ein("eq,eqc,eqb->ecb", et["wdet"], vals, et["phi"])
        return out

    def evaluate(self, U, xi, elems=None):
        """u at reference points xi[Q, d] of each element (for error norms)."""
        el = np.arange(self.ne) if elems is None else np.asarray(elems)
        x, J = self.map_points(el, xi)
        psi, dpsi = eval_basis(self.alphas, xi)
        Linv = np.linalg.inv(self.cholesky(el))
        phi = _ein("eab,qb->eqa", Linv, psi)
        return x, _ein("eqb,ecb->eqc", phi, U[el]), np.linalg.det(J)

    def element_volumes(self):
        _, J = self.map_points(np.arange(self.ne), self.xi_v)
        return _ein("q,eq->e", self.w_v, np.linalg.det(J))

    # ------------------------------------------------------------ layout helpers
    def to_flat(self, U):
        """Oracle layout U[e,c,b] -> flat element-fastest layout idx = (c*Nb + b)*Ne + e."""
        return np.ascontiguousarray(np.transpose(U, (1, 2, 0))).reshape(-1)

    def from_flat(self, w):
        return np.ascontiguousarray(np.asarray(w).reshape(self.nvar, self.nb, self.ne).transpose(2, 0, 1))
