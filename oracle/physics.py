"""Pointwise fluxes.  Every function accepts real or complex arrays.

Complex inputs are used for complex-step differentiation: branches (abs, max,
entropy-fix switch) are taken on the real part, so the imaginary part carries
the exact tangent of the branch that the real computation takes (ties pick
the first argument, sign(0) = +1).

Compressible Navier-Stokes, conserved variables U = (rho, rho*u, rho*E):
  p = (gamma-1)(rho*E - rho|u|^2/2),   H = (rho*E + p)/rho,   c^2 = gamma*p/rho
  F^c_p = (rho*u_p, rho*u_p*u + p*e_p, rho*u_p*H)
  F^v_p = (0, tau_p., sum_j tau_pj*u_j - q_p)
  tau = mu*(grad u + grad u^T - 2/3 div(u) I)   (Stokes hypothesis, as in the
        paper's viscous flux of Sec. 2.1)
  q = -mu*gamma/(Pr*(gamma-1)) * grad(p/rho)    (Fourier law, gas constant free)
Velocity and p/rho gradients come from the corrected conservative gradient G.
"""
import numpy as np


def rabs(x):
    """|x| with the branch decided on the real part (complex-step safe)."""
    return np.where(np.real(x) >= 0, x, -x)


def rmax(a, b):
    """max(a, b) decided on real parts; ties pick a (complex-step safe)."""
    return np.where(np.real(a) >= np.real(b), a, b)


class NavierStokes:
    def __init__(self, dim, gamma=1.4, prandtl=0.72, mu=1e-3, flux="roe", eta=None,
                 entropy_fix=0.1):
        self.d = int(dim)
        self.nvar = self.d + 2
        self.gamma = float(gamma)
        self.prandtl = float(prandtl)
        self.mu = float(mu)
        self.flux = flux
        self.eta = float(2 * self.d + 1) if eta is None else float(eta)
        self.entropy_fix = float(entropy_fix)

    # ---- primitive helpers -------------------------------------------------
    def _prim(self, U):
        d, g = self.d, self.gamma
        rho = U[..., 0]
        m = U[..., 1:1 + d]
        rE = U[..., d + 1]
        u = m / rho[..., None]
        p = (g - 1.0) * (rE - 0.5 * np.sum(m * u, axis=-1))
        return rho, u, rE, p

    def pressure(self, U):
        return self._prim(U)[3]

    def sound_speed(self, U):
        rho, _, _, p = self._prim(U)
        return np.sqrt(self.gamma * p / rho)

    # ---- physical fluxes ---------------------------------------------------
    def conv_flux(self, U):
        """F^c[..., p, c]."""
        d = self.d
        rho, u, rE, p = self._prim(U)
        F = np.zeros(U.shape[:-1] + (d, self.nvar), dtype=U.dtype)
        for P in range(d):
            F[..., P, 0] = rho * u[..., P]
            for j in range(d):
                F[..., P, 1 + j] = rho * u[..., P] * u[..., j]
            F[..., P, 1 + P] += p
            F[..., P, d + 1] = u[..., P] * (rE + p)
        return F

    def visc_flux(self, U, G):
        """F^v[..., p, c] from the state U[..., c] and corrected gradient G[..., c, p]."""
        d, g, mu = self.d, self.gamma, self.mu
        rho, u, rE, p = self._prim(U)
        dtype = np.result_type(U, G)
        # grad_u[..., j, P] = d u_j / d x_P
        grad_u = (G[..., 1:1 + d, :] - u[..., :, None] * G[..., 0:1, :]) / rho[..., None, None]
        div = sum(grad_u[..., j, j] for j in range(d))
        e = rE / rho
        grad_e = (G[..., d + 1, :] - e[..., None] * G[..., 0, :]) / rho[..., None]
        grad_pr = (g - 1.0) * (grad_e - np.einsum("...j,...jp->...p", u, grad_u))
        kap = mu * g / (self.prandtl * (g - 1.0))
        F = np.zeros(U.shape[:-1] + (d, self.nvar), dtype=dtype)
        for P in range(d):
            for j in range(d):
                tau = mu * (grad_u[..., j, P] + grad_u[..., P, j])
                if j == P:
                    tau = tau - (2.0 / 3.0) * mu * div
                F[..., P, 1 + j] = tau
                F[..., P, d + 1] += tau * u[..., j]
            F[..., P, d + 1] += kap * grad_pr[..., P]
        return F

    # ---- numerical convective flux -----------------------------------------
    def conv_numflux(self, UL, UR, n):
        """H^c(UL, UR, n)[..., c]; n[..., d] is the unit normal from L to R."""
        Fn = 0.5 * (np.einsum("...pc,...p->...c", self.conv_flux(UL), n)
                    + np.einsum("...pc,...p->...c", self.conv_flux(UR), n))
        if self.flux == "lf":
            rhoL, uL, _, pL = self._prim(UL)
            rhoR, uR, _, pR = self._prim(UR)
            cL = np.sqrt(self.gamma * pL / rhoL)
            cR = np.sqrt(self.gamma * pR / rhoR)
            unL = np.sum(uL * n, axis=-1)
            unR = np.sum(uR * n, axis=-1)
            lam = rmax(rabs(unL) + cL, rabs(unR) + cR)
            return Fn - 0.5 * lam[..., None] * (UR - UL)
        if self.flux == "roe":
            return Fn - 0.5 * self.roe_dissipation(UL, UR, n)
        raise ValueError(self.flux)

    def roe_dissipation(self, UL, UR, n, signed=False):
        """|A_roe|(UR - UL) as a sum of characteristic waves.

        signed=True replaces |lambda| by lambda, which must give
        F^c(UR).n - F^c(UL).n exactly (the Roe property); used as a pin.
        Harten's entropy fix |l|_delta = (l^2 + delta^2)/(2 delta) for
        |l| < delta, delta = entropy_fix * (|u~.n| + c~), on every wave.
        """
        d, g = self.d, self.gamma
        rhoL, uL, rEL, pL = self._prim(UL)
        rhoR, uR, rER, pR = self._prim(UR)
        HL = (rEL + pL) / rhoL
        HR = (rER + pR) / rhoR
        sL = np.sqrt(rhoL)
        sR = np.sqrt(rhoR)
        wsum = sL + sR
        ut = (sL[..., None] * uL + sR[..., None] * uR) / wsum[..., None]
        Ht = (sL * HL + sR * HR) / wsum
        q2 = np.sum(ut * ut, axis=-1)
        ct2 = (g - 1.0) * (Ht - 0.5 * q2)
        ct = np.sqrt(ct2)
        unt = np.sum(ut * n, axis=-1)
        rhot = sL * sR
        dr = rhoR - rhoL
        dp = pR - pL
        du = uR - uL
        dun = np.sum(du * n, axis=-1)
        a1 = (dp - rhot * ct * dun) / (2.0 * ct2)
        a5 = (dp + rhot * ct * dun) / (2.0 * ct2)
        a2 = dr - dp / ct2
        dut = du - dun[..., None] * n
        if signed:
            l1, l2, l5 = unt - ct, unt, unt + ct
        else:
            delta = self.entropy_fix * (rabs(unt) + ct)

            def fixabs(lam):
                al = rabs(lam)
                return np.where(np.real(al) < np.real(delta), (lam * lam + delta * delta) / (2.0 * delta), al)

            l1, l2, l5 = fixabs(unt - ct), fixabs(unt), fixabs(unt + ct)
        D = np.zeros(np.broadcast_shapes(UL.shape, UR.shape), dtype=np.result_type(UL, UR, n))
        D[..., 0] = l1 * a1 + l2 * a2 + l5 * a5
        for j in range(d):
            D[..., 1 + j] = (l1 * a1 * (ut[..., j] - ct * n[..., j])
                             + l2 * (a2 * ut[..., j] + rhot * dut[..., j])
                             + l5 * a5 * (ut[..., j] + ct * n[..., j]))
        D[..., d + 1] = (l1 * a1 * (Ht - ct * unt)
                         + l2 * (a2 * 0.5 * q2 + rhot * np.sum(ut * dut, axis=-1))
                         + l5 * a5 * (Ht + ct * unt))
        return D

    def max_wave_speed(self, U):
        rho, u, _, p = self._prim(U)
        return np.sqrt(np.sum(u * u, axis=-1)) + np.sqrt(self.gamma * p / rho)


class Diffusion:
    """Scalar diffusion: F^c = 0, F^v = mu * G (one variable)."""

    def __init__(self, dim, mu=1.0, eta=None):
        self.d = int(dim)
        self.nvar = 1
        self.mu = float(mu)
        self.eta = float(2 * self.d + 1) if eta is None else float(eta)

    def conv_flux(self, U):
        return np.zeros(U.shape[:-1] + (self.d, 1), dtype=U.dtype)

    def visc_flux(self, U, G):
        return self.mu * np.swapaxes(G, -1, -2)

    def conv_numflux(self, UL, UR, n):
        return np.zeros(np.broadcast_shapes(UL.shape, UR.shape), dtype=np.result_type(UL, UR))


class IncompressibleNS:
    """Incompressible Navier-Stokes equations of Sec. 2.1 (eq. ns), unit
    density, unknowns w = (u_1..u_d, p) (velocity first, pressure last):

      F_p = (u_p u + p e_p,  u_p)       convective part and the mass flux
      F^v_p = (nu (grad u + grad u^T - 2/3 div(u) I)_p.,  0)

    so that the residual of eq. NSdiscrRes carries the momentum equations and
    the divergence constraint tested with q.  The time derivative acts on the
    velocities only (mass form m_h of eq. massBil): ``mass`` is 1 for the d
    velocity components and 0 for the pressure.

    Interface flux.  The paper takes it from the exact solution of Riemann
    problems of an artificial compressibility perturbation of the Euler
    equations, defined in a cited work only.  Stand-in: the Lax-Friedrichs
    flux of that perturbed system, with the pressure equation
    (1/beta^2) dp/dt + div u = 0 (so that its flux is the residual's u),
        H = 1/2 (F(w_L) + F(w_R)).n - 1/2 lambda diag(1,..,1, 1/beta^2) (w_R - w_L),
    lambda = max over both sides of |u.n| + sqrt((u.n)^2 + beta^2), the
    largest eigenvalue modulus of that system's normal flux Jacobian.
    """

    def __init__(self, dim, nu=1e-2, beta=1.0, eta=None):
        self.d = int(dim)
        self.nvar = self.d + 1
        self.nu = float(nu)
        self.beta = float(beta)
        self.eta = float(2 * self.d + 1) if eta is None else float(eta)
        self.mass = np.array([1.0] * self.d + [0.0])

    def conv_flux(self, U):
        """F_p[..., p, c] (momentum: u_p u_i + p delta_pi; mass: u_p)."""
        d = self.d
        u = U[..., :d]
        p = U[..., d]
        F = np.zeros(U.shape[:-1] + (d, self.nvar), dtype=U.dtype)
        for P in range(d):
            for i in range(d):
                F[..., P, i] = u[..., P] * u[..., i]
            F[..., P, P] += p
            F[..., P, d] = u[..., P]
        return F

    def visc_flux(self, U, G):
        """F^v[..., p, c] from the corrected gradient G[..., c, p] (velocity rows)."""
        d, nu = self.d, self.nu
        dtype = np.result_type(U, G)
        g = G[..., :d, :]                       # g[..., i, j] = d u_i / d x_j
        div = sum(g[..., j, j] for j in range(d))
        F = np.zeros(U.shape[:-1] + (d, self.nvar), dtype=dtype)
        for P in range(d):
            for i in range(d):
                t = nu * (g[..., P, i] + g[..., i, P])
                if i == P:
                    t = t - (2.0 / 3.0) * nu * div
                F[..., P, i] = t
        return F

    def wave_speed_n(self, U, n):
        un = np.sum(U[..., :self.d] * n, axis=-1)
        return rabs(un) + np.sqrt(un * un + self.beta ** 2)

    def conv_numflux(self, UL, UR, n):
        Fn = 0.5 * (np.einsum("...pc,...p->...c", self.conv_flux(UL), n)
                    + np.einsum("...pc,...p->...c", self.conv_flux(UR), n))
        lam = rmax(self.wave_speed_n(UL, n), self.wave_speed_n(UR, n))
        scale = np.array([1.0] * self.d + [1.0 / self.beta ** 2])
        return Fn - 0.5 * lam[..., None] * scale * (UR - UL)

    def max_wave_speed(self, U):
        q = np.sqrt(np.sum(U[..., :self.d] ** 2, axis=-1))
        return q + np.sqrt(q * q + self.beta ** 2)
