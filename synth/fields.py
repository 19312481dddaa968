"""Analytic initial fields (plain numpy functions of physical coordinates).

Every field maps points x[..., d] to conserved variables
(rho, rho*u_1, ..., rho*u_d, rho*E)[..., d+2] of a perfect gas.  No
discretisation arithmetic lives here.
"""
import numpy as np


def primitive_to_conserved(rho, vel, p, gamma):
    """(rho, u[..., d], p) -> (rho, rho*u, rho*E) for a perfect gas."""
    rho = np.asarray(rho)
    vel = np.asarray(vel)
    ke = 0.5 * rho * np.sum(vel * vel, axis=-1)
    rhoE = p / (gamma - 1.0) + ke
    return np.concatenate([rho[..., None], rho[..., None] * vel, rhoE[..., None]], axis=-1)


class UniformState:
    """Constant free stream."""

    def __init__(self, rho, vel, p, gamma):
        self.rho, self.vel, self.p, self.gamma = float(rho), np.asarray(vel, float), float(p), gamma

    def __call__(self, x):
        shp = x.shape[:-1]
        rho = np.full(shp, self.rho)
        vel = np.broadcast_to(self.vel, shp + (len(self.vel),))
        p = np.full(shp, self.p)
        return primitive_to_conserved(rho, vel, p, self.gamma)


class FreeStreamPlusModes:
    """2D free stream plus small seeded sinusoids (the 16x16 Q2 workload).

    Primitives (rho, u, v, p) = free stream + amp * q_ref * sum over
    (kx, ky) in {1,2,3}^2 of a*sin(2*pi*(kx*x + ky*y) + phi), with
    a ~ N(0,1)/3 and phi ~ U[0, 2*pi) drawn per variable and mode.
    """

    def __init__(self, seed=1809, gamma=1.4, speed=0.2, angle=np.pi / 6, amp=1e-2):
        self.gamma = gamma
        self.rho0 = 1.0
        self.p0 = 1.0 / gamma  # c_inf = 1
        self.u0 = np.array([speed * np.cos(angle), speed * np.sin(angle)])
        self.qref = np.array([1.0, speed, speed, 1.0 / gamma])
        self.amp = amp
        rng = np.random.default_rng(seed)
        self.k = np.array([(kx, ky) for kx in (1, 2, 3) for ky in (1, 2, 3)], dtype=float)
        nm = len(self.k)
        self.a = rng.standard_normal((4, nm)) / 3.0
        self.phi = rng.uniform(0.0, 2.0 * np.pi, size=(4, nm))

    def primitives(self, x):
        arg = 2.0 * np.pi * (x[..., None, 0] * self.k[:, 0] + x[..., None, 1] * self.k[:, 1])
        pert = np.stack([np.sum(self.a[v] * np.sin(arg + self.phi[v]), axis=-1) for v in range(4)], axis=-1)
        pert = self.amp * self.qref * pert
        rho = self.rho0 + pert[..., 0]
        vel = self.u0 + pert[..., 1:3]
        p = self.p0 + pert[..., 3]
        return rho, vel, p

    def __call__(self, x):
        rho, vel, p = self.primitives(x)
        return primitive_to_conserved(rho, vel, p, self.gamma)


class TaylorGreenStandIn:
    """3D solenoidal large-scale velocity field with Taylor-Green scales.

    u = sum_{m=1..4} A_m sin(k_m . x + phi_m), k_m drawn from the integer
    vectors in {-1,0,1}^3 minus 0, A_m Gaussian and projected orthogonal to
    k_m (so div u = 0), scaled so that max|u| = V0 over a 48^3 sample lattice
    of the box.  rho = rho0*(1 + 0.01*cos(k_r . x + phi_r)),
    p = p0*(1 + 0.01*cos(k_p . x + phi_p)) with |k|_inf = 2 modes and
    p0 = rho0*V0^2/(gamma*Ma^2).
    """

    def __init__(self, seed=1600, gamma=1.4, mach=0.1, V0=1.0, rho0=1.0, L=2 * np.pi, nmodes=4):
        rng = np.random.default_rng(seed)
        self.gamma, self.rho0, self.V0 = gamma, rho0, V0
        self.p0 = rho0 * V0 * V0 / (gamma * mach * mach)
        cands = np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
                          if (a, b, c) != (0, 0, 0)], dtype=float)
        pick = rng.choice(len(cands), size=nmodes, replace=False)
        self.k = cands[pick] * (2 * np.pi / L)
        A = rng.standard_normal((nmodes, 3))
        for m in range(nmodes):
            km = self.k[m]
            A[m] -= km * (A[m] @ km) / (km @ km)
        self.phi = rng.uniform(0, 2 * np.pi, size=nmodes)
        c2 = np.array([(a, b, c) for a in range(-2, 3) for b in range(-2, 3) for c in range(-2, 3)
                       if max(abs(a), abs(b), abs(c)) == 2], dtype=float)
        self.kr = c2[rng.integers(len(c2))] * (2 * np.pi / L)
        self.kp = c2[rng.integers(len(c2))] * (2 * np.pi / L)
        self.phr, self.php = rng.uniform(0, 2 * np.pi, size=2)
        self.A = A
        # scale so that max |u| = V0 on a sample lattice
        s = (np.arange(48) + 0.5) * (L / 48)
        X = np.stack(np.meshgrid(s, s, s, indexing="ij"), axis=-1).reshape(-1, 3)
        umax = np.sqrt(np.max(np.sum(self._vel_unscaled(X) ** 2, axis=-1)))
        self.A *= V0 / umax

    def _vel_unscaled(self, x):
        arg = x @ self.k.T + self.phi  # [..., m]
        return np.sin(arg) @ self.A

    def primitives(self, x):
        vel = self._vel_unscaled(x)
        rho = self.rho0 * (1.0 + 0.01 * np.cos(x @ self.kr + self.phr))
        p = self.p0 * (1.0 + 0.01 * np.cos(x @ self.kp + self.php))
        return rho, vel, p

    def __call__(self, x):
        rho, vel, p = self.primitives(x)
        return primitive_to_conserved(rho, vel, p, self.gamma)


class TrigSum:
    """Smooth periodic field with analytic derivatives (for manufactured solutions).

    U_c(x) = a_c + sum_m b_{c,m} sin(k_m . x + phi_m); value(), grad() and
    hess() return U, dU/dx_p and d2U/dx_p dx_q.  Works for complex x.
    """

    def __init__(self, a, b, k, phi):
        self.a = np.asarray(a, float)          # [n]
        self.b = np.asarray(b, float)          # [n, m]
        self.k = np.asarray(k, float)          # [m, d]
        self.phi = np.asarray(phi, float)      # [m]

    def _arg(self, x):
        return x @ self.k.T + self.phi

    def value(self, x):
        return self.a + np.sin(self._arg(x)) @ self.b.T

    def __call__(self, x):
        return self.value(x)

    def grad(self, x):  # [..., n, d]
        c = np.cos(self._arg(x))  # [..., m]
        return np.einsum("...m,cm,md->...cd", c, self.b, self.k)

    def hess(self, x):  # [..., n, d, d]
        s = np.sin(self._arg(x))
        return -np.einsum("...m,cm,md,me->...cde", s, self.b, self.k, self.k)


class IncompressibleStandIn:
    """Velocity and pressure (u_1..u_d, p) for the incompressible equations.

    3D: the solenoidal velocity of TaylorGreenStandIn (max |u| = V0);
    2D: u = curl of the stream function psi = sum_m a_m sin(k_m . x + phi_m)
    (k_m integer multiples of 2 pi / L, a_m ~ N(0,1)), scaled to max |u| = V0
    on a sample lattice; both divergence-free.  p = p0 + amp * cos(k_p . x +
    phi_p) with a |k|_inf = 2 mode.
    """

    def __init__(self, dim, seed=7, L=1.0, V0=1.0, p0=0.5, amp=0.05):
        rng = np.random.default_rng(seed)
        self.dim, self.p0, self.amp = int(dim), p0, amp
        if self.dim == 3:
            self.tg = TaylorGreenStandIn(seed=seed, L=L, V0=V0)
        else:
            cands = np.array([(a, b) for a in (-1, 0, 1, 2) for b in (-1, 0, 1, 2) if (a, b) != (0, 0)], float)
            self.k2 = cands[rng.choice(len(cands), 4, replace=False)] * (2 * np.pi / L)
            self.a2 = rng.standard_normal(4)
            self.ph2 = rng.uniform(0, 2 * np.pi, 4)
            s = (np.arange(64) + 0.5) * (L / 64)
            X = np.stack(np.meshgrid(s, s, indexing="ij"), axis=-1).reshape(-1, 2)
            self.a2 *= V0 / np.sqrt(np.max(np.sum(self._vel2(X) ** 2, axis=-1)))
        kp = np.array([2, 1, -2][:self.dim], float) * (2 * np.pi / L)
        self.kp, self.php = kp, rng.uniform(0, 2 * np.pi)

    def _vel2(self, x):
        c = np.cos(x @ self.k2.T + self.ph2) * self.a2       # [..., m]
        return np.stack([c @ self.k2[:, 1], -(c @ self.k2[:, 0])], axis=-1)

    def __call__(self, x):
        vel = self.tg._vel_unscaled(x) if self.dim == 3 else self._vel2(x)
        p = self.p0 + self.amp * np.cos(x @ self.kp + self.php)
        return np.concatenate([vel, p[..., None]], axis=-1)
