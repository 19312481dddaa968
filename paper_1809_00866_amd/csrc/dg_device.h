// Device-side building blocks shared by the DG kernels: dual numbers for
// forward-mode differentiation and the pointwise compressible Navier-Stokes
// fluxes (perfect gas, Stokes stress, Fourier heat flux; Lax-Friedrichs or
// Roe convective flux with Harten's entropy fix).
#pragma once

#include <type_traits>

#include "dg_internal.h"

namespace dgk {

#define DEV __device__ __forceinline__

// ------------------------------------------------------------------ dual numbers
// value + tangent in working precision R (double, or float for the reduced
// precision variant)
template <class R>
struct dualT {
  R v, d;
  DEV dualT() = default;
  DEV dualT(R x) : v(x), d(R(0)) {}
  DEV dualT(R x, R y) : v(x), d(y) {}
};
using dual = dualT<double>;
using dualf = dualT<float>;
template <class R> DEV dualT<R> operator+(dualT<R> a, dualT<R> b) { return dualT<R>(a.v + b.v, a.d + b.d); }
template <class R> DEV dualT<R> operator-(dualT<R> a, dualT<R> b) { return dualT<R>(a.v - b.v, a.d - b.d); }
template <class R> DEV dualT<R> operator*(dualT<R> a, dualT<R> b) {
  return dualT<R>(a.v * b.v, a.d * b.v + a.v * b.d);
}
template <class R> DEV dualT<R> operator/(dualT<R> a, dualT<R> b) {
  R q = a.v / b.v;
  return dualT<R>(q, (a.d - q * b.d) / b.v);
}
template <class R> DEV dualT<R> operator-(dualT<R> a) { return dualT<R>(-a.v, -a.d); }
template <class R> DEV dualT<R> operator*(R s, dualT<R> a) { return dualT<R>(s * a.v, s * a.d); }
template <class R> DEV dualT<R> operator*(dualT<R> a, R s) { return dualT<R>(s * a.v, s * a.d); }
template <class R> DEV dualT<R> operator+(dualT<R> a, R s) { return dualT<R>(a.v + s, a.d); }
template <class R> DEV dualT<R> operator+(R s, dualT<R> a) { return dualT<R>(a.v + s, a.d); }
template <class R> DEV dualT<R> operator-(dualT<R> a, R s) { return dualT<R>(a.v - s, a.d); }
template <class R> DEV dualT<R> operator-(R s, dualT<R> a) { return dualT<R>(s - a.v, -a.d); }
template <class R> DEV dualT<R> operator/(dualT<R> a, R s) { return dualT<R>(a.v / s, a.d / s); }
template <class R> DEV dualT<R> operator/(R s, dualT<R> a) {
  R q = s / a.v;
  return dualT<R>(q, -q * a.d / a.v);
}
template <class R> DEV dualT<R>& operator+=(dualT<R>& a, dualT<R> b) { a = a + b; return a; }
template <class R> DEV dualT<R>& operator-=(dualT<R>& a, dualT<R> b) { a = a - b; return a; }
template <class R> DEV dualT<R> dsqrt(dualT<R> a) {
  R r = sqrt(a.v);
  return dualT<R>(r, R(0.5) * a.d / r);
}
DEV double dsqrt(double a) { return sqrt(a); }
DEV float dsqrt(float a) { return sqrtf(a); }
DEV double val(double a) { return a; }
DEV float val(float a) { return a; }
template <class R> DEV R val(dualT<R> a) { return a.v; }
DEV double out_part(double a) { return a; }
DEV float out_part(float a) { return a; }
template <class R> DEV R out_part(dualT<R> a) { return a.d; }
// working precision of a scalar type
template <class T> struct RealOf { using type = T; };
template <class R> struct RealOf<dualT<R>> { using type = R; };
template <class T> DEV T rabs(T a) { return val(a) >= 0 ? a : -a; }
template <class T> DEV T rmax(T a, T b) { return val(a) >= val(b) ? a : b; }

template <bool JVP, class R = double> struct Scalar { using type = R; };
template <class R> struct Scalar<true, R> { using type = dualT<R>; };

template <bool JVP> DEV typename Scalar<JVP>::type load2(const double* __restrict__ U, const double* __restrict__ V,
                                                         size_t i);
template <> DEV double load2<false>(const double* __restrict__ U, const double* __restrict__, size_t i) { return U[i]; }
template <> DEV dual load2<true>(const double* __restrict__ U, const double* __restrict__ V, size_t i) {
  return dual(U[i], V[i]);
}

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// ------------------------------------------------------------------ physics
// Conserved variables U = (rho, rho*u_1..d, rho*E); perfect gas.
template <class T, int DIM>
DEV void primitives(const T* U, double gd, T& rinv, T* u, T& p) {
  using R = typename RealOf<T>::type;
  const R g = (R)gd;
  rinv = R(1) / U[0];
  T ke = R(0);
  for (int j = 0; j < DIM; ++j) {
    u[j] = U[1 + j] * rinv;
    ke += U[1 + j] * u[j];
  }
  p = (g - R(1)) * (U[DIM + 1] - R(0.5) * ke);
}

// Convective flux in direction P: (rho u_P, rho u_P u + p e_P, u_P (rho E + p)).
template <class T, int DIM>
DEV void conv_flux_dir(const T* U, const T* u, const T& p, int P, T* F) {
  F[0] = U[1 + P];
  for (int j = 0; j < DIM; ++j) F[1 + j] = U[1 + P] * u[j];
  F[1 + P] += p;
  F[DIM + 1] = u[P] * (U[DIM + 1] + p);
}

// Numerical convective flux across a face of unit normal +e_P, L -> R.
template <class T, int DIM>
DEV void num_flux(const T* UL, const T* UR, int P, const Phys& ph, T* H) {
  using R = typename RealOf<T>::type;
  constexpr int NV = DIM + 2;
  const R g = (R)ph.gamma;
  T rinvL, uL[DIM], pL, rinvR, uR[DIM], pR;
  primitives<T, DIM>(UL, g, rinvL, uL, pL);
  primitives<T, DIM>(UR, g, rinvR, uR, pR);
  T FL[NV], FR[NV];
  conv_flux_dir<T, DIM>(UL, uL, pL, P, FL);
  conv_flux_dir<T, DIM>(UR, uR, pR, P, FR);
  for (int c = 0; c < NV; ++c) H[c] = R(0.5) * (FL[c] + FR[c]);
  if (ph.flux == DG_FLUX_LF) {
    // Lax-Friedrichs with the larger of the two normal wave speeds.
    T cL = dsqrt(g * pL * rinvL), cR = dsqrt(g * pR * rinvR);
    T lam = rmax(rabs(uL[P]) + cL, rabs(uR[P]) + cR);
    for (int c = 0; c < NV; ++c) H[c] -= R(0.5) * lam * (UR[c] - UL[c]);
    return;
  }
  // Roe: |A~|(U_R - U_L) as a sum of waves, Harten entropy fix on every wave.
  T sL = dsqrt(UL[0]), sR = dsqrt(UR[0]);
  T HL = (UL[DIM + 1] + pL) * rinvL, HR = (UR[DIM + 1] + pR) * rinvR;
  T iw = R(1) / (sL + sR);
  T ut[DIM], q2 = R(0);
  for (int j = 0; j < DIM; ++j) {
    ut[j] = (sL * uL[j] + sR * uR[j]) * iw;
    q2 += ut[j] * ut[j];
  }
  T Ht = (sL * HL + sR * HR) * iw;
  T ct2 = (g - R(1)) * (Ht - R(0.5) * q2);
  T ct = dsqrt(ct2);
  T ict2 = R(1) / ct2;
  T unt = ut[P];
  T rhot = sL * sR;
  T dr = UR[0] - UL[0];
  T dp = pR - pL;
  T du[DIM];
  for (int j = 0; j < DIM; ++j) du[j] = uR[j] - uL[j];
  T dun = du[P];
  T a1 = (dp - rhot * ct * dun) * (R(0.5) * ict2);
  T a5 = (dp + rhot * ct * dun) * (R(0.5) * ict2);
  T a2 = dr - dp * ict2;
  T delta = (R)ph.efix * (rabs(unt) + ct);
  auto fix = [&](T lam) {
    T al = rabs(lam);
    return val(al) < val(delta) ? (lam * lam + delta * delta) / (R(2) * delta) : al;
  };
  T l1 = fix(unt - ct), l2 = fix(unt), l5 = fix(unt + ct);
  T w1 = l1 * a1, w5 = l5 * a5, w2 = l2 * a2;
  T sh = R(0);  // u~ . du_t
  H[0] -= R(0.5) * (w1 + w2 + w5);
  for (int j = 0; j < DIM; ++j) {
    T dut = (j == P) ? T(R(0)) : du[j];
    sh += ut[j] * dut;
    T dj = w1 * ut[j] + w2 * ut[j] + l2 * rhot * dut + w5 * ut[j];
    if (j == P) dj += (w5 - w1) * ct;
    H[1 + j] -= R(0.5) * dj;
  }
  T de = w1 * (Ht - ct * unt) + w2 * (R(0.5) * q2) + l2 * rhot * sh + w5 * (Ht + ct * unt);
  H[DIM + 1] -= R(0.5) * de;
}

// Numerical convective flux across a face of unit normal n (any direction),
// L -> R: the same Lax-Friedrichs / Roe construction as num_flux with the
// normal velocity u.n and the tangential velocity jump du - (du.n) n.
template <class T, int DIM>
DEV void num_flux_n(const T* UL, const T* UR, const double* n, const Phys& ph, T* H) {
  using R = typename RealOf<T>::type;
  constexpr int NV = DIM + 2;
  const R g = (R)ph.gamma;
  T rinvL, uL[DIM], pL, rinvR, uR[DIM], pR;
  primitives<T, DIM>(UL, g, rinvL, uL, pL);
  primitives<T, DIM>(UR, g, rinvR, uR, pR);
  T unL = R(0), unR = R(0);
  for (int j = 0; j < DIM; ++j) {
    unL += uL[j] * (R)n[j];
    unR += uR[j] * (R)n[j];
  }
  H[0] = R(0.5) * (UL[0] * unL + UR[0] * unR);
  for (int j = 0; j < DIM; ++j) H[1 + j] = R(0.5) * (UL[1 + j] * unL + UR[1 + j] * unR + (pL + pR) * (R)n[j]);
  H[DIM + 1] = R(0.5) * (unL * (UL[DIM + 1] + pL) + unR * (UR[DIM + 1] + pR));
  if (ph.flux == DG_FLUX_LF) {
    T cL = dsqrt(g * pL * rinvL), cR = dsqrt(g * pR * rinvR);
    T lam = rmax(rabs(unL) + cL, rabs(unR) + cR);
    for (int c = 0; c < NV; ++c) H[c] -= R(0.5) * lam * (UR[c] - UL[c]);
    return;
  }
  T sL = dsqrt(UL[0]), sR = dsqrt(UR[0]);
  T HL = (UL[DIM + 1] + pL) * rinvL, HR = (UR[DIM + 1] + pR) * rinvR;
  T iw = R(1) / (sL + sR);
  T ut[DIM], q2 = R(0), unt = R(0);
  for (int j = 0; j < DIM; ++j) {
    ut[j] = (sL * uL[j] + sR * uR[j]) * iw;
    q2 += ut[j] * ut[j];
    unt += ut[j] * (R)n[j];
  }
  T Ht = (sL * HL + sR * HR) * iw;
  T ct2 = (g - R(1)) * (Ht - R(0.5) * q2);
  T ct = dsqrt(ct2);
  T ict2 = R(1) / ct2;
  T rhot = sL * sR;
  T dr = UR[0] - UL[0];
  T dp = pR - pL;
  T du[DIM], dun = R(0);
  for (int j = 0; j < DIM; ++j) {
    du[j] = uR[j] - uL[j];
    dun += du[j] * (R)n[j];
  }
  T a1 = (dp - rhot * ct * dun) * (R(0.5) * ict2);
  T a5 = (dp + rhot * ct * dun) * (R(0.5) * ict2);
  T a2 = dr - dp * ict2;
  T delta = (R)ph.efix * (rabs(unt) + ct);
  auto fix = [&](T lam) {
    T al = rabs(lam);
    return val(al) < val(delta) ? (lam * lam + delta * delta) / (R(2) * delta) : al;
  };
  T l1 = fix(unt - ct), l2 = fix(unt), l5 = fix(unt + ct);
  T w1 = l1 * a1, w5 = l5 * a5, w2 = l2 * a2;
  T sh = R(0);  // u~ . du_t
  H[0] -= R(0.5) * (w1 + w2 + w5);
  for (int j = 0; j < DIM; ++j) {
    T dut = du[j] - dun * (R)n[j];
    sh += ut[j] * dut;
    T dj = (w1 + w2 + w5) * ut[j] + l2 * rhot * dut + (w5 - w1) * ct * (R)n[j];
    H[1 + j] -= R(0.5) * dj;
  }
  T de = w1 * (Ht - ct * unt) + w2 * (R(0.5) * q2) + l2 * rhot * sh + w5 * (Ht + ct * unt);
  H[DIM + 1] -= R(0.5) * de;
}

// Velocity and p/rho gradients from the corrected conservative gradient G[c][j].
template <class T, int DIM>
struct ViscPrep {
  T u[DIM];
  T gu[DIM][DIM];  // d u_i / d x_j
  T gpr[DIM];      // d (p/rho) / d x_j
  T div;
};

template <class T, int DIM>
DEV void visc_prep(const T* U, const T (*G)[DIM], double gd, ViscPrep<T, DIM>& vp) {
  using R = typename RealOf<T>::type;
  const R g = (R)gd;
  T rinv = R(1) / U[0];
  for (int i = 0; i < DIM; ++i) vp.u[i] = U[1 + i] * rinv;
  T e = U[DIM + 1] * rinv;
  vp.div = R(0);
  for (int j = 0; j < DIM; ++j) {
    T s = R(0);
    for (int i = 0; i < DIM; ++i) {
      vp.gu[i][j] = (G[1 + i][j] - vp.u[i] * G[0][j]) * rinv;
      s += vp.u[i] * vp.gu[i][j];
    }
    T ge = (G[DIM + 1][j] - e * G[0][j]) * rinv;
    vp.gpr[j] = (g - R(1)) * (ge - s);
  }
  for (int i = 0; i < DIM; ++i) vp.div += vp.gu[i][i];
}

// Viscous flux in direction P: (0, tau_P., sum_j tau_Pj u_j + kappa d_P(p/rho)),
// tau = mu (grad u + grad u^T - 2/3 div u I), kappa = mu gamma / (Pr (gamma-1)).
template <class T, int DIM>
DEV void visc_flux_dir(const ViscPrep<T, DIM>& vp, int P, double mud, double kapd, T* Fv) {
  using R = typename RealOf<T>::type;
  const R mu = (R)mud, kap = (R)kapd;
  Fv[0] = R(0);
  T work = R(0);
  for (int j = 0; j < DIM; ++j) {
    T tau = mu * (vp.gu[j][P] + vp.gu[P][j]);
    if (j == P) tau -= (R(2) / R(3)) * mu * vp.div;
    Fv[1 + j] = tau;
    work += tau * vp.u[j];
  }
  Fv[DIM + 1] = work + kap * vp.gpr[P];
}


// ------------------------------------------------------------------ physics policies
// The reference kernels take the pointwise physics as a policy: the number of
// variables, how many of them carry a time derivative (the mass form of the
// implicit operator: a prefix of the variables), the volume flux F_j = F^c_j -
// F^v_j of every direction j, and the face flux H^c - F^v . e_P.
struct CompressiblePhys {
  template <int DIM> static constexpr int nv() { return DIM + 2; }
  template <int DIM> static constexpr int nmass() { return DIM + 2; }
  template <class T, int DIM>
  static DEV void volume_flux(const T* u, const T (*G)[DIM], const Phys& ph, T (*F)[DIM + 2]) {
    const double kap = ph.mu * ph.gamma / (ph.prandtl * (ph.gamma - 1.0));
    T rinv, vel[DIM], pr;
    primitives<T, DIM>(u, ph.gamma, rinv, vel, pr);
    ViscPrep<T, DIM> vp;
    visc_prep<T, DIM>(u, G, ph.gamma, vp);
    for (int j = 0; j < DIM; ++j) {
      T Fc[DIM + 2], Fv[DIM + 2];
      conv_flux_dir<T, DIM>(u, vel, pr, j, Fc);
      visc_flux_dir<T, DIM>(vp, j, ph.mu, kap, Fv);
      for (int c = 0; c < DIM + 2; ++c) F[j][c] = Fc[c] - Fv[c];
    }
  }
  template <class T, int DIM>
  static DEV void face_flux(const T* uL, const T* uR, const T* ua, const T (*Ga)[DIM], int P, const Phys& ph,
                            T* Hn) {
    const double kap = ph.mu * ph.gamma / (ph.prandtl * (ph.gamma - 1.0));
    num_flux<T, DIM>(uL, uR, P, ph, Hn);
    ViscPrep<T, DIM> vp;
    visc_prep<T, DIM>(ua, Ga, ph.gamma, vp);
    T Fv[DIM + 2];
    visc_flux_dir<T, DIM>(vp, P, ph.mu, kap, Fv);
    for (int c = 0; c < DIM + 2; ++c) Hn[c] = Hn[c] - Fv[c];
  }
};

// Incompressible Navier-Stokes (Sec. 2.1, eq. ns): w = (u_1..u_d, p), unit
// density; F_j = (u_j u + p e_j, u_j) - (nu (grad u + grad u^T - 2/3 div u I)_j., 0);
// only the velocities carry a time derivative (eq. massBil).  Interface flux:
// Lax-Friedrichs of the artificial compressibility system
// (1/beta^2) dp/dt + div u = 0 (the paper's exact Riemann solver of that
// system is defined in a cited work only): mean normal flux minus
// lambda/2 diag(1,..,1, 1/beta^2) (w_R - w_L), lambda = max over both sides of
// |u.n| + sqrt((u.n)^2 + beta^2).
struct IncompressiblePhys {
  template <int DIM> static constexpr int nv() { return DIM + 1; }
  template <int DIM> static constexpr int nmass() { return DIM; }
  template <class T, int DIM>
  static DEV void visc_dir(const T (*G)[DIM], int P, double nud, T* Fv) {
    using R = typename RealOf<T>::type;
    const R nu = (R)nud;
    T div = R(0);
    for (int i = 0; i < DIM; ++i) div += G[i][i];
    for (int i = 0; i < DIM; ++i) {
      T t = nu * (G[P][i] + G[i][P]);
      if (i == P) t -= (R(2) / R(3)) * nu * div;
      Fv[i] = t;
    }
    Fv[DIM] = R(0);
  }
  template <class T, int DIM>
  static DEV void volume_flux(const T* u, const T (*G)[DIM], const Phys& ph, T (*F)[DIM + 1]) {
    for (int j = 0; j < DIM; ++j) {
      T Fv[DIM + 1];
      visc_dir<T, DIM>(G, j, ph.mu, Fv);
      for (int i = 0; i < DIM; ++i) F[j][i] = u[j] * u[i] - Fv[i];
      F[j][j] += u[DIM];
      F[j][DIM] = u[j];
    }
  }
  template <class T, int DIM>
  static DEV void face_flux(const T* uL, const T* uR, const T* ua, const T (*Ga)[DIM], int P, const Phys& ph,
                            T* Hn) {
    using R = typename RealOf<T>::type;
    const R b2 = (R)(ph.beta * ph.beta);
    const T unL = uL[P], unR = uR[P];
    const T lam = rmax(rabs(unL) + dsqrt(unL * unL + b2), rabs(unR) + dsqrt(unR * unR + b2));
    T Fv[DIM + 1];
    visc_dir<T, DIM>(Ga, P, ph.mu, Fv);
    for (int i = 0; i < DIM; ++i)
      Hn[i] = R(0.5) * (uL[i] * unL + uR[i] * unR) - R(0.5) * lam * (uR[i] - uL[i]) - Fv[i];
    Hn[P] += R(0.5) * (uL[DIM] + uR[DIM]);
    Hn[DIM] = R(0.5) * (unL + unR) - (R(0.5) / b2) * lam * (uR[DIM] - uL[DIM]);
  }
};

// Scalar diffusion (the BR2 Laplacian of the paper's Poisson assessment, App.
// B): one variable, F^c = 0, F^v = mu grad u (corrected gradient), face flux
// -mu ({grad u} + eta {r}) . e_P.
struct DiffusionPhys {
  template <int DIM> static constexpr int nv() { return 1; }
  template <int DIM> static constexpr int nmass() { return 1; }
  template <class T, int DIM>
  static DEV void volume_flux(const T* u, const T (*G)[DIM], const Phys& ph, T (*F)[1]) {
    using R = typename RealOf<T>::type;
    for (int j = 0; j < DIM; ++j) F[j][0] = -(R)ph.mu * G[0][j];
  }
  template <class T, int DIM>
  static DEV void face_flux(const T* uL, const T* uR, const T* ua, const T (*Ga)[DIM], int P, const Phys& ph,
                            T* Hn) {
    using R = typename RealOf<T>::type;
    Hn[0] = -(R)ph.mu * Ga[0][P];
  }
};

}  // namespace dgk
