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
struct dual {
  double v, d;
  DEV dual() = default;
  DEV dual(double x) : v(x), d(0.0) {}
  DEV dual(double x, double y) : v(x), d(y) {}
};
DEV dual operator+(dual a, dual b) { return dual(a.v + b.v, a.d + b.d); }
DEV dual operator-(dual a, dual b) { return dual(a.v - b.v, a.d - b.d); }
DEV dual operator*(dual a, dual b) { return dual(a.v * b.v, a.d * b.v + a.v * b.d); }
DEV dual operator/(dual a, dual b) {
  double q = a.v / b.v;
  return dual(q, (a.d - q * b.d) / b.v);
}
DEV dual operator-(dual a) { return dual(-a.v, -a.d); }
DEV dual operator*(double s, dual a) { return dual(s * a.v, s * a.d); }
DEV dual operator*(dual a, double s) { return dual(s * a.v, s * a.d); }
DEV dual operator+(dual a, double s) { return dual(a.v + s, a.d); }
DEV dual operator+(double s, dual a) { return dual(a.v + s, a.d); }
DEV dual operator-(dual a, double s) { return dual(a.v - s, a.d); }
DEV dual operator-(double s, dual a) { return dual(s - a.v, -a.d); }
DEV dual operator/(dual a, double s) { return dual(a.v / s, a.d / s); }
DEV dual operator/(double s, dual a) {
  double q = s / a.v;
  return dual(q, -q * a.d / a.v);
}
DEV dual& operator+=(dual& a, dual b) { a = a + b; return a; }
DEV dual& operator-=(dual& a, dual b) { a = a - b; return a; }
DEV dual dsqrt(dual a) {
  double r = sqrt(a.v);
  return dual(r, 0.5 * a.d / r);
}
DEV double dsqrt(double a) { return sqrt(a); }
DEV double val(double a) { return a; }
DEV double val(dual a) { return a.v; }
DEV double out_part(double a) { return a; }
DEV double out_part(dual a) { return a.d; }
template <class T> DEV T rabs(T a) { return val(a) >= 0.0 ? a : -a; }
template <class T> DEV T rmax(T a, T b) { return val(a) >= val(b) ? a : b; }

template <bool JVP> struct Scalar { using type = double; };
template <> struct Scalar<true> { using type = dual; };

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
DEV void primitives(const T* U, double g, T& rinv, T* u, T& p) {
  rinv = 1.0 / U[0];
  T ke = 0.0;
  for (int j = 0; j < DIM; ++j) {
    u[j] = U[1 + j] * rinv;
    ke += U[1 + j] * u[j];
  }
  p = (g - 1.0) * (U[DIM + 1] - 0.5 * ke);
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
  constexpr int NV = DIM + 2;
  const double g = ph.gamma;
  T rinvL, uL[DIM], pL, rinvR, uR[DIM], pR;
  primitives<T, DIM>(UL, g, rinvL, uL, pL);
  primitives<T, DIM>(UR, g, rinvR, uR, pR);
  T FL[NV], FR[NV];
  conv_flux_dir<T, DIM>(UL, uL, pL, P, FL);
  conv_flux_dir<T, DIM>(UR, uR, pR, P, FR);
  for (int c = 0; c < NV; ++c) H[c] = 0.5 * (FL[c] + FR[c]);
  if (ph.flux == DG_FLUX_LF) {
    // Lax-Friedrichs with the larger of the two normal wave speeds.
    T cL = dsqrt(g * pL * rinvL), cR = dsqrt(g * pR * rinvR);
    T lam = rmax(rabs(uL[P]) + cL, rabs(uR[P]) + cR);
    for (int c = 0; c < NV; ++c) H[c] -= 0.5 * lam * (UR[c] - UL[c]);
    return;
  }
  // Roe: |A~|(U_R - U_L) as a sum of waves, Harten entropy fix on every wave.
  T sL = dsqrt(UL[0]), sR = dsqrt(UR[0]);
  T HL = (UL[DIM + 1] + pL) * rinvL, HR = (UR[DIM + 1] + pR) * rinvR;
  T iw = 1.0 / (sL + sR);
  T ut[DIM], q2 = 0.0;
  for (int j = 0; j < DIM; ++j) {
    ut[j] = (sL * uL[j] + sR * uR[j]) * iw;
    q2 += ut[j] * ut[j];
  }
  T Ht = (sL * HL + sR * HR) * iw;
  T ct2 = (g - 1.0) * (Ht - 0.5 * q2);
  T ct = dsqrt(ct2);
  T ict2 = 1.0 / ct2;
  T unt = ut[P];
  T rhot = sL * sR;
  T dr = UR[0] - UL[0];
  T dp = pR - pL;
  T du[DIM];
  for (int j = 0; j < DIM; ++j) du[j] = uR[j] - uL[j];
  T dun = du[P];
  T a1 = (dp - rhot * ct * dun) * (0.5 * ict2);
  T a5 = (dp + rhot * ct * dun) * (0.5 * ict2);
  T a2 = dr - dp * ict2;
  T delta = ph.efix * (rabs(unt) + ct);
  auto fix = [&](T lam) {
    T al = rabs(lam);
    return val(al) < val(delta) ? (lam * lam + delta * delta) / (2.0 * delta) : al;
  };
  T l1 = fix(unt - ct), l2 = fix(unt), l5 = fix(unt + ct);
  T w1 = l1 * a1, w5 = l5 * a5, w2 = l2 * a2;
  T sh = 0.0;  // u~ . du_t
  H[0] -= 0.5 * (w1 + w2 + w5);
  for (int j = 0; j < DIM; ++j) {
    T dut = (j == P) ? T(0.0) : du[j];
    sh += ut[j] * dut;
    T dj = w1 * ut[j] + w2 * ut[j] + l2 * rhot * dut + w5 * ut[j];
    if (j == P) dj += (w5 - w1) * ct;
    H[1 + j] -= 0.5 * dj;
  }
  T de = w1 * (Ht - ct * unt) + w2 * (0.5 * q2) + l2 * rhot * sh + w5 * (Ht + ct * unt);
  H[DIM + 1] -= 0.5 * de;
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
DEV void visc_prep(const T* U, const T (*G)[DIM], double g, ViscPrep<T, DIM>& vp) {
  T rinv = 1.0 / U[0];
  for (int i = 0; i < DIM; ++i) vp.u[i] = U[1 + i] * rinv;
  T e = U[DIM + 1] * rinv;
  vp.div = 0.0;
  for (int j = 0; j < DIM; ++j) {
    T s = 0.0;
    for (int i = 0; i < DIM; ++i) {
      vp.gu[i][j] = (G[1 + i][j] - vp.u[i] * G[0][j]) * rinv;
      s += vp.u[i] * vp.gu[i][j];
    }
    T ge = (G[DIM + 1][j] - e * G[0][j]) * rinv;
    vp.gpr[j] = (g - 1.0) * (ge - s);
  }
  for (int i = 0; i < DIM; ++i) vp.div += vp.gu[i][i];
}

// Viscous flux in direction P: (0, tau_P., sum_j tau_Pj u_j + kappa d_P(p/rho)),
// tau = mu (grad u + grad u^T - 2/3 div u I), kappa = mu gamma / (Pr (gamma-1)).
template <class T, int DIM>
DEV void visc_flux_dir(const ViscPrep<T, DIM>& vp, int P, double mu, double kap, T* Fv) {
  Fv[0] = 0.0;
  T work = 0.0;
  for (int j = 0; j < DIM; ++j) {
    T tau = mu * (vp.gu[j][P] + vp.gu[P][j]);
    if (j == P) tau -= (2.0 / 3.0) * mu * vp.div;
    Fv[1 + j] = tau;
    work += tau * vp.u[j];
  }
  Fv[DIM + 1] = work + kap * vp.gpr[P];
}


}  // namespace dgk
