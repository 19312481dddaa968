// DG residual and exact Jv on curved (multilinear) elements (Sec. 2.1-2.2,
// eq. NSdiscrRes): per-element and per-face basis tables (each element's own
// orthonormalised basis, physical gradients, Nanson normals and area
// weights) read from memory, pointwise fluxes on the vector ALU in FP64
// (dual numbers for Jv).
//
// Pass 1, one workgroup per face (p, e) (owner e, neighbour across its +p
// face): traces of both sides, the local BR2 lifting coefficients of both
// sides, rho^{S}_{c,j,b} = -1/2 sum_f w_f|J_f| [[U_c]] n_j phi^S_b, the face
// flux Hn = H^c(U_L, U_R, n) - F^v({U}, {grad U} + eta {r}) . n, and its
// projection w_f|J_f| Hn phi^S_b on each side.
// Pass 2, one workgroup per element: the elemental lifting R^K (sum of the
// local liftings of its 2d faces), the volume flux at the volume points with
// G = grad U + R^K, its projection on the physical gradients of the basis,
// plus the gathered face projections (+ on the owner side, - on the
// neighbour side).
#include "dg_device.h"

namespace dgk {

namespace {

template <int DIM, int NB, int NQ1, bool JVP>
__global__ __launch_bounds__(64) void k_face_curved(const double* __restrict__ U, const double* __restrict__ V,
                                                    CurvedTables ct, Mesh m, Phys ph) {
  using T = typename Scalar<JVP>::type;
  constexpr int NV = DIM + 2, NFQ = ipow(NQ1, DIM - 1), NS = JVP ? 2 : 1;
  static_assert(NFQ <= 64, "one thread per face point");
  __shared__ double sU[NS][2][NV][NB];
  __shared__ double sJ[NS][NFQ][NV];
  __shared__ double sRho[NS][2][NV][DIM][NB];
  __shared__ double sH[NFQ][NV];
  const int tid = threadIdx.x;
  const int P = blockIdx.y;
  const int64_t ne = m.ne;
  const int64_t e = blockIdx.x;
  const int64_t er = m.nbr[(size_t)(2 * P + 1) * ne + e];
  const size_t f = (size_t)P * ne + e;
  const double kap = ph.mu * ph.gamma / (ph.prandtl * (ph.gamma - 1.0));

  for (int i = tid; i < NS * 2 * NV * NB; i += 64) {
    const int b = i % NB, c = (i / NB) % NV, side = (i / (NB * NV)) % 2, s = i / (2 * NV * NB);
    const double* X = s == 0 ? U : V;
    sU[s][side][c][b] = X[(size_t)(c * NB + b) * ne + (side == 0 ? e : er)];
  }
  __syncthreads();

  // traces at face point fq = tid
  T uL[NV], uR[NV], gL[NV][DIM], gR[NV][DIM];
  if (tid < NFQ) {
    const double* phL = ct.fPhiL + (f * NFQ + tid) * NB;
    const double* phR = ct.fPhiR + (f * NFQ + tid) * NB;
    const double* gpL = ct.fGPhiL + (f * NFQ + tid) * DIM * NB;
    const double* gpR = ct.fGPhiR + (f * NFQ + tid) * DIM * NB;
    for (int c = 0; c < NV; ++c) {
      T a = 0.0, r = 0.0, ga[DIM], gr[DIM];
      for (int j = 0; j < DIM; ++j) {
        ga[j] = 0.0;
        gr[j] = 0.0;
      }
#pragma unroll 1
      for (int b = 0; b < NB; ++b) {
        T xl, xr;
        if constexpr (JVP) {
          xl = T(sU[0][0][c][b], sU[NS - 1][0][c][b]);
          xr = T(sU[0][1][c][b], sU[NS - 1][1][c][b]);
        } else {
          xl = sU[0][0][c][b];
          xr = sU[0][1][c][b];
        }
        a += phL[b] * xl;
        r += phR[b] * xr;
        for (int j = 0; j < DIM; ++j) {
          ga[j] += gpL[j * NB + b] * xl;
          gr[j] += gpR[j * NB + b] * xr;
        }
      }
      uL[c] = a;
      uR[c] = r;
      for (int j = 0; j < DIM; ++j) {
        gL[c][j] = ga[j];
        gR[c][j] = gr[j];
      }
      const T jmp = a - r;
      sJ[0][tid][c] = val(jmp);
      if constexpr (JVP) sJ[NS - 1][tid][c] = out_part(jmp);
    }
    if constexpr (JVP) {
      if (ph.stab_only) {  // tangent through the face lifting term only
        for (int c = 0; c < NV; ++c) {
          uL[c].d = 0.0;
          uR[c].d = 0.0;
          for (int j = 0; j < DIM; ++j) {
            gL[c][j].d = 0.0;
            gR[c][j].d = 0.0;
          }
        }
      }
    }
  }
  __syncthreads();

  // local lifting coefficients of both sides
  for (int i = tid; i < 2 * NV * DIM * NB; i += 64) {
    const int b = i % NB, j = (i / NB) % DIM, c = (i / (NB * DIM)) % NV, side = i / (NB * DIM * NV);
    const double* tb = side == 0 ? ct.fPhiL : ct.fPhiR;
    double sv = 0.0, st = 0.0;
    for (int fq = 0; fq < NFQ; ++fq) {
      const double wn = ct.fW[f * NFQ + fq] * ct.fN[(f * NFQ + fq) * DIM + j] * tb[(f * NFQ + fq) * NB + b];
      sv += wn * sJ[0][fq][c];
      if (JVP) st += wn * sJ[NS - 1][fq][c];
    }
    sRho[0][side][c][j][b] = -0.5 * sv;
    if (JVP) sRho[NS - 1][side][c][j][b] = -0.5 * st;
    double* out = ct.fRho + (f * 2 * 2 + 0 * 2 + side) * NV * DIM * NB;
    out[(c * DIM + j) * NB + b] = -0.5 * sv;
    double* outt = ct.fRho + (f * 2 * 2 + 1 * 2 + side) * NV * DIM * NB;
    outt[(c * DIM + j) * NB + b] = (JVP && !ph.stab_only) ? -0.5 * st : 0.0;
  }
  __syncthreads();

  // face flux at face point fq = tid
  if (tid < NFQ) {
    const double* phL = ct.fPhiL + (f * NFQ + tid) * NB;
    const double* phR = ct.fPhiR + (f * NFQ + tid) * NB;
    const double* n = ct.fN + (f * NFQ + tid) * DIM;
    T ua[NV], Ga[NV][DIM];
    for (int c = 0; c < NV; ++c) {
      ua[c] = 0.5 * (uL[c] + uR[c]);
      for (int j = 0; j < DIM; ++j) {
        T rl = 0.0, rr = 0.0;
#pragma unroll 1
        for (int b = 0; b < NB; ++b) {
          if constexpr (JVP) {
            rl += phL[b] * T(sRho[0][0][c][j][b], sRho[NS - 1][0][c][j][b]);
            rr += phR[b] * T(sRho[0][1][c][j][b], sRho[NS - 1][1][c][j][b]);
          } else {
            rl += phL[b] * sRho[0][0][c][j][b];
            rr += phR[b] * sRho[0][1][c][j][b];
          }
        }
        Ga[c][j] = 0.5 * (gL[c][j] + gR[c][j]) + ph.eta * (0.5 * (rl + rr));
      }
    }
    T Hn[NV];
    num_flux_n<T, DIM>(uL, uR, n, ph, Hn);
    ViscPrep<T, DIM> vp;
    visc_prep<T, DIM>(ua, Ga, ph.gamma, vp);
    for (int j = 0; j < DIM; ++j) {
      T Fv[NV];
      visc_flux_dir<T, DIM>(vp, j, ph.mu, kap, Fv);
      for (int c = 0; c < NV; ++c) Hn[c] -= n[j] * Fv[c];
    }
    const double w = ct.fW[f * NFQ + tid];
    for (int c = 0; c < NV; ++c) sH[tid][c] = w * out_part(Hn[c]);
  }
  __syncthreads();

  // projection on both sides
  for (int i = tid; i < 2 * NV * NB; i += 64) {
    const int b = i % NB, c = (i / NB) % NV, side = i / (NB * NV);
    const double* tb = side == 0 ? ct.fPhiL : ct.fPhiR;
    double s = 0.0;
    for (int fq = 0; fq < NFQ; ++fq) s += sH[fq][c] * tb[(f * NFQ + fq) * NB + b];
    ct.fProj[((f * 2 + side) * NV + c) * NB + b] = s;
  }
}

template <int DIM, int NB, int NQ1, bool JVP>
__global__ __launch_bounds__(128) void k_volume_curved(const double* __restrict__ U, const double* __restrict__ V,
                                                      CurvedTables ct, double* __restrict__ out, double shift,
                                                      Mesh m, Phys ph) {
  using T = typename Scalar<JVP>::type;
  constexpr int NV = DIM + 2, NQ = ipow(NQ1, DIM), NS = JVP ? 2 : 1;
  static_assert(NQ <= 128, "one thread per volume point");
  __shared__ double sU[NS][NV][NB];
  __shared__ double sR[NS][NV][DIM][NB];
  __shared__ double sF[NQ][DIM][NV];
  const int tid = threadIdx.x;
  const int64_t ne = m.ne;
  const int64_t e = blockIdx.x;
  const double kap = ph.mu * ph.gamma / (ph.prandtl * (ph.gamma - 1.0));

  for (int i = tid; i < NS * NV * NB; i += 128) {
    const int b = i % NB, c = (i / NB) % NV, s = i / (NB * NV);
    sU[s][c][b] = (s == 0 ? U : V)[(size_t)(c * NB + b) * ne + e];
  }
  // elemental lifting: owner side of the +p faces, neighbour side of the -p faces
  for (int i = tid; i < NS * NV * DIM * NB; i += 128) {
    const int b = i % NB, j = (i / NB) % DIM, c = (i / (NB * DIM)) % NV, s = i / (NB * DIM * NV);
    double a = 0.0;
    for (int p = 0; p < DIM; ++p) {
      const size_t fo = (size_t)p * ne + e;
      const size_t fm = (size_t)p * ne + m.nbr[(size_t)(2 * p) * ne + e];
      a += ct.fRho[((fo * 2 + s) * 2 + 0) * NV * DIM * NB + (c * DIM + j) * NB + b];
      a += ct.fRho[((fm * 2 + s) * 2 + 1) * NV * DIM * NB + (c * DIM + j) * NB + b];
    }
    sR[s][c][j][b] = a;
  }
  __syncthreads();

  if (tid < NQ) {
    const double* phi = ct.vPhi + ((size_t)e * NQ + tid) * NB;
    const double* gphi = ct.vGPhi + ((size_t)e * NQ + tid) * DIM * NB;
    T u[NV], G[NV][DIM];
    for (int c = 0; c < NV; ++c) {
      T a = 0.0, g[DIM];
      for (int j = 0; j < DIM; ++j) g[j] = 0.0;
#pragma unroll 1
      for (int b = 0; b < NB; ++b) {
        T x;
        if constexpr (JVP)
          x = T(sU[0][c][b], sU[NS - 1][c][b]);
        else
          x = sU[0][c][b];
        a += phi[b] * x;
        for (int j = 0; j < DIM; ++j) {
          T rk;
          if constexpr (JVP)
            rk = T(sR[0][c][j][b], sR[NS - 1][c][j][b]);
          else
            rk = sR[0][c][j][b];
          g[j] += gphi[j * NB + b] * x + phi[b] * rk;
        }
      }
      u[c] = a;
      for (int j = 0; j < DIM; ++j) G[c][j] = g[j];
    }
    T rinv, vel[DIM], pr;
    primitives<T, DIM>(u, ph.gamma, rinv, vel, pr);
    ViscPrep<T, DIM> vp;
    visc_prep<T, DIM>(u, G, ph.gamma, vp);
    const double w = ct.vW[(size_t)e * NQ + tid];
    for (int j = 0; j < DIM; ++j) {
      T Fc[NV], Fv[NV];
      conv_flux_dir<T, DIM>(u, vel, pr, j, Fc);
      visc_flux_dir<T, DIM>(vp, j, ph.mu, kap, Fv);
      for (int c = 0; c < NV; ++c) sF[tid][j][c] = w * out_part(Fc[c] - Fv[c]);
    }
  }
  __syncthreads();

  for (int i = tid; i < NV * NB; i += 128) {
    const int b = i % NB, c = i / NB;
    double a = 0.0;
    for (int q = 0; q < NQ; ++q) {
      const double* gphi = ct.vGPhi + ((size_t)e * NQ + q) * DIM * NB;
      for (int j = 0; j < DIM; ++j) a -= sF[q][j][c] * gphi[j * NB + b];
    }
    for (int p = 0; p < DIM; ++p) {
      const size_t fo = (size_t)p * ne + e;
      const size_t fm = (size_t)p * ne + m.nbr[(size_t)(2 * p) * ne + e];
      a += ct.fProj[((fo * 2 + 0) * NV + c) * NB + b];
      a -= ct.fProj[((fm * 2 + 1) * NV + c) * NB + b];
    }
    const size_t idx = (size_t)(c * NB + b) * ne + e;
    if (JVP) a += shift * V[idx];
    out[idx] = a;
  }
}

template <int DIM, int NB, int NQ1>
__global__ void k_project_curved(const double* __restrict__ f, double* __restrict__ w, CurvedTables ct, int64_t ne) {
  constexpr int NV = DIM + 2, NQ = ipow(NQ1, DIM);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)NV * NB * ne) return;
  const int64_t e = i % ne;
  const int cb = (int)(i / ne), c = cb / NB, b = cb % NB;
  double a = 0.0;
  for (int q = 0; q < NQ; ++q)
    a += ct.vW[(size_t)e * NQ + q] * ct.vPhi[((size_t)e * NQ + q) * NB + b] * f[((size_t)c * NQ + q) * ne + e];
  w[i] = a;
}

template <int DIM, int NB, int NQ1>
__global__ __launch_bounds__(256) void k_wave_speed_curved(const double* __restrict__ w, double* __restrict__ partial,
                                                           CurvedTables ct, Mesh m, Phys ph) {
  constexpr int NV = DIM + 2, NQ = ipow(NQ1, DIM);
  __shared__ double red[256];
  double mx = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < (int64_t)NQ * m.ne; i += (int64_t)gridDim.x * 256) {
    const int64_t e = i % m.ne;
    const int q = (int)(i / m.ne);
    const double* phi = ct.vPhi + ((size_t)e * NQ + q) * NB;
    double u[NV];
    for (int c = 0; c < NV; ++c) {
      double a = 0.0;
      for (int b = 0; b < NB; ++b) a += phi[b] * w[((size_t)c * NB + b) * m.ne + e];
      u[c] = a;
    }
    double rinv, vel[DIM], p;
    primitives<double, DIM>(u, ph.gamma, rinv, vel, p);
    double s = 0.0;
    for (int j = 0; j < DIM; ++j) s += vel[j] * vel[j];
    const double a = sqrt(s) + sqrt(ph.gamma * p * rinv);
    mx = (a > mx || a != a) ? a : mx;
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      const double o = red[threadIdx.x + st];
      if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

}  // namespace

// (cfg id, dim, nb, nq1d): the configurations of the affine kernels
#define DG_CURVED_CONFIGS(X) \
  X(0, 2, 9, 4)              \
  X(1, 2, 6, 4)              \
  X(2, 3, 4, 2)              \
  X(3, 3, 10, 3)             \
  X(4, 3, 20, 4)             \
  X(5, 3, 35, 5)

hipError_t launch_face_curved(int cfg, bool jvp, const double* U, const double* V, const CurvedTables& ct,
                              const Mesh& m, const Phys& ph, hipStream_t s) {
#define X(id, d, nb_, nq_)                                                          \
  case id: {                                                                        \
    dim3 grid((unsigned)m.ne, d);                                                   \
    if (jvp)                                                                        \
      k_face_curved<d, nb_, nq_, true><<<grid, 64, 0, s>>>(U, V, ct, m, ph);        \
    else                                                                            \
      k_face_curved<d, nb_, nq_, false><<<grid, 64, 0, s>>>(U, V, ct, m, ph);       \
    return hipGetLastError();                                                       \
  }
  switch (cfg) { DG_CURVED_CONFIGS(X) }
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_volume_curved(int cfg, bool jvp, const double* U, const double* V, const CurvedTables& ct,
                                double* out, double shift, const Mesh& m, const Phys& ph, hipStream_t s) {
#define X(id, d, nb_, nq_)                                                                           \
  case id: {                                                                                         \
    if (jvp)                                                                                         \
      k_volume_curved<d, nb_, nq_, true><<<(unsigned)m.ne, 128, 0, s>>>(U, V, ct, out, shift, m, ph);  \
    else                                                                                             \
      k_volume_curved<d, nb_, nq_, false><<<(unsigned)m.ne, 128, 0, s>>>(U, V, ct, out, shift, m, ph); \
    return hipGetLastError();                                                                        \
  }
  switch (cfg) { DG_CURVED_CONFIGS(X) }
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_project_curved(int cfg, const double* f, double* w, const CurvedTables& ct, int64_t ne,
                                 hipStream_t s) {
#define X(id, d, nb_, nq_)                                                                             \
  case id: {                                                                                           \
    const int64_t n = (int64_t)(d + 2) * nb_ * ne;                                                     \
    k_project_curved<d, nb_, nq_><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(f, w, ct, ne);           \
    return hipGetLastError();                                                                          \
  }
  switch (cfg) { DG_CURVED_CONFIGS(X) }
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_wave_speed_curved(int cfg, const double* w, double* partial, int nblocks, const CurvedTables& ct,
                                    const Mesh& m, const Phys& ph, hipStream_t s) {
#define X(id, d, nb_, nq_)                                                                    \
  case id: {                                                                                  \
    k_wave_speed_curved<d, nb_, nq_><<<nblocks, 256, 0, s>>>(w, partial, ct, m, ph);          \
    return hipGetLastError();                                                                 \
  }
  switch (cfg) { DG_CURVED_CONFIGS(X) }
#undef X
  return hipErrorInvalidValue;
}

}  // namespace dgk
