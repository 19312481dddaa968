// DG residual and Jacobian-vector product kernels for gfx950 (FP64).
//
// Residual of eq. (NSdiscrRes) (Sec. 2.2):
//   R_Kbc = - sum_q w_q|J| sum_j F_jc(U_q, G_q) d_j phi_b(x_q)
//           + sum_{faces} (+/-) sum_f w_f|J_f| Hn_c(x_f) phi_b(x_f)
// with F = F^c - F^v, the BR2 corrected gradient G = grad U + R^K in the
// volume and the face flux
//   Hn = H^c(U_L, U_R, n) - F^v({U}, {grad U} + eta {r}) . n
// (Sec. 2.1, eq. vflux, with the lifting sign of the consistent gradient).
//
// Two kernels per evaluation:
//   face   : one lane per (face, face point); traces of both sides, averaged
//            local lifting, numerical flux -> Hn at the face points
//            (layout [p][c][fq][e], e = owner element of the +p face).
//   volume : a tile of TE elements per workgroup; modal corrected gradients
//            (derivative + elemental lifting, exact on affine elements),
//            pointwise volume flux, weighted-transpose projection, plus the
//            2*dim face contributions gathered from Hn (no atomics).
// The Jacobian-vector product runs the same kernels on dual numbers
// (value, tangent): forward-mode differentiation of the residual, i.e. the
// Jacobian forms j_h of Sec. 2.2 applied to v.  Branches (|.|, max, entropy
// fix) follow the value part; ties take the first operand.
#include "dg_device.h"

namespace dgk {

// ------------------------------------------------------------------ face kernel
// Body for one face direction p (a compile-time constant, so every index into
// the per-lane arrays is static and nothing spills to scratch).
template <class PHY, int DIM, int NB, int NQ1, bool JVP, int p>
DEV void face_body(const double* __restrict__ U, const double* __restrict__ V, double* __restrict__ H,
                   const Tables& tb, const Mesh& m, const Phys& ph) {
  using T = typename Scalar<JVP>::type;
  constexpr int NV = PHY::template nv<DIM>();
  constexpr int NFQ = ipow(NQ1, DIM - 1);
  const int lane = threadIdx.x & 63;
  const int slot = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t ne = m.ne;
  const int64_t e = (int64_t)blockIdx.x * 64 + lane;
  if (e >= ne) return;
  const int64_t er = m.nbr[(2 * p + 1) * ne + e];
  for (int fq = slot; fq < NFQ; fq += 4) {
    T uL[NV], uR[NV], gL[NV][DIM], gR[NV][DIM], rb[NV];
    for (int c = 0; c < NV; ++c) {
      uL[c] = 0.0;
      uR[c] = 0.0;
      rb[c] = 0.0;
      for (int j = 0; j < DIM; ++j) {
        gL[c][j] = 0.0;
        gR[c][j] = 0.0;
      }
    }
    const double* phP = tb.fPhi + ((size_t)(p * 2 + 1) * NFQ + fq) * NB;
    const double* phM = tb.fPhi + ((size_t)(p * 2 + 0) * NFQ + fq) * NB;
    const double* lfL = tb.fLift + ((size_t)(p * 2 + 0) * NFQ + fq) * NB;
    const double* lfR = tb.fLift + ((size_t)(p * 2 + 1) * NFQ + fq) * NB;
    for (int c = 0; c < NV; ++c) {
#pragma unroll 4
      for (int b = 0; b < NB; ++b) {
        const size_t i = (size_t)(c * NB + b) * ne;
        T a = load2<JVP>(U, V, i + e);
        T r = load2<JVP>(U, V, i + er);
        uL[c] += phP[b] * a;
        uR[c] += phM[b] * r;
        rb[c] += lfL[b] * a + lfR[b] * r;
        for (int j = 0; j < DIM; ++j) {
          gL[c][j] += tb.fDphi[((size_t)((p * 2 + 1) * DIM + j) * NFQ + fq) * NB + b] * a;
          gR[c][j] += tb.fDphi[((size_t)((p * 2 + 0) * DIM + j) * NFQ + fq) * NB + b] * r;
        }
      }
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
    T ua[NV], Ga[NV][DIM];
    for (int c = 0; c < NV; ++c) {
      ua[c] = 0.5 * (uL[c] + uR[c]);
      for (int j = 0; j < DIM; ++j) Ga[c][j] = 0.5 * (gL[c][j] + gR[c][j]);
      Ga[c][p] += ph.eta * rb[c];
    }
    T Hn[NV];
    PHY::template face_flux<T, DIM>(uL, uR, ua, Ga, p, ph, Hn);
    for (int c = 0; c < NV; ++c) H[((size_t)(p * NV + c) * NFQ + fq) * ne + e] = out_part(Hn[c]);
  }
}

template <class PHY, int DIM, int NB, int NQ1, bool JVP>
__global__ __launch_bounds__(256) void k_face(const double* __restrict__ U, const double* __restrict__ V,
                                              double* __restrict__ H, Tables tb, Mesh m, Phys ph) {
  switch (blockIdx.y) {
    case 0: face_body<PHY, DIM, NB, NQ1, JVP, 0>(U, V, H, tb, m, ph); break;
    case 1: face_body<PHY, DIM, NB, NQ1, JVP, 1>(U, V, H, tb, m, ph); break;
    default:
      if constexpr (DIM == 3) face_body<PHY, DIM, NB, NQ1, JVP, 2>(U, V, H, tb, m, ph);
      break;
  }
}

// ------------------------------------------------------------------ volume kernel
template <class PHY, int DIM, int NB, int NQ1, bool JVP, int TE, int QC>
__global__ __launch_bounds__(256) void k_volume(const double* __restrict__ U, const double* __restrict__ V,
                                                const double* __restrict__ H, double* __restrict__ out, double shift,
                                                Tables tb, Mesh m, Phys ph) {
  using T = typename Scalar<JVP>::type;
  constexpr int NV = PHY::template nv<DIM>();
  constexpr int NQ = ipow(NQ1, DIM);
  constexpr int NFQ = ipow(NQ1, DIM - 1);
  constexpr int NS = JVP ? 2 : 1;
  // sX[s][f][c][b][t]: s = value/tangent, f = 0 modal U, f = 1+j modal G_j
  __shared__ double sX[NS][1 + DIM][NV][NB][TE];
  __shared__ double sF[DIM][NV][QC][TE];
  const int tid = threadIdx.x;
  const int64_t ne = m.ne;
  const int64_t e0 = (int64_t)blockIdx.x * TE;

  for (int it = tid; it < NV * NB * TE; it += 256) {
    const int t = it % TE, cb = it / TE;
    const int64_t e = e0 + t;
    double a = 0.0, d = 0.0;
    if (e < ne) {
      a = U[(size_t)cb * ne + e];
      if (JVP) d = V[(size_t)cb * ne + e];
    }
    (&sX[0][0][0][0][0])[cb * TE + t] = a;
    if (JVP) (&sX[NS - 1][0][0][0][0])[cb * TE + t] = d;
  }
  __syncthreads();
  // modal corrected gradient: Ghat_p = L0 U_e + L1 U_{e+p} + L2 U_{e-p}
  for (int it = tid; it < DIM * NV * NB * TE; it += 256) {
    int r = it;
    const int t = r % TE;
    r /= TE;
    const int b = r % NB;
    r /= NB;
    const int c = r % NV;
    const int p = r / NV;
    const int64_t e = e0 + t;
    double g = 0.0, gd = 0.0;
    if (e < ne) {
      const int64_t ep = m.nbr[(2 * p + 1) * ne + e], em = m.nbr[(2 * p) * ne + e];
      const double* L0 = tb.vLift + (((size_t)p * 3 + 0) * NB + b) * NB;
      const double* L1 = tb.vLift + (((size_t)p * 3 + 1) * NB + b) * NB;
      const double* L2 = tb.vLift + (((size_t)p * 3 + 2) * NB + b) * NB;
      for (int bp = 0; bp < NB; ++bp) {
        const size_t i = (size_t)(c * NB + bp) * ne;
        g += L0[bp] * sX[0][0][c][bp][t] + L1[bp] * U[i + ep] + L2[bp] * U[i + em];
        if (JVP) gd += L0[bp] * sX[NS - 1][0][c][bp][t] + L1[bp] * V[i + ep] + L2[bp] * V[i + em];
      }
    }
    sX[0][1 + p][c][b][t] = g;
    if (JVP) sX[NS - 1][1 + p][c][b][t] = gd;
  }
  __syncthreads();

  constexpr int NIT = NV * NB * TE;
  constexpr int PER = (NIT + 255) / 256;
  double acc[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) acc[k] = 0.0;

  for (int q0 = 0; q0 < NQ; q0 += QC) {
    for (int it = tid; it < QC * TE; it += 256) {
      const int t = it % TE, ql = it / TE, q = q0 + ql;
      if (q < NQ) {
        const double* phq = tb.vPhi + (size_t)q * NB;
        T u[NV], G[NV][DIM];
        for (int c = 0; c < NV; ++c) {
          u[c] = 0.0;
          for (int j = 0; j < DIM; ++j) G[c][j] = 0.0;
        }
        for (int b = 0; b < NB; ++b) {
          const double w = phq[b];
          for (int c = 0; c < NV; ++c) {
            if constexpr (JVP) {
              u[c] += w * dual(sX[0][0][c][b][t], sX[1][0][c][b][t]);
              for (int j = 0; j < DIM; ++j) G[c][j] += w * dual(sX[0][1 + j][c][b][t], sX[1][1 + j][c][b][t]);
            } else {
              u[c] += w * sX[0][0][c][b][t];
              for (int j = 0; j < DIM; ++j) G[c][j] += w * sX[0][1 + j][c][b][t];
            }
          }
        }
        T F[DIM][NV];
        PHY::template volume_flux<T, DIM>(u, G, ph, F);
        for (int j = 0; j < DIM; ++j)
          for (int c = 0; c < NV; ++c) sF[j][c][ql][t] = out_part(F[j][c]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int it = tid + k * 256;
      if (it < NIT) {
        const int t = it % TE, cb = it / TE, b = cb % NB, c = cb / NB;
        double a = acc[k];
        for (int ql = 0; ql < QC; ++ql) {
          const int q = q0 + ql;
          if (q < NQ)
            for (int j = 0; j < DIM; ++j) a -= tb.vWD[((size_t)j * NQ + q) * NB + b] * sF[j][c][ql][t];
        }
        acc[k] = a;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int it = tid + k * 256;
    if (it < NIT) {
      const int t = it % TE, cb = it / TE, b = cb % NB, c = cb / NB;
      const int64_t e = e0 + t;
      if (e < ne) {
        double a = acc[k];
        for (int p = 0; p < DIM; ++p) {
          const int64_t em = m.nbr[(2 * p) * ne + e];
          const double* wP = tb.fWPhi + ((size_t)(p * 2 + 1) * NFQ) * NB + b;
          const double* wM = tb.fWPhi + ((size_t)(p * 2 + 0) * NFQ) * NB + b;
          for (int fq = 0; fq < NFQ; ++fq) {
            const size_t hi = ((size_t)(p * NV + c) * NFQ + fq) * ne;
            a += wP[fq * NB] * H[hi + e] - wM[fq * NB] * H[hi + em];
          }
        }
        // shift times the mass form: the variables with a time derivative
        if (JVP && c < PHY::template nmass<DIM>()) a += shift * V[(size_t)cb * ne + e];
        out[(size_t)cb * ne + e] = a;
      }
    }
  }
}

// ------------------------------------------------------------------ small kernels
template <int DIM, int NB, int NQ1>
__global__ void k_project(const double* __restrict__ f, double* __restrict__ w, Tables tb, int64_t ne, int nv) {
  constexpr int NQ = ipow(NQ1, DIM);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nv * NB * ne) return;
  const int64_t e = i % ne;
  const int cb = (int)(i / ne), c = cb / NB, b = cb % NB;
  double a = 0.0;
  for (int q = 0; q < NQ; ++q) a += tb.vWPhi[q * NB + b] * f[((size_t)c * NQ + q) * ne + e];
  w[i] = a;
}

template <int DIM, int NB, int NQ1>
__global__ void k_points(double* __restrict__ xyz, Tables tb, Mesh m) {
  constexpr int NQ = ipow(NQ1, DIM);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)NQ * m.ne) return;
  const int64_t e = i % m.ne;
  const int q = (int)(i / m.ne);
  for (int j = 0; j < DIM; ++j)
    xyz[((size_t)j * NQ + q) * m.ne + e] = m.x0[j * m.ne + e] + 0.5 * (tb.vXi[q * DIM + j] + 1.0) * m.h[j];
}

// per-block maxima of |u| + c over the volume points of a grid-stride set of elements
// (incompressible: |u| + sqrt(|u|^2 + beta^2), the largest speed of the
// artificial compressibility system of the interface flux)
template <class PHY, int DIM, int NB, int NQ1>
__global__ __launch_bounds__(256) void k_wave_speed(const double* __restrict__ w, double* __restrict__ partial,
                                                     Tables tb, Mesh m, Phys ph) {
  constexpr int NV = PHY::template nv<DIM>(), NQ = ipow(NQ1, DIM);
  constexpr bool kInc = std::is_same<PHY, IncompressiblePhys>::value;
  __shared__ double red[256];
  double mx = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < (int64_t)NQ * m.ne; i += (int64_t)gridDim.x * 256) {
    const int64_t e = i % m.ne;
    const int q = (int)(i / m.ne);
    double u[NV];
    for (int c = 0; c < NV; ++c) {
      double a = 0.0;
      for (int b = 0; b < NB; ++b) a += tb.vPhi[q * NB + b] * w[((size_t)c * NB + b) * m.ne + e];
      u[c] = a;
    }
    double a;
    if constexpr (std::is_same<PHY, DiffusionPhys>::value) {
      a = 0.0;
    } else if constexpr (kInc) {
      double s = 0.0;
      for (int j = 0; j < DIM; ++j) s += u[j] * u[j];
      a = sqrt(s) + sqrt(s + ph.beta * ph.beta);
    } else {
      double rinv, vel[DIM], p;
      primitives<double, DIM>(u, ph.gamma, rinv, vel, p);
      double s = 0.0;
      for (int j = 0; j < DIM; ++j) s += vel[j] * vel[j];
      a = sqrt(s) + sqrt(ph.gamma * p * rinv);
    }
    mx = (a > mx || a != a) ? a : mx;
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      const double o = red[threadIdx.x + st];
      red[threadIdx.x] = (o > red[threadIdx.x] || o != o) ? o : red[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ------------------------------------------------------------------ dispatch
// Compiled configurations (dim, nb, nq1d) and tile sizes of the volume kernel.
#define DG_CONFIGS(X)   \
  X(0, 2, 9, 4)         \
  X(1, 2, 6, 4)         \
  X(2, 3, 4, 2)         \
  X(3, 3, 10, 3)        \
  X(4, 3, 20, 4)        \
  X(5, 3, 35, 5)        \
  X(6, 2, 3, 3)         \
  X(7, 2, 10, 5)        \
  X(8, 2, 28, 8)

int config_index(int dim, int nb, int nq1d) {
#define X(id, d, nb_, nq_) \
  if (dim == d && nb == nb_ && nq1d == nq_) return id;
  DG_CONFIGS(X)
#undef X
  return -1;
}

template <int NB, bool JVP> struct VolTile {
  static constexpr int TE = JVP ? 8 : 16;
  static constexpr int QC = 256 / TE;
};

template <class PHY>
hipError_t face_dispatch(int cfg, bool jvp, const double* U, const double* V, double* H, const Tables& tb,
                         const Mesh& m, const Phys& ph, hipStream_t s) {
#define X(id, d, nb_, nq_)                                                                          \
  case id: {                                                                                        \
    dim3 grid((unsigned)((m.ne + 63) / 64), d);                                                     \
    if (jvp)                                                                                        \
      k_face<PHY, d, nb_, nq_, true><<<grid, 256, 0, s>>>(U, V, H, tb, m, ph);                      \
    else                                                                                            \
      k_face<PHY, d, nb_, nq_, false><<<grid, 256, 0, s>>>(U, V, H, tb, m, ph);                     \
    return hipGetLastError();                                                                       \
  }
  switch (cfg) { DG_CONFIGS(X) }
#undef X
  return hipErrorInvalidValue;
}

template <class PHY>
hipError_t volume_dispatch(int cfg, bool jvp, const double* U, const double* V, const double* H, double* out,
                           double shift, const Tables& tb, const Mesh& m, const Phys& ph, hipStream_t s) {
#define X(id, d, nb_, nq_)                                                                                    \
  case id: {                                                                                                  \
    if (jvp) {                                                                                                \
      using TL = VolTile<nb_, true>;                                                                          \
      dim3 grid((unsigned)((m.ne + TL::TE - 1) / TL::TE));                                                    \
      k_volume<PHY, d, nb_, nq_, true, TL::TE, TL::QC><<<grid, 256, 0, s>>>(U, V, H, out, shift, tb, m, ph); \
    } else {                                                                                                  \
      using TL = VolTile<nb_, false>;                                                                         \
      dim3 grid((unsigned)((m.ne + TL::TE - 1) / TL::TE));                                                    \
      k_volume<PHY, d, nb_, nq_, false, TL::TE, TL::QC><<<grid, 256, 0, s>>>(U, V, H, out, shift, tb, m, ph);\
    }                                                                                                         \
    return hipGetLastError();                                                                                 \
  }
  switch (cfg) { DG_CONFIGS(X) }
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_face(int cfg, bool jvp, const double* U, const double* V, double* H, const Tables& tb,
                       const Mesh& m, const Phys& ph, hipStream_t s) {
  if (ph.model == DG_PHYS_INCOMPRESSIBLE) return face_dispatch<IncompressiblePhys>(cfg, jvp, U, V, H, tb, m, ph, s);
  if (ph.model == DG_PHYS_DIFFUSION) return face_dispatch<DiffusionPhys>(cfg, jvp, U, V, H, tb, m, ph, s);
  return face_dispatch<CompressiblePhys>(cfg, jvp, U, V, H, tb, m, ph, s);
}

hipError_t launch_volume(int cfg, bool jvp, const double* U, const double* V, const double* H, double* out,
                         double shift, const Tables& tb, const Mesh& m, const Phys& ph, hipStream_t s) {
  if (ph.model == DG_PHYS_INCOMPRESSIBLE)
    return volume_dispatch<IncompressiblePhys>(cfg, jvp, U, V, H, out, shift, tb, m, ph, s);
  if (ph.model == DG_PHYS_DIFFUSION)
    return volume_dispatch<DiffusionPhys>(cfg, jvp, U, V, H, out, shift, tb, m, ph, s);
  return volume_dispatch<CompressiblePhys>(cfg, jvp, U, V, H, out, shift, tb, m, ph, s);
}

hipError_t launch_project(int cfg, int nv, const double* f, double* w, const Tables& tb, const Mesh& m,
                          hipStream_t s) {
#define X(id, d, nb_, nq_)                                                          \
  case id: {                                                                        \
    int64_t n = (int64_t)nv * nb_ * m.ne;                                           \
    k_project<d, nb_, nq_><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(f, w, tb, m.ne, nv); \
    return hipGetLastError();                                                       \
  }
  switch (cfg) { DG_CONFIGS(X) }
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_points(int cfg, double* xyz, const Tables& tb, const Mesh& m, hipStream_t s) {
#define X(id, d, nb_, nq_)                                                         \
  case id: {                                                                       \
    int64_t n = (int64_t)ipow(nq_, d) * m.ne;                                      \
    k_points<d, nb_, nq_><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(xyz, tb, m); \
    return hipGetLastError();                                                      \
  }
  switch (cfg) { DG_CONFIGS(X) }
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_wave_speed(int cfg, const double* w, double* partial, int nblocks, const Tables& tb,
                             const Mesh& m, const Phys& ph, hipStream_t s) {
#define X(id, d, nb_, nq_)                                                            \
  case id: {                                                                          \
    if (ph.model == DG_PHYS_INCOMPRESSIBLE)                                           \
      k_wave_speed<IncompressiblePhys, d, nb_, nq_><<<nblocks, 256, 0, s>>>(w, partial, tb, m, ph); \
    else if (ph.model == DG_PHYS_DIFFUSION)                                           \
      k_wave_speed<DiffusionPhys, d, nb_, nq_><<<nblocks, 256, 0, s>>>(w, partial, tb, m, ph); \
    else                                                                              \
      k_wave_speed<CompressiblePhys, d, nb_, nq_><<<nblocks, 256, 0, s>>>(w, partial, tb, m, ph);   \
    return hipGetLastError();                                                         \
  }
  switch (cfg) { DG_CONFIGS(X) }
#undef X
  return hipErrorInvalidValue;
}

}  // namespace dgk
