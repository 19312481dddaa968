// DG residual and exact Jv on curved (multilinear) elements (Sec. 2.1-2.2,
// eq. NSdiscrRes): the compressible equations in FP64 and FP32, the scalar
// BR2 Laplacian of the Poisson assessment (App. B) in FP64; dual numbers for
// Jv; the face products of pass 3 on the matrix cores, the rest on the vector
// ALU.
//
// Element K's orthonormal basis is phi = L^{-1} psi, with L L^T the mass
// matrix of the reference basis psi on K.  Every contraction therefore runs
// against the shared reference tables of psi (read through the caches by all
// elements) on coefficients transformed by the element's L^{-1}:
//   u(x) = sum_a psi_a(xi) Ut_a,             Ut = L^{-T} U,
//   grad_x u = K grad_xi u,                  K = J^{-T} at the point,
//   R_b = sum_{a<=b} L^{-1}_{ba} Yt_a,       Yt = the projection on psi.
// Only L^{-1} (packed) and the point geometry are stored per element and
// face.
//
// Pass 1 (k_modal_curved), one workgroup per element: Ut and Vt.
// Pass 2 (k_face_curved), one workgroup per face (p, e) (owner e, neighbour
// across its +p face), one lane per (side, face point): traces of both sides,
// the jump [[U]] = U_owner - U_neighbour (stored for pass 3), the averaged
// lifting {r} at the face points through the face's point-to-point matrix
// P_fg = sum_sides phi(x_f).phi(x_g):
//   {r}_cj(x_f) = -1/4 sum_g P_fg w_g n_j(x_g) [[U_c]](x_g),
// and w_f|J_f| times the normal flux H^c(U_L, U_R, n) - F^v({U}, {G}).n.
// Pass 3 (k_volume_curved), one workgroup per element: the elemental lifting
// R^K = sum over its 2d faces of the local liftings, in the reference basis
// Rt = L^{-T} L^{-1} rho_t with rho_t_{a,c,j} = -1/2 sum_f psi_a w n_j [[U_c]];
// the volume flux with G = grad U + R^K at the volume points, mapped to
// reference directions (w|J| K^T F); its projection on grad_xi psi and the
// face fluxes gathered on psi of each face (+ owner, - neighbour side); and
// finally L^{-1}.
#include "dg_device.h"

namespace dgk {

namespace {

// block id -> work unit: consecutive units on one XCD (blocks are dealt to
// the 8 XCDs in turn, each with its own L2)
DEV int64_t xcd_unit(int64_t bid, int64_t nblk) {
  constexpr int64_t kXcd = 8;
  const int64_t q = nblk / kXcd, r = nblk % kXcd, x = bid % kXcd;
  return x * q + (x < r ? x : r) + bid / kXcd;
}

template <bool JVP, class R>
DEV typename Scalar<JVP, R>::type mk(R v, R t) {
  if constexpr (JVP)
    return dualT<R>(v, t);
  else
    return v;
}

// value (and tangent) stored adjacently: one 16-byte (FP64) or 8-byte (FP32)
// LDS read per dual
template <bool JVP, class R>
DEV typename Scalar<JVP, R>::type ld2(const R* p) {
  if constexpr (JVP) {
    using V2 = typename std::conditional<sizeof(R) == 8, double2, float2>::type;
    const V2 v = *reinterpret_cast<const V2*>(p);
    return dualT<R>(v.x, v.y);
  } else {
    return p[0];
  }
}

// 16x16x4 matrix-core step: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// D[i][j] lands in lane j + 16 g, register r with i = drow(g, r).
typedef double cv_f64x4 __attribute__((ext_vector_type(4)));
typedef float cv_f32x4 __attribute__((ext_vector_type(4)));
template <class R>
struct CMma;
template <>
struct CMma<double> {
  using frag = cv_f64x4;
  static DEV frag mma(double a, double b, frag c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static DEV int drow(int g, int r) { return g + 4 * r; }
};
template <>
struct CMma<float> {
  using frag = cv_f32x4;
  static DEV frag mma(float a, float b, frag c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static DEV int drow(int g, int r) { return 4 * g + r; }
};

// DIFF (all kernels below): the scalar Laplacian of the Poisson assessment
// (one variable, no convective flux, F^v = mu grad u) instead of the
// compressible equations.
template <class R, int DIM, int NB, bool JVP, bool DIFF = false>
__global__ __launch_bounds__(64) void k_modal_curved(const double* __restrict__ U, const double* __restrict__ V,
                                                     CurvedTablesT<R> ct, int64_t ne) {
  constexpr int NV = DIFF ? 1 : DIM + 2, NBT = NB * (NB + 1) / 2, NS = JVP ? 2 : 1, NX = NV * NB;
  __shared__ R sL[NBT];
  __shared__ R sX[NS * NX];
  const int tid = threadIdx.x;
  const int64_t e = blockIdx.x;
  for (int i = tid; i < NBT; i += 64) sL[i] = ct.Linv[(size_t)e * NBT + i];
  for (int i = tid; i < NS * NX; i += 64) sX[i] = (i < NX ? U : V)[(size_t)(i % NX) * ne + e];
  __syncthreads();
  for (int i = tid; i < NS * NX; i += 64) {
    const int a = i % NB, row = i - a;  // row = (s, c) * NB
    R acc = 0.0;
    for (int b = 0; b < NB; ++b) {  // same b in every lane: consecutive a read consecutive words
      const R l = sL[b * (b + 1) / 2 + a];
      acc += (b >= a ? l : R(0)) * sX[row + b];
    }
    (i < NX ? ct.Ut : ct.Vt)[(size_t)e * NX + (i % NX)] = acc;
  }
}

template <class R, int DIM, int NB, int NQ1, bool JVP, bool DIFF = false>
__global__ __launch_bounds__(64) void k_face_curved(CurvedTablesT<R> ct, Mesh m, Phys ph) {
  using T = typename Scalar<JVP, R>::type;
  constexpr int NV = DIFF ? 1 : DIM + 2, NFQ = ipow(NQ1, DIM - 1), NS = JVP ? 2 : 1, NC = NV * DIM, NX = NV * NB;
  constexpr int GF = DIM + 1 + 2 * DIM * DIM, NTR = NV * (1 + DIM);
  static_assert(NFQ <= 32, "one lane per (side, face point)");
  constexpr int NW = 2 * NS * NX > NS * NC * NFQ ? 2 * NS * NX : NS * NC * NFQ;
  constexpr int NKL = (NC + 1) / 2;  // {r} columns per lane half
  __shared__ __align__(16) R sW[NW];     // coefficients of both sides, then sX, then sR
  // Traces of both sides: values and physical gradients.  FP64 (kSum): the
  // gradients enter the flux only as the sum of the two sides, which both
  // sides add into one slot (two LDS atomic adds onto zero: a + b either way,
  // so the sum is deterministic); the 6 KB saved let 8 instead of 6
  // workgroups share a CU (P4: face 0.60 -> 0.51 ms).  FP32 keeps both sides'
  // gradients (the atomic form measured 0.29 -> 0.51 ms there).
  constexpr bool kSum = sizeof(R) == 8;
  __shared__ R sT[2][NS][kSum ? NV : NTR][NFQ];  // values (and FP32 gradients) per side
  __shared__ R sG[kSum ? NS : 1][kSum ? NC : 1][NFQ];     // FP64 gradient sums
  __shared__ R sH[2][NV][NFQ];           // convective and viscous parts of the normal flux
  R* sU = sW;                                               // [side][c][a][value/tangent]
  auto sX = reinterpret_cast<R(*)[NC][NFQ]>(sW);            // [s][c*DIM+j][fq]: w n_j [[U_c]]
  auto sR = reinterpret_cast<R(*)[NC][NFQ]>(sW);            // {r}_cj at the face points (over sX)
  const int tid = threadIdx.x, side = tid >> 5, fq = tid & 31;
  // work units (element, direction), direction fastest, a contiguous range
  // of elements per XCD (blocks are dealt to the 8 XCDs in turn)
  const int64_t ne = m.ne;
  const int64_t u = xcd_unit(blockIdx.x, gridDim.x);
  const int P = (int)(u % DIM);
  const int64_t e = u / DIM;
  const int64_t er = m.nbr[(size_t)(2 * P + 1) * ne + e];
  const size_t f = (size_t)P * ne + e;
  const R* geo = ct.fGeo + f * GF * NFQ;
  const bool act = fq < NFQ;

  const R* __restrict__ vtn = ct.VtN ? ct.VtN : ct.Vt;  // the neighbour's tangent
  for (int i = tid; i < 2 * NS * NX; i += 64) {  // [side][c][a][value/tangent]
    const int sd = i / (NS * NX), s = (i / NX) % NS;
    sU[(sd * NX + i % NX) * NS + s] = (s ? (sd ? vtn : ct.Vt) : ct.Ut)[(size_t)(sd ? er : e) * NX + (i % NX)];
  }
  if constexpr (kSum)
    for (int i = tid; i < NS * NC * NFQ; i += 64) (&sG[0][0][0])[i] = R(0);
  __syncthreads();

  // traces of this lane's side at face point fq
  if (act) {
    const int ls = side == 0 ? 2 * P + 1 : 2 * P;  // local face: owner at xi_P = +1, neighbour at -1
    const R* ps = ct.rFPsiT + (size_t)ls * NB * NFQ + fq;
    const R* dps = ct.rFDPsiT + (size_t)ls * DIM * NB * NFQ + fq;
    const R* xs = sU + side * NS * NX;
    T u[NV], g[NV][DIM];
    for (int c = 0; c < NV; ++c) {
      u[c] = 0.0;
      for (int r = 0; r < DIM; ++r) g[c][r] = 0.0;
    }
    // unrolled over 5 (FP64) / 7 (FP32) modes: the table loads of several
    // modes in flight (2 left the lanes waiting on them: 0.78 -> 0.60 ms FP64,
    // 0.40 -> 0.29 ms FP32 at P4 24^3)
    constexpr int kTU = sizeof(R) == 8 ? 5 : 7;
#pragma unroll kTU
    for (int b = 0; b < NB; ++b) {  // each table entry read once for all variables
      const R pb = ps[b * NFQ];
      R db[DIM];
      for (int r = 0; r < DIM; ++r) db[r] = dps[(r * NB + b) * NFQ];
      for (int c = 0; c < NV; ++c) {
        const T x = ld2<JVP, R>(xs + (c * NB + b) * NS);
        u[c] += pb * x;
        for (int r = 0; r < DIM; ++r) g[c][r] += db[r] * x;
      }
    }
    R K[DIM][DIM];
    for (int i = 0; i < DIM; ++i)
      for (int r = 0; r < DIM; ++r) K[i][r] = geo[(size_t)(DIM + 1 + side * DIM * DIM + i * DIM + r) * NFQ + fq];
    for (int c = 0; c < NV; ++c) {
      sT[side][0][c][fq] = val(u[c]);
      if constexpr (JVP) sT[side][NS - 1][c][fq] = out_part(u[c]);
      for (int i = 0; i < DIM; ++i) {  // reference to physical gradient
        T t = 0.0;
        for (int r = 0; r < DIM; ++r) t += K[i][r] * g[c][r];
        if constexpr (kSum) {
          atomicAdd(&sG[0][c * DIM + i][fq], val(t));
          if constexpr (JVP) atomicAdd(&sG[NS - 1][c * DIM + i][fq], out_part(t));
        } else {
          sT[side][0][NV + c * DIM + i][fq] = val(t);
          if constexpr (JVP) sT[side][NS - 1][NV + c * DIM + i][fq] = out_part(t);
        }
      }
    }
  }
  __syncthreads();

  // jumps (kept for the elemental liftings) and w n [[U]]
  double n[DIM];  // the numerical flux takes an FP64 normal
  for (int j = 0; j < DIM; ++j) n[j] = act ? geo[(size_t)j * NFQ + fq] : 0.0;
  const R W = act ? geo[(size_t)DIM * NFQ + fq] : R(0);
  if (side == 0 && act) {
    for (int c = 0; c < NV; ++c) {
      const R jv = sT[0][0][c][fq] - sT[1][0][c][fq];
      const R jt = JVP ? sT[0][NS - 1][c][fq] - sT[1][NS - 1][c][fq] : 0.0;
      ct.fJmp[((f * 2 + 0) * NV + c) * NFQ + fq] = jv;
      ct.fJmp[((f * 2 + 1) * NV + c) * NFQ + fq] = (JVP && !ph.stab_only) ? jt : 0.0;
      for (int j = 0; j < DIM; ++j) {
        sX[0][c * DIM + j][fq] = W * n[j] * jv;
        if constexpr (JVP) sX[NS - 1][c * DIM + j][fq] = W * n[j] * jt;
      }
    }
  }
  __syncthreads();

  // {r} = -1/4 P X, the (c, j) columns shared between the two halves; held
  // in registers until every lane has read X, then written over it
  R rv[NKL], rt[NKL];
  for (int q = 0; q < NKL; ++q) rv[q] = rt[q] = R(0);
  if (act) {
    const R* Pf = ct.fP + f * NFQ * NFQ + fq;  // P is symmetric: row fq read along g
#pragma unroll 5
    for (int gq = 0; gq < NFQ; ++gq) {  // each entry of P read once for all columns
      const R pv = Pf[gq * NFQ];
#pragma unroll
      for (int q = 0; q < NKL; ++q) {
        const int k = side + 2 * q < NC ? side + 2 * q : NC - 1;
        rv[q] += pv * sX[0][k][gq];
        if constexpr (JVP) rt[q] += pv * sX[NS - 1][k][gq];
      }
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int q = 0; q < NKL; ++q) {
      const int k = side + 2 * q;
      if (k < NC) {
        sR[0][k][fq] = R(-0.25) * rv[q];
        if constexpr (JVP) sR[NS - 1][k][fq] = R(-0.25) * rt[q];
      }
    }
  }
  __syncthreads();

  // normal flux: convective part on the owner-side lanes, viscous part on the
  // neighbour-side lanes (in the stabilisation-only tangent, only the face
  // lifting term eta {r} carries a tangent)
  const bool tr = JVP && !ph.stab_only;
  if (act) {
    T Hp[NV];
    if (side == 0) {
      if constexpr (DIFF) {
        Hp[0] = R(0);  // no convective flux
      } else {
        T uL[NV], uR[NV];
        for (int c = 0; c < NV; ++c) {
          uL[c] = mk<JVP, R>(sT[0][0][c][fq], tr ? sT[0][NS - 1][c][fq] : R(0));
          uR[c] = mk<JVP, R>(sT[1][0][c][fq], tr ? sT[1][NS - 1][c][fq] : R(0));
        }
        num_flux_n<T, DIM>(uL, uR, n, ph, Hp);
      }
    } else {
      T ua[NV], Ga[NV][DIM];
      for (int c = 0; c < NV; ++c) {
        ua[c] = R(0.5) * mk<JVP, R>(sT[0][0][c][fq] + sT[1][0][c][fq],
                                    tr ? sT[0][NS - 1][c][fq] + sT[1][NS - 1][c][fq] : R(0));
        for (int i = 0; i < DIM; ++i) {
          const int k = NV + c * DIM + i;
          if constexpr (kSum)  // owner + neighbour gradient trace
            Ga[c][i] = R(0.5) * mk<JVP, R>(sG[0][k - NV][fq], tr ? sG[NS - 1][k - NV][fq] : R(0)) +
                       (R)ph.eta * mk<JVP, R>(sR[0][c * DIM + i][fq], sR[NS - 1][c * DIM + i][fq]);
          else
            Ga[c][i] = R(0.5) * mk<JVP, R>(sT[0][0][k][fq] + sT[1][0][k][fq],
                                           tr ? sT[0][NS - 1][k][fq] + sT[1][NS - 1][k][fq] : R(0)) +
                       (R)ph.eta * mk<JVP, R>(sR[0][c * DIM + i][fq], sR[NS - 1][c * DIM + i][fq]);
        }
      }
      if constexpr (DIFF) {  // -mu {grad u + eta r}.n
        Hp[0] = 0.0;
        for (int j = 0; j < DIM; ++j) Hp[0] -= (R)n[j] * ((R)ph.mu * Ga[0][j]);
      } else {
        const double kap = ph.mu * ph.gamma / (ph.prandtl * (ph.gamma - 1.0));
        ViscPrep<T, DIM> vp;
        visc_prep<T, DIM>(ua, Ga, ph.gamma, vp);
        for (int c = 0; c < NV; ++c) Hp[c] = 0.0;
        for (int j = 0; j < DIM; ++j) {
          T Fv[NV];
          visc_flux_dir<T, DIM>(vp, j, ph.mu, kap, Fv);
          for (int c = 0; c < NV; ++c) Hp[c] -= (R)n[j] * Fv[c];
        }
      }
    }
    for (int c = 0; c < NV; ++c) sH[side][c][fq] = out_part(Hp[c]);
  }
  __syncthreads();
  for (int i = tid; i < NV * NFQ; i += 64) {
    const int gq = i % NFQ, c = i / NFQ;
    ct.fHn[f * NV * NFQ + i] = geo[(size_t)DIM * NFQ + gq] * (sH[0][c][gq] + sH[1][c][gq]);
  }
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// Launch bound: FP32 at three waves per SIMD (at most 170 registers: room for
// the prefetched face data below without spills; measured faster than four
// waves with spills and than the register-lean form at four)
template <class R, int DIM, int NB, int NQ1, bool JVP, bool DIFF = false>
__global__ __launch_bounds__(128, sizeof(R) == 8 ? 1 : 3) void k_volume_curved(const double* __restrict__ V, CurvedTablesT<R> ct,
                                                      double* __restrict__ out, double shift, Mesh m, Phys ph) {
  using T = typename Scalar<JVP, R>::type;
  constexpr int NV = DIFF ? 1 : DIM + 2, NQ = ipow(NQ1, DIM), NFQ = ipow(NQ1, DIM - 1), NS = JVP ? 2 : 1;
  constexpr int NBT = NB * (NB + 1) / 2, NC = NV * DIM, NX = NV * NB, GV = DIM * DIM + 1;
  constexpr int GF = DIM + 1 + 2 * DIM * DIM;
  constexpr int NA = NS * NC * NB, NF = NQ * DIM * NV;
  constexpr int NR = NS * NC + NV, MT = (NR + 15) / 16, NT = (NB + 15) / 16, NTW = (MT * NT + 1) / 2;
  constexpr int KSF = (NFQ + 3) / 4;
  constexpr int NSTG = NR * NFQ + NFQ * NB;  // one face: w n [[U]], w Hn, psi
  static_assert(NQ <= 128, "one thread per volume point");
  static_assert(DIM * NB <= 128, "one thread per (reference direction, mode) in the projection");
  static_assert(DIM * NV * NB <= NA, "projection partials fit the lifting buffer");
  __shared__ __align__(16) R sU[NS * NX];      // Ut, Vt interleaved
  __shared__ R sL[NBT];                        // L^{-1}, packed rows
  __shared__ R sLc[NBT];                       // L^{-1}, packed columns
  __shared__ __align__(16) R sA[NA];           // rho_t, Rt (interleaved), projection partials
  __shared__ R sB[cmax(NA, cmax(NF, NSTG))];  // face staging, L^{-1} rho_t, then w|J| K^T F
  __shared__ R sY[NX];                         // projection on psi
  const int tid = threadIdx.x;
  const int64_t ne = m.ne;
  const int64_t e = xcd_unit(blockIdx.x, gridDim.x);
  const bool vt = JVP && !ph.stab_only;  // tangent of the volume terms

  for (int i = tid; i < NB * NB; i += 128) {
    const int b = i / NB, a = i % NB;
    if (a <= b) {
      const R l = ct.Linv[(size_t)e * NBT + b * (b + 1) / 2 + a];
      sL[b * (b + 1) / 2 + a] = l;
      sLc[a * NB - a * (a - 1) / 2 + b - a] = l;
    }
  }
  for (int i = tid; i < NS * NX; i += 128)  // value and tangent interleaved: [c][a][s]
    sU[(i % NX) * NS + i / NX] = i < NX ? ct.Ut[(size_t)e * NX + i] : (vt ? ct.Vt[(size_t)e * NX + i - NX] : 0.0);

  // the 2d faces one at a time: +p faces (owner side, xi_p = +1) and -p faces
  // (neighbour side, xi_p = -1).  Rows of the staged face matrix: w n_j [[U_c]]
  // (value, tangent) then w Hn; each thread accumulates a 2-mode x RG-row
  // block of their products with psi of the face: the local liftings rho_t
  // and the face part of the projection.
  // Each of the two waves accumulates its share of the 16x16 tiles of the
  // (row x mode) product over the 2d faces on the matrix cores; K runs over
  // the face points (zero-padded to a multiple of 4).
  using MM = CMma<R>;
  typename MM::frag acc[NTW];
  for (int t = 0; t < NTW; ++t)
    for (int r = 0; r < 4; ++r) acc[t][r] = R(0);
  const int wv = tid >> 6, ln = tid & 63, li = ln & 15, lg = ln >> 4;
  R* sXs = sB;                  // [NR][NFQ]
  R* sPs = sB + NR * NFQ;       // [NFQ][NB]
  // The loads of face hf + 1 are issued before the products of face hf and
  // land in registers while those run (the staging loads' latency was a fifth
  // of the kernel); the products w n_j [[U]] are formed at the LDS write.
  constexpr int NXE = NS * NC * NFQ, NHE = NV * NFQ, NPE = NFQ * NB;
  constexpr int PX = (NXE + 127) / 128, PH = (NHE + 127) / 128, PP = (NPE + 127) / 128;
  size_t fidx[2 * DIM];  // face record of the 2d faces: own +p faces, the -p neighbours' +p faces
#pragma unroll
  for (int hf = 0; hf < 2 * DIM; ++hf)
    fidx[hf] = (size_t)(hf >> 1) * ne + ((hf & 1) ? m.nbr[(size_t)(2 * (hf >> 1)) * ne + e] : e);
  R pw[PX], pn[PX], pj[PX], ph_[PH], pp[PP];
  const R* __restrict__ jmpN = ct.fJmpN ? ct.fJmpN : ct.fJmp;  // records of the -p faces
  const R* __restrict__ hnN = ct.fHnN ? ct.fHnN : ct.fHn;
  auto fetch = [&](int hf) {
    const size_t f = fidx[hf];
    const int p = hf >> 1, ls = (hf & 1) ? 2 * p : 2 * p + 1;
    const R* geo = ct.fGeo + f * GF * NFQ;
    const R* __restrict__ jmp = (hf & 1) ? jmpN : ct.fJmp;
    const R* __restrict__ hn = (hf & 1) ? hnN : ct.fHn;
#pragma unroll
    for (int u = 0; u < PX; ++u) {
      const int i = tid + 128 * u < NXE ? tid + 128 * u : NXE - 1;
      const int gq = i % NFQ, k = (i / NFQ) % NC, s = i / (NC * NFQ), c = k / DIM, j = k % DIM;
      pw[u] = geo[(size_t)DIM * NFQ + gq];
      pn[u] = geo[(size_t)j * NFQ + gq];
      pj[u] = jmp[((f * 2 + s) * NV + c) * NFQ + gq];
    }
#pragma unroll
    for (int u = 0; u < PH; ++u) ph_[u] = hn[f * NHE + (tid + 128 * u < NHE ? tid + 128 * u : NHE - 1)];
#pragma unroll
    for (int u = 0; u < PP; ++u) pp[u] = ct.rFPsi[(size_t)ls * NPE + (tid + 128 * u < NPE ? tid + 128 * u : NPE - 1)];
  };
  fetch(0);
  for (int hf = 0; hf < 2 * DIM; ++hf) {
    const int h = hf & 1;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PX; ++u)
      if (tid + 128 * u < NXE) sXs[tid + 128 * u] = pw[u] * pn[u] * pj[u];
#pragma unroll
    for (int u = 0; u < PH; ++u)
      if (tid + 128 * u < NHE) sXs[NXE + tid + 128 * u] = ph_[u] * (h ? -1.0 : 1.0);
#pragma unroll
    for (int u = 0; u < PP; ++u)
      if (tid + 128 * u < NPE) sPs[tid + 128 * u] = pp[u];
    __syncthreads();
    if (hf + 1 < 2 * DIM) fetch(hf + 1);
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
      const int tile = wv + 2 * t;
      if (tile < MT * NT) {  // uniform per wave
        const int row = (tile / NT) * 16 + li, mode = (tile % NT) * 16 + li;
        const int rowc = row < NR ? row : NR - 1, modec = mode < NB ? mode : NB - 1;
#pragma unroll
        for (int ks = 0; ks < KSF; ++ks) {
          const int k = 4 * ks + lg, kc = k < NFQ ? k : NFQ - 1;
          const R av = sXs[rowc * NFQ + kc], bv = sPs[kc * NB + modec];
          acc[t] = MM::mma((row < NR && k < NFQ) ? av : R(0), (mode < NB && k < NFQ) ? bv : R(0), acc[t]);
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NTW; ++t) {
    const int tile = wv + 2 * t;
    if (tile < MT * NT) {
      const int mode = (tile % NT) * 16 + li;
      for (int r = 0; r < 4; ++r) {
        const int row = (tile / NT) * 16 + MM::drow(lg, r);
        if (row < NR && mode < NB) {
          if (row < NS * NC)
            sA[row * NB + mode] = R(-0.5) * acc[t][r];
          else
            sY[(row - NS * NC) * NB + mode] = acc[t][r];
        }
      }
    }
  }
  __syncthreads();
  // the triangular products run uniform loops (one index for every lane) over
  // the row- or column-packed copy that makes neighbouring lanes read
  // neighbouring words; each thread takes one mode of RG rows, so every
  // entry of L^{-1} it reads serves RG products (the sums keep their order)
  constexpr int NROW = NS * NC, RG = (NROW + 2) / 3, NRG = (NROW + RG - 1) / RG;
  for (int it = tid; it < NB * NRG; it += 128) {  // L^{-1} rho_t
    const int b = it % NB, r0 = (it / NB) * RG;
    R acc[RG];
#pragma unroll
    for (int rr = 0; rr < RG; ++rr) acc[rr] = R(0);
    for (int a = 0; a < NB; ++a) {
      const R l = sLc[a * NB - a * (a - 1) / 2 + b - a];
      const R lm = a <= b ? l : R(0);
#pragma unroll
      for (int rr = 0; rr < RG; ++rr) acc[rr] += lm * sA[(r0 + rr < NROW ? r0 + rr : NROW - 1) * NB + a];
    }
#pragma unroll
    for (int rr = 0; rr < RG; ++rr)
      if (r0 + rr < NROW) sB[(r0 + rr) * NB + b] = acc[rr];
  }
  __syncthreads();
  for (int it = tid; it < NB * NRG; it += 128) {  // Rt = L^{-T} L^{-1} rho_t, value and tangent interleaved
    const int a = it % NB, r0 = (it / NB) * RG;
    R acc[RG];
#pragma unroll
    for (int rr = 0; rr < RG; ++rr) acc[rr] = R(0);
    for (int b = 0; b < NB; ++b) {
      const R l = sL[b * (b + 1) / 2 + a];
      const R lm = b >= a ? l : R(0);
#pragma unroll
      for (int rr = 0; rr < RG; ++rr) acc[rr] += lm * sB[(r0 + rr < NROW ? r0 + rr : NROW - 1) * NB + b];
    }
#pragma unroll
    for (int rr = 0; rr < RG; ++rr) {
      const int row = r0 + rr;  // (value/tangent, variable-direction)
      if (row < NROW) sA[((row % NC) * NB + a) * NS + row / NC] = acc[rr];
    }
  }
  __syncthreads();

  if (tid < NQ) {
    const double kap = ph.mu * ph.gamma / (ph.prandtl * (ph.gamma - 1.0));
    const R* geo = ct.vGeo + (size_t)e * GV * NQ + tid;
    R K[DIM][DIM];
    for (int i = 0; i < DIM; ++i)
      for (int r = 0; r < DIM; ++r) K[i][r] = geo[(size_t)(i * DIM + r) * NQ];
    const R wd = geo[(size_t)(DIM * DIM) * NQ];
    const R* ps = ct.rPsiT + tid;
    const R* dps = ct.rDPsiT + tid;
    T u[NV], G[NV][DIM];
    {
      T gx[NV][DIM];
      for (int c = 0; c < NV; ++c) {
        u[c] = 0.0;
        for (int r = 0; r < DIM; ++r) gx[c][r] = 0.0;
      }
      // unrolled over 7 modes in FP32 (0.63 -> 0.59 ms at P4 24^3); FP64 keeps 2:
      // more would cost it a wave per SIMD (measured 1.07 -> 1.5 ms)
#pragma unroll (sizeof(R) == 8 ? 2 : 7)
      for (int b = 0; b < NB; ++b) {  // each table entry read once for all variables
        const R pb = ps[b * NQ];
        R db[DIM];
        for (int r = 0; r < DIM; ++r) db[r] = dps[(r * NB + b) * NQ];
        for (int c = 0; c < NV; ++c) {
          const T x = ld2<JVP, R>(sU + (c * NB + b) * NS);
          u[c] += pb * x;
          for (int r = 0; r < DIM; ++r) gx[c][r] += db[r] * x;
        }
      }
      for (int c = 0; c < NV; ++c)
        for (int i = 0; i < DIM; ++i) {
          T t = 0.0;
          for (int r = 0; r < DIM; ++r) t += K[i][r] * gx[c][r];
          G[c][i] = t;
        }
    }
#pragma unroll 2
    for (int b = 0; b < NB; ++b) {  // + R^K
      const R pb = ps[b * NQ];
      for (int c = 0; c < NV; ++c)
        for (int r = 0; r < DIM; ++r)
          G[c][r] += pb * ld2<JVP, R>(sA + ((c * DIM + r) * NB + b) * NS);
    }
    R Ft[DIM][NV];
    for (int r = 0; r < DIM; ++r)
      for (int c = 0; c < NV; ++c) Ft[r][c] = 0.0;
    if constexpr (DIFF) {  // F_p = -mu G_p
      for (int p = 0; p < DIM; ++p) {
        const R fp = out_part(-(R)ph.mu * G[0][p]);
        for (int r = 0; r < DIM; ++r) Ft[r][0] += K[p][r] * fp;
      }
    } else {
      T rinv, vel[DIM], pr;
      primitives<T, DIM>(u, ph.gamma, rinv, vel, pr);
      ViscPrep<T, DIM> vp;
      visc_prep<T, DIM>(u, G, ph.gamma, vp);
      for (int p = 0; p < DIM; ++p) {
        T Fc[NV], Fv[NV];
        conv_flux_dir<T, DIM>(u, vel, pr, p, Fc);
        visc_flux_dir<T, DIM>(vp, p, ph.mu, kap, Fv);
        for (int c = 0; c < NV; ++c) {
          const R fp = out_part(Fc[c] - Fv[c]);
          for (int r = 0; r < DIM; ++r) Ft[r][c] += K[p][r] * fp;
        }
      }
    }
    for (int r = 0; r < DIM; ++r)
      for (int c = 0; c < NV; ++c) sB[(tid * DIM + r) * NV + c] = wd * Ft[r][c];
  }
  __syncthreads();

  if (tid < DIM * NB) {  // volume projection on d psi_a / d xi_r, one thread per (r, a)
    const int a = tid % NB, r = tid / NB;
    R acc[NV];
    for (int c = 0; c < NV; ++c) acc[c] = 0.0;
    const R* dp = ct.rDPsi + r * NB + a;
#pragma unroll 8
    for (int q = 0; q < NQ; ++q) {
      const R d = dp[q * DIM * NB];
      for (int c = 0; c < NV; ++c) acc[c] += d * sB[(q * DIM + r) * NV + c];
    }
    for (int c = 0; c < NV; ++c) sA[(r * NV + c) * NB + a] = acc[c];
  }
  __syncthreads();
  for (int i = tid; i < NX; i += 128) {
    const int a = i % NB, c = i / NB;
    R y = sY[i];
    for (int r = 0; r < DIM; ++r) y -= sA[(r * NV + c) * NB + a];
    sY[i] = y;
  }
  __syncthreads();
  for (int i = tid; i < NX; i += 128) {
    const int b = i % NB, c = i / NB;
    R acc = 0.0;
    for (int a = 0; a < NB; ++a) {
      const R l = sLc[a * NB - a * (a - 1) / 2 + b - a];
      acc += (a <= b ? l : R(0)) * sY[c * NB + a];
    }
    const size_t idx = (size_t)(c * NB + b) * ne + e;
    double o = acc;
    if (JVP) o += shift * V[idx];
    out[idx] = o;
  }
}

// w = L^{-1} sum_q w_q|J_q| psi(xi_q) f_q
template <int DIM, int NB, int NQ1, bool DIFF = false>
__global__ __launch_bounds__(64) void k_project_curved(const double* __restrict__ f, double* __restrict__ w,
                                                       CurvedTables ct, int64_t ne) {
  constexpr int NV = DIFF ? 1 : DIM + 2, NQ = ipow(NQ1, DIM), NBT = NB * (NB + 1) / 2, GV = DIM * DIM + 1;
  __shared__ double sT[NV * NB];
  const int64_t e = blockIdx.x;
  const double* wd = ct.vGeo + ((size_t)e * GV + DIM * DIM) * NQ;
  for (int i = threadIdx.x; i < NV * NB; i += 64) {
    const int a = i % NB, c = i / NB;
    double acc = 0.0;
    for (int q = 0; q < NQ; ++q) acc += wd[q] * ct.rPsiT[a * NQ + q] * f[((size_t)c * NQ + q) * ne + e];
    sT[i] = acc;
  }
  __syncthreads();
  const double* Li = ct.Linv + (size_t)e * NBT;
  for (int i = threadIdx.x; i < NV * NB; i += 64) {
    const int b = i % NB, c = i / NB;
    double acc = 0.0;
    for (int a = 0; a <= b; ++a) acc += Li[b * (b + 1) / 2 + a] * sT[c * NB + a];
    w[(size_t)(c * NB + b) * ne + e] = acc;
  }
}

// max |u| + c over the volume points; reads Ut (the modal pass on w runs first)
template <int DIM, int NB, int NQ1>
__global__ __launch_bounds__(256) void k_wave_speed_curved(double* __restrict__ partial, CurvedTables ct, Mesh m,
                                                           Phys ph) {
  constexpr int NV = DIM + 2, NQ = ipow(NQ1, DIM);
  __shared__ double red[256];
  double mx = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < (int64_t)NQ * m.ne; i += (int64_t)gridDim.x * 256) {
    const int64_t e = i % m.ne;
    const int q = (int)(i / m.ne);
    const double* ut = ct.Ut + (size_t)e * NV * NB;
    double u[NV];
    for (int c = 0; c < NV; ++c) {
      double a = 0.0;
      for (int b = 0; b < NB; ++b) a += ct.rPsiT[b * NQ + q] * ut[c * NB + b];
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
// the scalar Laplacian of the Poisson assessment: 2D P2 / P3 / P6, FP64
#define DG_CURVED_DIFF_CONFIGS(X) \
  X(1, 2, 6, 4)                   \
  X(7, 2, 10, 5)                  \
  X(8, 2, 28, 8)

}  // namespace dgk

namespace dgk {

bool has_curved(int cfg, bool diffusion) {
#define X(id, d, nb_, nq_) \
  if (cfg == id) return true;
  if (diffusion) {
    DG_CURVED_DIFF_CONFIGS(X)
  } else {
    DG_CURVED_CONFIGS(X)
  }
#undef X
  return false;
}

namespace {

template <class R>
hipError_t modal_curved(int cfg, bool jvp, const double* U, const double* V, const CurvedTablesT<R>& ct, int64_t ne,
                        hipStream_t s) {
  if (ct.diffusion) {  // FP64 only
    if constexpr (sizeof(R) == 8) {
#define X(id, d, nb_, nq_)                                                                  \
  case id: {                                                                                \
    if (jvp)                                                                                \
      k_modal_curved<R, d, nb_, true, true><<<(unsigned)ne, 64, 0, s>>>(U, V, ct, ne);      \
    else                                                                                    \
      k_modal_curved<R, d, nb_, false, true><<<(unsigned)ne, 64, 0, s>>>(U, V, ct, ne);     \
    return hipGetLastError();                                                               \
  }
      switch (cfg) { DG_CURVED_DIFF_CONFIGS(X) }
#undef X
    }
    return hipErrorInvalidValue;
  }
#define X(id, d, nb_, nq_)                                                          \
  case id: {                                                                        \
    if (jvp)                                                                        \
      k_modal_curved<R, d, nb_, true><<<(unsigned)ne, 64, 0, s>>>(U, V, ct, ne);    \
    else                                                                            \
      k_modal_curved<R, d, nb_, false><<<(unsigned)ne, 64, 0, s>>>(U, V, ct, ne);   \
    return hipGetLastError();                                                       \
  }
  switch (cfg) { DG_CURVED_CONFIGS(X) }
#undef X
  return hipErrorInvalidValue;
}

template <class R>
hipError_t face_curved(int cfg, bool jvp, const CurvedTablesT<R>& ct, const Mesh& m, const Phys& ph, hipStream_t s) {
  if (ct.diffusion) {
    if constexpr (sizeof(R) == 8) {
#define X(id, d, nb_, nq_)                                                          \
  case id: {                                                                        \
    const unsigned grid = (unsigned)m.ne * d;                                       \
    if (jvp)                                                                        \
      k_face_curved<R, d, nb_, nq_, true, true><<<grid, 64, 0, s>>>(ct, m, ph);     \
    else                                                                            \
      k_face_curved<R, d, nb_, nq_, false, true><<<grid, 64, 0, s>>>(ct, m, ph);    \
    return hipGetLastError();                                                       \
  }
      switch (cfg) { DG_CURVED_DIFF_CONFIGS(X) }
#undef X
    }
    return hipErrorInvalidValue;
  }
#define X(id, d, nb_, nq_)                                                          \
  case id: {                                                                        \
    const unsigned grid = (unsigned)m.ne * d;                                       \
    if (jvp)                                                                        \
      k_face_curved<R, d, nb_, nq_, true><<<grid, 64, 0, s>>>(ct, m, ph);           \
    else                                                                            \
      k_face_curved<R, d, nb_, nq_, false><<<grid, 64, 0, s>>>(ct, m, ph);          \
    return hipGetLastError();                                                       \
  }
  switch (cfg) { DG_CURVED_CONFIGS(X) }
#undef X
  return hipErrorInvalidValue;
}

template <class R>
hipError_t volume_curved(int cfg, bool jvp, const double* V, const CurvedTablesT<R>& ct, double* out, double shift,
                         const Mesh& m, const Phys& ph, hipStream_t s) {
  if (ct.diffusion) {
    if constexpr (sizeof(R) == 8) {
#define X(id, d, nb_, nq_)                                                                                \
  case id: {                                                                                              \
    if (jvp)                                                                                              \
      k_volume_curved<R, d, nb_, nq_, true, true><<<(unsigned)m.ne, 128, 0, s>>>(V, ct, out, shift, m, ph);  \
    else                                                                                                  \
      k_volume_curved<R, d, nb_, nq_, false, true><<<(unsigned)m.ne, 128, 0, s>>>(V, ct, out, shift, m, ph); \
    return hipGetLastError();                                                                             \
  }
      switch (cfg) { DG_CURVED_DIFF_CONFIGS(X) }
#undef X
    }
    return hipErrorInvalidValue;
  }
#define X(id, d, nb_, nq_)                                                                          \
  case id: {                                                                                        \
    if (jvp)                                                                                        \
      k_volume_curved<R, d, nb_, nq_, true><<<(unsigned)m.ne, 128, 0, s>>>(V, ct, out, shift, m, ph);  \
    else                                                                                            \
      k_volume_curved<R, d, nb_, nq_, false><<<(unsigned)m.ne, 128, 0, s>>>(V, ct, out, shift, m, ph); \
    return hipGetLastError();                                                                       \
  }
  switch (cfg) { DG_CURVED_CONFIGS(X) }
#undef X
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_modal_curved(int cfg, bool jvp, const double* U, const double* V, const CurvedTables& ct,
                               int64_t ne, hipStream_t s) {
  return modal_curved<double>(cfg, jvp, U, V, ct, ne, s);
}
hipError_t launch_face_curved(int cfg, bool jvp, const CurvedTables& ct, const Mesh& m, const Phys& ph,
                              hipStream_t s) {
  return face_curved<double>(cfg, jvp, ct, m, ph, s);
}
hipError_t launch_volume_curved(int cfg, bool jvp, const double* V, const CurvedTables& ct, double* out,
                                double shift, const Mesh& m, const Phys& ph, hipStream_t s) {
  return volume_curved<double>(cfg, jvp, V, ct, out, shift, m, ph, s);
}
hipError_t launch_modal_curved_f32(int cfg, bool jvp, const double* U, const double* V, const CurvedTablesF& ct,
                                   int64_t ne, hipStream_t s) {
  return modal_curved<float>(cfg, jvp, U, V, ct, ne, s);
}
hipError_t launch_face_curved_f32(int cfg, bool jvp, const CurvedTablesF& ct, const Mesh& m, const Phys& ph,
                                  hipStream_t s) {
  return face_curved<float>(cfg, jvp, ct, m, ph, s);
}
hipError_t launch_volume_curved_f32(int cfg, bool jvp, const double* V, const CurvedTablesF& ct, double* out,
                                    double shift, const Mesh& m, const Phys& ph, hipStream_t s) {
  return volume_curved<float>(cfg, jvp, V, ct, out, shift, m, ph, s);
}

hipError_t launch_project_curved(int cfg, const double* f, double* w, const CurvedTables& ct, int64_t ne,
                                 hipStream_t s) {
  if (ct.diffusion) {
#define X(id, d, nb_, nq_)                                                               \
  case id: {                                                                             \
    k_project_curved<d, nb_, nq_, true><<<(unsigned)ne, 64, 0, s>>>(f, w, ct, ne);       \
    return hipGetLastError();                                                            \
  }
    switch (cfg) { DG_CURVED_DIFF_CONFIGS(X) }
#undef X
    return hipErrorInvalidValue;
  }
#define X(id, d, nb_, nq_)                                                         \
  case id: {                                                                       \
    k_project_curved<d, nb_, nq_><<<(unsigned)ne, 64, 0, s>>>(f, w, ct, ne);       \
    return hipGetLastError();                                                      \
  }
  switch (cfg) { DG_CURVED_CONFIGS(X) }
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_wave_speed_curved(int cfg, const double* w, double* partial, int nblocks, const CurvedTables& ct,
                                    const Mesh& m, const Phys& ph, hipStream_t s) {
  if (ct.diffusion) return hipErrorInvalidValue;  // the wave speed of the compressible equations
#define X(id, d, nb_, nq_)                                                                  \
  case id: {                                                                                \
    k_modal_curved<double, d, nb_, false><<<(unsigned)m.ne, 64, 0, s>>>(w, w, ct, m.ne);            \
    k_wave_speed_curved<d, nb_, nq_><<<nblocks, 256, 0, s>>>(partial, ct, m, ph);           \
    return hipGetLastError();                                                               \
  }
  switch (cfg) { DG_CURVED_CONFIGS(X) }
#undef X
  return hipErrorInvalidValue;
}

}  // namespace dgk
