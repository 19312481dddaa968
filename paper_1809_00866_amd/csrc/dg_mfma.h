// MFMA kernels for the 3D residual and exact Jacobian-vector product
// (gfx950: v_mfma_f64_16x16x4, v_mfma_f32_16x16x4 and the BF16 16x16x16
// instruction), instantiated per precision in dg_mfma_f64.hip,
// dg_mfma_f32.hip and dg_mfma_bf16.hip.  Same arithmetic as the reference kernels in
// dg_kernels.hip (eq. NSdiscrRes with BR2 liftings, Sec. 2.1-2.2); the dense
// contractions run as MFMA tiles of 16 elements (or faces) x 16 quadrature
// points, the pointwise fluxes on the vector ALU.
//
// MFMA operand layout (FP64 16x16x4): A[i][k] in lane i + 16k, B[k][j] in
// lane j + 16k, D[i][j] in lane j + 16 (i % 4), register i / 4.  With
// g = lane / 16 and col = lane % 16 a lane therefore holds rows g, g+4, g+8,
// g+12 of column col, which is exactly the B operand of a following MFMA
// whose k-steps walk those rows in order.
//
// Gradient kernel (one wave per tile of 16 elements, direction and
// value/tangent): the modal corrected gradients G_p = d_p U + R^K_p by MFMA
// from the element and its +/-p neighbours, written to a global buffer.
// Volume kernel (one workgroup = 4 waves = 16 elements):
//   1. modal fields per element (U and the three G_p) are loaded in
//      B-fragment order and kept in registers (each wave owns a quarter of the
//      (value/tangent, field, variable) column blocks);
//   2. per block of 16 quadrature points: MFMA interpolation -> LDS stage ->
//      one thread per (point, element) evaluates the volume flux (dual numbers
//      for Jv) -> LDS stage -> MFMA weighted-transpose projection into
//      per-wave accumulators (rows = modes, columns = elements);
//   3. the 2*dim face fluxes of every element are projected with MFMA
//      (gathered from the face-flux buffer, no atomics) and the result is
//      written once.
// Face kernel (one workgroup = 4 waves = 16 faces of one direction): MFMA
// traces of both sides (values, averaged gradients, averaged lifting) -> LDS
// stage -> one thread per (face point, face) evaluates the numerical flux.
// With one 16-point block (P2, P3) only the two value traces and the normal
// averaged gradient contract over modes; the tangential averaged gradients
// and the averaged lifting are point-to-point products of those traces.
#pragma once
#include "dg_device.h"

namespace dgk {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// MFMA precision policy.  Both 16x16x4 instructions take A[i][k] from lane
// i + 16k and B[k][j] from lane j + 16k; they differ in where the result
// rows land: FP64 returns row g + 4r of column l%16 in register r of lane
// group g = l/16, FP32 returns row 4g + r.  A result used directly as the next
// B operand therefore carries, at fragment (k-step ks, lane group g), the
// mode g + 4 ks (FP64) or 16 (ks/4) + 4 g + ks%4 (FP32); fields loaded from
// memory into such fragments follow the same order, and the interpolation
// table's columns are built to match (4 k-steps per 16 modes in FP32).
template <class R> struct MP;
template <> struct MP<double> {
  using frag = f64x4;
  static constexpr bool kBf16 = false;
  static DEV frag mma(double a, double b, frag c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static DEV int drow(int g, int r) { return g + 4 * r; }
  static DEV int bmode(int g, int ks) { return g + 4 * ks; }
  static constexpr int ksv(int nb) { return (nb + 3) / 4; }
};
template <> struct MP<float> {
  using frag = f32x4;
  static constexpr bool kBf16 = false;
  static DEV frag mma(float a, float b, frag c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static DEV int drow(int g, int r) { return 4 * g + r; }
  static DEV int bmode(int g, int ks) { return 16 * (ks >> 2) + 4 * g + (ks & 3); }
  static constexpr int ksv(int nb) { return 4 * ((nb + 15) / 16); }
};
// BF16 contractions with FP32 accumulation (the kernels otherwise run as the
// FP32 operator: FP32 tables, stages and pointwise arithmetic).  The BF16
// 16x16x16 instruction takes four k values per lane, A[i][4g + j] and
// B[4g + j][col] in slot j of lane i + 16g (resp. col + 16g), and returns
// D[4g + r][col] in register r: the result layout of the FP32 16x16x4
// instruction.  Four consecutive FP32 k-steps, whose lane group g holds one k
// value of A and the same k value of B, therefore make one BF16 MFMA with
// k-step j in slot j: the products pair up lane by lane whatever rows the
// k-steps stand for, so every FP32 operand table and fragment order serves
// unchanged.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
struct MPB : MP<float> {
  static constexpr bool kBf16 = true;
};

// The mean mode of a state (b = 0, the element average: e.g. about 33 for the
// total energy of the low-Mach workloads, against fluctuations of order 1e-2 of
// it) is kept out of the BF16 products: its contribution to the value traces,
// the value fields at the volume points and the corrected gradients is added
// in FP32 (A(row, mode 0) * U_0), and the BF16 chains see a zero there.  BF16
// rounding of the mean alone would make a relative residual error of 3e-2; the
// remaining modes give 1.6e-3 (P3).
//
// acc + sum_{ks < NK} A(ks) B(ks) over the k-steps of one contraction chain:
// one MFMA per k-step in FP64 / FP32, one BF16 MFMA per group of four k-steps
// (operands rounded to BF16 to nearest even, the last group zero-padded).
template <class MM, int NK, class FA, class FB>
DEV typename MM::frag chain(const FA& a, const FB& b, typename MM::frag d) {
  if constexpr (MM::kBf16) {
#pragma unroll
    for (int kb = 0; kb < (NK + 3) / 4; ++kb) {
      bf16x4 av, bv;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int ks = 4 * kb + j;
        av[j] = (__bf16)(ks < NK ? (float)a(ks) : 0.0f);
        bv[j] = (__bf16)(ks < NK ? (float)b(ks) : 0.0f);
      }
      d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, d, 0, 0, 0);
    }
  } else {
#pragma unroll
    for (int ks = 0; ks < NK; ++ks) d = MM::mma(a(ks), b(ks), d);
  }
  return d;
}

// FP64 contractions over the modes whose last 16-row mode block holds at most
// 4 live rows (P3: modes 16-19, P4: 32-34) run that block on the 4-block
// 4x4x4 instruction instead of a 16x16x4 tile three quarters zeros: the same
// rate per flop, a quarter of the passes.  Block v of the instruction takes
// A[w][k] from lane 16 k + 4 v + w (the FP64 tables' last mode block holds
// row l % 4 in lane l), B[k][u] from lane 16 k + 4 v + u -- the 16x16x4 B
// fragment unchanged, column 4 v + u -- and returns D[w][u] in lane
// 16 w + 4 v + u: row g = lane / 16 of column lane % 16, where the 16x16x4
// result keeps row g in its register 0 (measured on the device).
template <class MM, int NB>
constexpr bool rem4() {
  constexpr int MB = (NB + 15) / 16;
  return std::is_same<MM, MP<double>>::value && MB >= 2 && NB - 16 * (MB - 1) <= 4;
}
template <int NK, class FA, class FB>
DEV double chain4(const FA& a, const FB& b, double d) {
#pragma unroll
  for (int ks = 0; ks < NK; ++ks) d = __builtin_amdgcn_mfma_f64_4x4x4f64(a(ks), b(ks), d, 0, 0, 0);
  return d;
}

// Tile processed by this workgroup.  Workgroups are dispatched round-robin
// over the 8 XCDs (each with its own L2); giving every XCD a contiguous range
// of tiles keeps a tile's face neighbours (x: adjacent tiles, y: 2 tiles
// away, z: 64 tiles away on a 32^3 lattice) in the same L2.
DEV int64_t xcd_tile(int64_t bid, int64_t nblk) {
  constexpr int64_t kXcd = 8;
  const int64_t q = nblk / kXcd, r = nblk % kXcd, x = bid % kXcd;
  return x * q + (x < r ? x : r) + bid / kXcd;
}

// ------------------------------------------------------------------ corrected gradients
// Modal corrected gradients G_p = d_p U + R^K_p of every element (the modal
// form of the BR2 consistent gradient on affine elements):
//   G_p = L_{p,0} U_e + L_{p,1} U_{e+p} + L_{p,2} U_{e-p},
// one wave per (tile of 16 elements, direction p, value/tangent s), all
// variables; B fragments straight from global memory (no LDS, no barriers).
// Output layout Gm[s][p][c][b][e].  The tangent (s = 1) reads the element's
// own coefficients from V and its neighbours' from Vn (V for the ordinary Jv;
// zeros when probing the diagonal blocks element by element).
template <class R, int NB, class MM>
__global__ __launch_bounds__(64) void k_grad_mfma(const double* __restrict__ U, const double* __restrict__ V,
                                                  const double* __restrict__ Vn, R* __restrict__ Gm,
                                                  const R* __restrict__ lA, Mesh m) {
  using F = typename MM::frag;
  constexpr int DIM = 3, NV = 5;
  constexpr int KSB = (NB + 3) / 4, MB = (NB + 15) / 16;
  const int lane = threadIdx.x;
  const int g = lane >> 4, col = lane & 15;
  const int64_t ne = m.ne;
  const int64_t e = xcd_tile(blockIdx.x, gridDim.x) * 16 + col;
  const bool ev = e < ne;
  const int p = blockIdx.y, s = blockIdx.z;
  const double* __restrict__ X = (s == 0) ? U : V;
  const double* __restrict__ Xn = (s == 0) ? U : Vn;
  // Loads use clamped, always valid addresses and a select instead of a branch
  // (a branch per load keeps the scheduler from batching them).
  const int64_t ec = ev ? e : ne - 1;
  const int64_t es[3] = {ec, m.nbr[(2 * p + 1) * ne + ec], m.nbr[(2 * p) * ne + ec]};  // element, +p, -p
#pragma unroll 1
  for (int c = 0; c < NV; ++c) {
    R bf[3 * KSB], m0[3];
#pragma unroll
    for (int ks3 = 0; ks3 < 3 * KSB; ++ks3) {
      const int src = ks3 / KSB, bp = g + 4 * (ks3 % KSB);
      const R x = (R)(src == 0 ? X : Xn)[(size_t)(c * NB + (bp < NB ? bp : NB - 1)) * ne + es[src]];
      bf[ks3] = (ev && bp < NB) ? x : R(0);
    }
    if constexpr (MM::kBf16) {  // mean modes in FP32, out of the BF16 chain
#pragma unroll
      for (int src = 0; src < 3; ++src) {
        m0[src] = ev ? (R)(src == 0 ? X : Xn)[(size_t)(c * NB) * ne + es[src]] : R(0);
        if (g == 0) bf[src * KSB] = R(0);
      }
    }
    // FP64 P4: one mode block at a time (all three unrolled hold their A
    // operands in flight and leave one wave per SIMD)
    constexpr bool kRem = rem4<MM, NB>();
    constexpr int MBM = kRem ? MB - 1 : MB;  // 16x16x4 mode blocks
    constexpr int kMbUnroll = (sizeof(R) == 8 && MB > 2) ? 1 : MB;
#pragma unroll kMbUnroll
    for (int mb = 0; mb < MBM; ++mb) {
      const R* __restrict__ la = lA + ((size_t)p * MB + mb) * 3 * KSB * 64 + lane;
      F d = chain<MM, 3 * KSB>([&](int ks3) { return la[ks3 * 64]; }, [&](int ks3) { return bf[ks3]; },
                               F{0, 0, 0, 0});
      if constexpr (MM::kBf16) {
        const R* __restrict__ l0 = lA + ((size_t)p * MB + mb) * 3 * KSB * 64;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int src = 0; src < 3; ++src) d[r] += l0[src * KSB * 64 + MM::drow(g, r)] * m0[src];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int b = 16 * mb + MM::drow(g, r);
        if (ev && b < NB) Gm[((size_t)((s * DIM + p) * NV + c) * NB + b) * ne + e] = d[r];
      }
    }
    if constexpr (kRem) {  // the last mode block: row g of column col
      const R* __restrict__ la = lA + ((size_t)p * MB + MB - 1) * 3 * KSB * 64 + lane;
      const double d0 = chain4<3 * KSB>([&](int ks3) { return la[ks3 * 64]; }, [&](int ks3) { return bf[ks3]; }, 0.0);
      const int b = 16 * (MB - 1) + g;
      if (ev && b < NB) Gm[((size_t)((s * DIM + p) * NV + c) * NB + b) * ne + e] = d0;
    }
  }
}

// ------------------------------------------------------------------ volume
// OCC is the minimum number of waves per SIMD the register allocation must
// allow (launch bound): 2 caps a lane at 256 registers, 1 lets it use 512
// (the accumulation registers too) without spilling.  The default is 1 for
// FP64 P4 (measured faster than occupancy 2 with spills) and 2 otherwise;
// the autotuner may pick the other one per configuration.
template <class R, int NB>
constexpr int volume_occupancy() { return (NB > 20 && sizeof(R) == 8) ? 1 : 2; }

// FG: the corrected gradients are formed in the kernel from the element and
// its +/-p neighbours (the chains of k_grad_mfma, same operands and order,
// so the same bits) instead of being read from the buffer Gm.
// Hm: the face fluxes read on the element's -p faces; Vn: the neighbours'
// tangent coefficients of the corrected gradients formed in the kernel (FG).
// H and V for the ordinary operator; probing the diagonal blocks element by
// element passes the fluxes of the +face neighbours' tangents and zeros.
template <class R, int NB, int NQ1, int KL, bool JVP, class MM, int OCC, bool FG>
__global__ __launch_bounds__(256, OCC) void k_volume_mfma(const double* __restrict__ U, const double* __restrict__ V,
                                                     const double* __restrict__ Vn,
                                                     const R* __restrict__ Gm, const R* __restrict__ H,
                                                     const R* __restrict__ Hm, double* __restrict__ out,
                                                     double shift, MTablesT<R> mt, Mesh m, Phys ph) {
  using T = typename Scalar<JVP, R>::type;
  using F = typename MM::frag;
  constexpr int DIM = 3, NV = 5;
  constexpr int NQ = ipow(NQ1, 3), NFQ = ipow(NQ1, 2);
  constexpr int KSB = (NB + 3) / 4, MB = (NB + 15) / 16, RBQ = (NQ + 15) / 16;
  constexpr int KSV = MM::ksv(NB);            // fragment k-steps of the modal fields
  constexpr int KSP = DIM * 4, KSF = (NFQ + 3) / 4;
  constexpr int NS = JVP ? 2 : 1;
  constexpr int NFC = (1 + DIM) * NV;        // (field, variable) pairs per value/tangent
  constexpr int NCBW = NS * NFC / 4;          // column blocks per wave
  constexpr int NPB = NV * MB;                // projection accumulator blocks (variable, mode block)
  constexpr int NPBW = (NPB + 3) / 4;
  // FP64 P3/P4: the last mode block of every contraction over the modes on
  // the 4x4x4 instruction (rem4); the 16x16x4 projection blocks come first in
  // the block order, so they spread evenly over the waves
  constexpr bool kRem = rem4<MM, NB>();
  constexpr int MBM = kRem ? MB - 1 : MB;
  auto pblock = [](int pb, int& c, int& mb) {
    if (pb < NV * MBM) {
      c = pb / MBM;
      mb = pb % MBM;
    } else {
      c = pb - NV * MBM;
      mb = MB - 1;
    }
  };
  static_assert(NFC % 4 == 0, "column blocks must split over 4 waves");
  __shared__ R stage[NFC][16][16];
  __shared__ R ptab[MB * KSP * 64];  // projection table of the current point block (A operands of every wave)

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, col = lane & 15;
  const int64_t ne = m.ne;
  const int64_t e0 = xcd_tile(blockIdx.x, gridDim.x) * 16;
  const int64_t e = e0 + col;
  const bool ev = e < ne;
  const int64_t ec = ev ? e : ne - 1;  // clamped element: loads stay branch-free
  const double kap = ph.mu * ph.gamma / (ph.prandtl * (ph.gamma - 1.0));

  // ---- 1. modal fields in B-fragment order: Bf[i][ks] = X[b = bmode(g, ks)][e],
  // X = U (or V) for f = 0 and the corrected gradient G_f for f = 1..3.
  R Bf[NCBW][KSV];
  R m0[NCBW];  // BF16: the mean mode of the value fields, applied in FP32
#pragma unroll
  for (int i = 0; i < NCBW; ++i) {
    const int s = i / (NFC / 4);
    const int fc = wave + 4 * (i % (NFC / 4));
    const int f = fc / NV, c = fc % NV;
    const double* __restrict__ X = ((s == 0) ? U : V) + (size_t)c * NB * ne;
    const R* __restrict__ Gf = FG ? nullptr : Gm + (size_t)((s * DIM + (f > 0 ? f - 1 : 0)) * NV + c) * NB * ne;
    m0[i] = R(0);
    if (f == 0) {
#pragma unroll
      for (int ks = 0; ks < KSV; ++ks) {
        const int b = MM::bmode(g, ks);
        const R x = (R)X[(size_t)(b < NB ? b : NB - 1) * ne + ec];
        Bf[i][ks] = (ev && b < NB) ? x : R(0);
      }
      if constexpr (MM::kBf16) {
        m0[i] = ev ? (R)X[ec] : R(0);
        if (g == 0) Bf[i][0] = R(0);  // mode bmode(0, 0) = 0
      }
    } else if constexpr (FG) {
      // G_p = L_{p,0} X_e + L_{p,1} X_{e+p} + L_{p,2} X_{e-p} by MFMA, the
      // chains of k_grad_mfma: result block mb, register r holds mode
      // 16 mb + drow(g, r) = bmode(g, 4 mb + r), i.e. k-step 4 mb + r of
      // this B fragment (modes >= NB come out zero: zero table rows)
      const int pd = f - 1;
      const int64_t es3[3] = {ec, m.nbr[(2 * pd + 1) * ne + ec], m.nbr[(2 * pd) * ne + ec]};
      const double* __restrict__ Xn = ((s == 0) ? U : Vn) + (size_t)c * NB * ne;
      R bf3[3 * KSB], g0[3];
#pragma unroll
      for (int ks3 = 0; ks3 < 3 * KSB; ++ks3) {
        const int src = ks3 / KSB, bp = g + 4 * (ks3 % KSB);
        const R x = (R)(src == 0 ? X : Xn)[(size_t)(bp < NB ? bp : NB - 1) * ne + es3[src]];
        bf3[ks3] = (ev && bp < NB) ? x : R(0);
      }
      if constexpr (MM::kBf16) {
#pragma unroll
        for (int src = 0; src < 3; ++src) {
          g0[src] = ev ? (R)(src == 0 ? X : Xn)[es3[src]] : R(0);
          if (g == 0) bf3[src * KSB] = R(0);
        }
      }
#pragma unroll
      for (int mb = 0; mb < MBM; ++mb) {
        const R* __restrict__ la = mt.lA + ((size_t)pd * MB + mb) * 3 * KSB * 64 + lane;
        F d = chain<MM, 3 * KSB>([&](int ks3) { return la[ks3 * 64]; }, [&](int ks3) { return bf3[ks3]; },
                                 F{0, 0, 0, 0});
        if constexpr (MM::kBf16) {
          const R* __restrict__ l0 = mt.lA + ((size_t)pd * MB + mb) * 3 * KSB * 64;
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int src = 0; src < 3; ++src) d[r] += l0[src * KSB * 64 + MM::drow(g, r)] * g0[src];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (4 * mb + r < KSV) Bf[i][4 * mb + r] = d[r];
      }
      if constexpr (kRem) {  // k-step 4 (MB - 1) holds mode 16 (MB - 1) + g
        const R* __restrict__ la = mt.lA + ((size_t)pd * MB + MB - 1) * 3 * KSB * 64 + lane;
        Bf[i][4 * (MB - 1)] =
            chain4<3 * KSB>([&](int ks3) { return la[ks3 * 64]; }, [&](int ks3) { return bf3[ks3]; }, 0.0);
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < KSV; ++ks) {
        const int b = MM::bmode(g, ks);
        const R x = Gf[(size_t)(b < NB ? b : NB - 1) * ne + ec];
        Bf[i][ks] = (ev && b < NB) ? x : R(0);
      }
    }
  }

  F acc[NPBW];
#pragma unroll
  for (int i = 0; i < NPBW; ++i) acc[i] = F{0, 0, 0, 0};

  const int ql = tid >> 4, et = tid & 15;  // pointwise mapping: (point in block, element)
  for (int rb = 0; rb < RBQ; ++rb) {
    // stage this block's projection table (read after the barriers below;
    // the previous block's projection ended with a barrier)
    for (int idx = tid; idx < MB * KSP * 64; idx += 256) ptab[idx] = mt.pA[(size_t)rb * MB * KSP * 64 + idx];
    __syncthreads();
    R st[NS][NFC];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      // ---- 2a. MFMA interpolation of this wave's column blocks
#pragma unroll
      for (int i = s * (NFC / 4); i < (s + 1) * (NFC / 4); ++i) {
        const int fc = wave + 4 * (i % (NFC / 4));
        const R* __restrict__ va = mt.vA + (size_t)rb * KSV * 64 + lane;
        F d = chain<MM, KSV>([&](int ks) { return va[ks * 64]; }, [&](int ks) { return Bf[i][ks]; },
                             F{0, 0, 0, 0});
        if constexpr (MM::kBf16) {
          if (fc < NV) {  // value field: its mean mode (k-step 0, lane group 0 of the table)
#pragma unroll
            for (int r = 0; r < 4; ++r) d[r] += mt.vA[(size_t)rb * KSV * 64 + MM::drow(g, r)] * m0[i];
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) stage[fc][MM::drow(g, r)][col] = d[r];
      }
      __syncthreads();
#pragma unroll
      for (int fc = 0; fc < NFC; ++fc) st[s][fc] = stage[fc][ql][et];
      __syncthreads();
    }
    // ---- 2b. pointwise volume flux F = F^c - F^v (tangent for Jv), written to
    // the stage direction by direction (every read of the stage is complete).
    const int q = 16 * rb + ql;
    if (q < NQ && e0 + et < ne) {
      T u[NV], G[NV][DIM];
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        if constexpr (JVP) {
          u[c] = T(st[0][c], st[NS - 1][c]);
#pragma unroll
          for (int j = 0; j < DIM; ++j) G[c][j] = T(st[0][(1 + j) * NV + c], st[NS - 1][(1 + j) * NV + c]);
        } else {
          u[c] = st[0][c];
#pragma unroll
          for (int j = 0; j < DIM; ++j) G[c][j] = st[0][(1 + j) * NV + c];
        }
      }
      T rinv, vel[DIM], pr;
      primitives<T, DIM>(u, ph.gamma, rinv, vel, pr);
      ViscPrep<T, DIM> vp;
      visc_prep<T, DIM>(u, G, ph.gamma, vp);
#pragma unroll
      for (int j = 0; j < DIM; ++j) {
        T Fc[NV], Fv[NV];
        conv_flux_dir<T, DIM>(u, vel, pr, j, Fc);
        visc_flux_dir<T, DIM>(vp, j, ph.mu, kap, Fv);
#pragma unroll
        for (int c = 0; c < NV; ++c) stage[j * NV + c][ql][et] = out_part(Fc[c] - Fv[c]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < DIM; ++j)
#pragma unroll
        for (int c = 0; c < NV; ++c) stage[j * NV + c][ql][et] = R(0);
    }
    __syncthreads();
    // ---- 2c. MFMA projection: R[b][e] += -sum_{j,q} w|J| d_j phi(q,b) F_j(q,e)
#pragma unroll
    for (int i = 0; i < NPBW; ++i) {
      const int pb = wave + 4 * i;
      if (pb < NPB) {
        int c, mb;
        pblock(pb, c, mb);
        auto aop = [&](int ks) { return ptab[(mb * KSP + ks) * 64 + lane]; };
        auto bop = [&](int ks) {
          const int k = g + 4 * ks;
          return stage[(k >> 4) * NV + c][k & 15][col];
        };
        if (kRem && mb == MB - 1) {
          if constexpr (kRem) acc[i][0] = chain4<KSP>(aop, bop, acc[i][0]);
        } else {
          acc[i] = chain<MM, KSP>(aop, bop, acc[i]);
        }
      }
    }
    __syncthreads();
  }

  // ---- 3. face contributions (+ on the element's own +p faces, - on its -p faces);
  // the face projection table of direction p is staged in the idle stage buffer
  static_assert(2 * MB * KSF * 64 <= NFC * 256, "face table slice must fit the stage buffer");
  R* ftab = &stage[0][0][0];
#pragma unroll
  for (int p = 0; p < DIM; ++p) {
    for (int idx = tid; idx < 2 * MB * KSF * 64; idx += 256) ftab[idx] = mt.fA[(size_t)p * 2 * MB * KSF * 64 + idx];
    __syncthreads();
    const int64_t em = m.nbr[(2 * p) * ne + ec];
#pragma unroll
    for (int i = 0; i < NPBW; ++i) {
      const int pb = wave + 4 * i;
      if (pb < NPB) {
        int c, mb;
        pblock(pb, c, mb);
        // k-steps (side, face point) with side 0 (the -p face, read from the
        // -p neighbour's record) first
        auto aop = [&](int k2) {
          const int side = k2 / KSF, ks = k2 % KSF;
          return ftab[((side * MB + mb) * KSF + ks) * 64 + lane];
        };
        auto bop = [&](int k2) {
          const int side = k2 / KSF, ks = k2 % KSF;
          const int fq = g + 4 * ks;
          const R h = (side ? H : Hm)[((size_t)(p * NV + c) * NFQ + (fq < NFQ ? fq : NFQ - 1)) * ne + (side ? ec : em)];
          return (ev && fq < NFQ) ? h : R(0);
        };
        if (kRem && mb == MB - 1) {
          if constexpr (kRem) acc[i][0] = chain4<2 * KSF>(aop, bop, acc[i][0]);
        } else {
          acc[i] = chain<MM, 2 * KSF>(aop, bop, acc[i]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < NPBW; ++i) {
    const int pb = wave + 4 * i;
    if (pb < NPB) {
      int c, mb;  // the last mode block holds rows 16 mb + g in register 0 only
      pblock(pb, c, mb);
      if (ev) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int b = 16 * mb + MM::drow(g, r);
          if (b < NB) {
            const size_t idx = (size_t)(c * NB + b) * ne + e;
            double a = (double)acc[i][r];
            if (JVP) a += shift * V[idx];
            out[idx] = a;
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------------ faces
// P4 (35 modes, two face-point blocks): the trace table of the current point
// block is staged in LDS next to the stage buffer (reading the A operands from
// L2 left the MFMA chains waiting); in FP64 the kernel also runs at one wave
// per SIMD, which makes room for the table and removes the register spills of
// the dual-number flux.  The smaller configurations read the table from L2 at
// occupancy 2 or more (staging it measured slower there).
// The staged FP64 P4 table takes 116 KB of LDS, one workgroup per CU: that
// configuration exists at occupancy 1 only.
template <class R, int NB>
struct FaceTab {
  static constexpr bool lds = NB > 20;
  static constexpr int occupancy = (lds && sizeof(R) == 8) ? 1 : 2;
  static constexpr bool only_default = lds && sizeof(R) == 8;
  // work units (tile, direction) in a 1D grid with the direction fastest (the
  // three directions of a tile back to back on one XCD) instead of one grid
  // row per direction: P4 FP32 face Jv 0.177 -> 0.165 ms at 24^3, FP64 level;
  // at P3 the row form measured 1 % faster in FP64
  static constexpr bool dir_fast = lds;
};

template <class R, int NB, int NQ1, bool JVP, int P, class MM>
DEV void face_mfma_body(const double* __restrict__ U, const double* __restrict__ V,
                        const double* __restrict__ Vr, R* __restrict__ H,
                        const MTablesT<R>& mt, const Mesh& m, const Phys& ph, R (*stage)[16][16], R* ttab,
                        int64_t tile) {
  using T = typename Scalar<JVP, R>::type;
  using F = typename MM::frag;
  constexpr int DIM = 3, NV = 5;
  constexpr int NFQ = ipow(NQ1, 2);
  constexpr int KSB = (NB + 3) / 4, RBF = (NFQ + 15) / 16;
  constexpr int NS = JVP ? 2 : 1;
  constexpr int NCH = 6;                     // uL, uR, G_1..3 (averaged), {r}
  static_assert(NV == 5, "balanced split: 4 waves own variables 0..3, variable 4 is shared");
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, col = lane & 15;
  const int64_t ne = m.ne;
  const int64_t e0 = (FaceTab<R, NB>::dir_fast ? tile : xcd_tile(blockIdx.x, gridDim.x)) * 16;
  const int64_t e = e0 + col;
  const bool ev = e < ne;
  const int64_t ec = ev ? e : ne - 1;  // clamped element: loads stay branch-free
  const int64_t er = m.nbr[(2 * P + 1) * ne + ec];
  const double kap = ph.mu * ph.gamma / (ph.prandtl * (ph.gamma - 1.0));

  // B fragments of (value/tangent s, variable c): k-steps 0..KSB-1 from the
  // owner, KSB..2KSB-1 from the +P neighbour
  // (BF16: entries 2KSB, 2KSB + 1 hold the mean modes of both sides, applied
  // in FP32, and the chains see zeros at mode 0)
  // (tangent: the owner's coefficients from V, the neighbour's from Vr)
  auto load_b = [&](int s, int c, R* bf) {
    const double* __restrict__ X = (s == 0) ? U : V;
    const double* __restrict__ Xr = (s == 0) ? U : Vr;
#pragma unroll
    for (int ks2 = 0; ks2 < 2 * KSB; ++ks2) {
      const int b = g + 4 * (ks2 < KSB ? ks2 : ks2 - KSB);
      const int64_t es = ks2 < KSB ? ec : er;
      const R x = (R)(ks2 < KSB ? X : Xr)[(size_t)(c * NB + (b < NB ? b : NB - 1)) * ne + es];
      bf[ks2] = (ev && b < NB) ? x : R(0);
    }
    if constexpr (MM::kBf16) {
      bf[2 * KSB] = ev ? (R)X[(size_t)(c * NB) * ne + ec] : R(0);
      bf[2 * KSB + 1] = ev ? (R)Xr[(size_t)(c * NB) * ne + er] : R(0);
      if (g == 0) bf[0] = bf[KSB] = R(0);
    }
  };
  // trace channel ch of one column block into the stage; the trace table of
  // the current point block is read from LDS when the kernel stages it there
  constexpr bool kTabLds = FaceTab<R, NB>::lds;
  auto put = [&](int ch, int c, const F& d) {
#pragma unroll
    for (int r = 0; r < 4; ++r) stage[ch * NV + c][MM::drow(g, r)][col] = d[r];
  };
  // channel 0 (uL) contracts the owner's k-steps, channel 1 (uR) the
  // neighbour's, the others both
  auto trace_d = [&](int rbf, int ch, const R* bf) {
    auto a_of = [&](int ks2) {
      return kTabLds ? ttab[(ch * 2 * KSB + ks2) * 64 + lane]
                     : mt.tA[((((size_t)P * RBF + rbf) * NCH + ch) * 2 * KSB + ks2) * 64 + lane];
    };
    const F z = {0, 0, 0, 0};
    F d;
    if (ch == 0)
      d = chain<MM, KSB>(a_of, [&](int k) { return bf[k]; }, z);
    else if (ch == 1)
      d = chain<MM, KSB>([&](int k) { return a_of(KSB + k); }, [&](int k) { return bf[KSB + k]; }, z);
    else
      d = chain<MM, 2 * KSB>(a_of, [&](int k) { return bf[k]; }, z);
    if constexpr (MM::kBf16) {  // mean modes of both sides (k-steps 0 and KSB, lane group 0)
      auto a_row = [&](int ks2, int row) {
        return kTabLds ? ttab[(ch * 2 * KSB + ks2) * 64 + row]
                       : mt.tA[((((size_t)P * RBF + rbf) * NCH + ch) * 2 * KSB + ks2) * 64 + row];
      };
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = MM::drow(g, r);
        if (ch != 1) d[r] += a_row(0, row) * bf[2 * KSB];
        if (ch != 0) d[r] += a_row(KSB, row) * bf[2 * KSB + 1];
      }
    }
    return d;
  };
  auto trace = [&](int rbf, int ch, int c, const R* bf) { put(ch, c, trace_d(rbf, ch, bf)); };
  // One point block: the tangential components of the averaged gradient are
  // d/dx_t of the averaged trace {U} = (uL + uR)/2 on the face points (exact:
  // the points resolve the trace polynomial), and the averaged lifting is a map
  // of the jump uL - uR on the same points (the quadrature that defines it):
  // 16-point contractions instead of ones over the modes of both sides.  The
  // trace results, held as MFMA result rows, are the B operand of these
  // products as they stand.
  constexpr bool kPts = RBF == 1;
  constexpr int KT = std::is_same<R, double>::value ? (NFQ + 3) / 4 : 4;
  auto point_channels = [&](int c, const R* bf) {
    const F dL = trace_d(0, 0, bf), dR = trace_d(0, 1, bf);
    put(0, c, dL);
    put(1, c, dR);
    R avg[4], jmp[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      avg[r] = R(0.5) * (dL[r] + dR[r]);
      jmp[r] = dL[r] - dR[r];
    }
#pragma unroll
    for (int jt = 0; jt < 3; ++jt) {
      const F d = chain<MM, KT>([&](int ks) { return mt.dA[((P * 3 + jt) * 4 + ks) * 64 + lane]; },
                                [&](int ks) { return jt < 2 ? avg[ks] : jmp[ks]; }, F{0, 0, 0, 0});
      const int ch = jt == 2 ? 5 : 2 + ((jt == 0) ? (P == 0 ? 1 : 0) : (P == 2 ? 1 : 2));
      put(ch, c, d);
    }
  };
  // all six channels of variable c from its B fragments
  auto channels = [&](int rbf, int c, const R* bf) {
    if constexpr (kPts) {
      point_channels(c, bf);
      trace(rbf, 2 + P, c, bf);
    } else {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) trace(rbf, ch, c, bf);
    }
  };
  // Work split.  Balanced (one or two face-point blocks, i.e. every compiled
  // configuration): wave w traces the channels of variable w.  With one point block wave 3 keeps only
  // the trace and point products (uL, uR, tangential G, {r}) of variables 3
  // and 4 (the point products need both traces in its own registers) and the
  // normal-gradient chains of variables 3 and 4 go to waves 1 and 2: 32/42/42/44
  // MFMA k-steps per wave and value/tangent pass at P3.  At P4 (all channels
  // modal) the channels of variable 4 are shared out as {uL, G_1}, {uR, G_2},
  // {G_3}, {r}: at most 117 k-steps per wave and pass instead of the 180 of
  // whole column blocks (P4 face Jv 0.402 -> 0.336 ms FP64, 0.186 -> 0.177 ms
  // FP32; P3 FP32 0.110 -> 0.096 ms).  Otherwise (more point blocks) column
  // block cb = w + 4i goes to wave w whole.
  constexpr bool kBalanced = RBF <= 2;
  constexpr int NCB = NS * NV;               // (value/tangent, variable) column blocks
  constexpr int NCBW = kBalanced ? NS : (NCB + 3) / 4;
  constexpr int NBF = 2 * KSB + (MM::kBf16 ? 2 : 0);  // fragment entries (BF16: + the two mean modes)
  R Bf[NCBW][NBF];
#pragma unroll
  for (int i = 0; i < NCBW; ++i) {
    const int cb = kBalanced ? i * NV + wave : wave + 4 * i;
    if (cb < NCB) {
      load_b(cb / NV, cb % NV, Bf[i]);
    } else {
#pragma unroll
      for (int ks2 = 0; ks2 < NBF; ++ks2) Bf[i][ks2] = R(0);
    }
  }

  const int fql = tid >> 4, ft = tid & 15;
  for (int rbf = 0; rbf < RBF; ++rbf) {
    if constexpr (kTabLds) {
      // the previous point block's last table reads precede its final barrier
      const R* __restrict__ src = mt.tA + ((size_t)P * RBF + rbf) * NCH * 2 * KSB * 64;
      for (int idx = tid; idx < NCH * 2 * KSB * 64; idx += 256) ttab[idx] = src[idx];
      __syncthreads();
    }
    R st[NS][NCH * NV];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if constexpr (kBalanced) {
        R Bs[NBF];
        if constexpr (kPts) {
          if (wave != 0) load_b(s, wave == 1 ? 3 : 4, Bs);
          if (wave == 3) {
            point_channels(3, Bf[s]);
            point_channels(4, Bs);
          } else {
            if (wave != 0) trace(rbf, 2 + P, wave == 1 ? 3 : 4, Bs);
            channels(rbf, wave, Bf[s]);
          }
        } else {
          load_b(s, 4, Bs);
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch) {
            const int owner = ch < 4 ? (ch & 1) : ch - 2;
            if (owner == wave) trace(rbf, ch, 4, Bs);
          }
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch) trace(rbf, ch, wave, Bf[s]);
        }
      } else {
#pragma unroll
        for (int i = 0; i < NCBW; ++i) {
          const int cb = wave + 4 * i;
          if (cb < NCB && cb / NV == s) channels(rbf, cb % NV, Bf[i]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < NCH * NV; ++k) st[s][k] = stage[k][fql][ft];
      __syncthreads();
    }
    if constexpr (JVP) {
      if (ph.stab_only) {  // tangent through the face lifting channel {r} only
#pragma unroll
        for (int k = 0; k < 5 * NV; ++k) st[NS - 1][k] = R(0);
      }
    }
    const int fq = 16 * rbf + fql;
    const int64_t ef = e0 + ft;
    if (fq < NFQ && ef < ne) {
      T uL[NV], uR[NV], Ga[NV][DIM];
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        if constexpr (JVP) {
          uL[c] = T(st[0][0 * NV + c], st[NS - 1][0 * NV + c]);
          uR[c] = T(st[0][1 * NV + c], st[NS - 1][1 * NV + c]);
#pragma unroll
          for (int j = 0; j < DIM; ++j) Ga[c][j] = T(st[0][(2 + j) * NV + c], st[NS - 1][(2 + j) * NV + c]);
          Ga[c][P] += (R)ph.eta * T(st[0][5 * NV + c], st[NS - 1][5 * NV + c]);
        } else {
          uL[c] = st[0][0 * NV + c];
          uR[c] = st[0][1 * NV + c];
#pragma unroll
          for (int j = 0; j < DIM; ++j) Ga[c][j] = st[0][(2 + j) * NV + c];
          Ga[c][P] += (R)ph.eta * st[0][5 * NV + c];
        }
      }
      T Hn[NV];
      num_flux<T, DIM>(uL, uR, P, ph, Hn);
      T ua[NV];
#pragma unroll
      for (int c = 0; c < NV; ++c) ua[c] = R(0.5) * (uL[c] + uR[c]);
      ViscPrep<T, DIM> vp;
      visc_prep<T, DIM>(ua, Ga, ph.gamma, vp);
      T Fv[NV];
      visc_flux_dir<T, DIM>(vp, P, ph.mu, kap, Fv);
#pragma unroll
      for (int c = 0; c < NV; ++c) H[((size_t)(P * NV + c) * NFQ + fq) * ne + ef] = out_part(Hn[c] - Fv[c]);
    }
  }
}

// The Jv tangent of the face's owner comes from V, that of its +P neighbour
// from Vr (V for the ordinary Jv; probing the diagonal blocks element by
// element passes zeros for one of the two).
template <class R, int NB, int NQ1, bool JVP, class MM, int OCC>
__global__ __launch_bounds__(256, OCC) void k_face_mfma(const double* __restrict__ U, const double* __restrict__ V,
                                                   const double* __restrict__ Vr, R* __restrict__ H,
                                                   MTablesT<R> mt, Mesh m, Phys ph) {
  __shared__ R stage[6 * 5][16][16];
  __shared__ R ttab[FaceTab<R, NB>::lds ? 6 * 2 * ((NB + 3) / 4) * 64 : 1];
  int64_t tile = 0;  // (the row form computes its tile in the body)
  int P = blockIdx.y;
  if constexpr (FaceTab<R, NB>::dir_fast) {
    const int64_t u = xcd_tile(blockIdx.x, gridDim.x);
    tile = u / 3;
    P = (int)(u % 3);
  }
  switch (P) {
    case 0: face_mfma_body<R, NB, NQ1, JVP, 0, MM>(U, V, Vr, H, mt, m, ph, stage, ttab, tile); break;
    case 1: face_mfma_body<R, NB, NQ1, JVP, 1, MM>(U, V, Vr, H, mt, m, ph, stage, ttab, tile); break;
    default: face_mfma_body<R, NB, NQ1, JVP, 2, MM>(U, V, Vr, H, mt, m, ph, stage, ttab, tile); break;
  }
}

// ------------------------------------------------------------------ dispatch
// (cfg id, nb, nq1d) of the 3D configurations with MFMA kernels; ids match
// the configuration table of dg_kernels.hip.
#define DG_MFMA_CONFIGS(X) \
  X(3, 10, 3, 3)           \
  X(4, 20, 4, 4)           \
  X(5, 35, 5, 5)

// occ: waves per SIMD of the launch bound, 0 for the configuration's default;
// a shape the configuration does not have returns hipErrorInvalidValue.
template <class R, class MM>
hipError_t face_mfma_dispatch(int cfg, bool jvp, const double* U, const double* V, R* H, const MTablesT<R>& mt,
                              const Mesh& m, const Phys& ph, int occ, hipStream_t s, const double* Vr) {
  if (!Vr) Vr = V;
#define X(id, nb_, nq_, kl_)                                                               \
  case id: {                                                                               \
    using FT = FaceTab<R, nb_>;                                                            \
    const int o = occ ? occ : FT::occupancy;                                               \
    const unsigned nt = (unsigned)((m.ne + 15) / 16);                                      \
    const dim3 grid = FT::dir_fast ? dim3(nt * 3) : dim3(nt, 3);                           \
    if (o == 1) {                                                                          \
      if (jvp)                                                                             \
        k_face_mfma<R, nb_, nq_, true, MM, 1><<<grid, 256, 0, s>>>(U, V, Vr, H, mt, m, ph);    \
      else                                                                                 \
        k_face_mfma<R, nb_, nq_, false, MM, 1><<<grid, 256, 0, s>>>(U, V, Vr, H, mt, m, ph);   \
    } else if (o == 2) {                                                                   \
      if constexpr (FT::only_default) {                                                    \
        return hipErrorInvalidValue;                                                       \
      } else {                                                                             \
        if (jvp)                                                                           \
          k_face_mfma<R, nb_, nq_, true, MM, 2><<<grid, 256, 0, s>>>(U, V, Vr, H, mt, m, ph);  \
        else                                                                               \
          k_face_mfma<R, nb_, nq_, false, MM, 2><<<grid, 256, 0, s>>>(U, V, Vr, H, mt, m, ph); \
      }                                                                                    \
    } else {                                                                               \
      return hipErrorInvalidValue;                                                         \
    }                                                                                      \
    return hipGetLastError();                                                              \
  }
  switch (cfg) { DG_MFMA_CONFIGS(X) }
#undef X
  return hipErrorInvalidValue;
}

template <class R, class MM, int OCC, bool FG>
hipError_t volume_launch(int nb, int nq, int kl, bool jvp, const double* U, const double* V, const double* Vn,
                         const R* Gm, const R* H, const R* Hm, double* out, double shift, const MTablesT<R>& mt,
                         const Mesh& m, const Phys& ph, hipStream_t s) {
  const dim3 grid((unsigned)((m.ne + 15) / 16));
#define X(id, nb_, nq_, kl_)                                                                                       \
  if (nb == nb_ && nq == nq_ && kl == kl_) {                                                                       \
    if (jvp)                                                                                                       \
      k_volume_mfma<R, nb_, nq_, kl_, true, MM, OCC, FG><<<grid, 256, 0, s>>>(U, V, Vn, Gm, H, Hm, out, shift, mt, m, ph);  \
    else                                                                                                           \
      k_volume_mfma<R, nb_, nq_, kl_, false, MM, OCC, FG><<<grid, 256, 0, s>>>(U, V, Vn, Gm, H, Hm, out, shift, mt, m, ph); \
    return hipGetLastError();                                                                                      \
  }
  DG_MFMA_CONFIGS(X)
#undef X
  return hipErrorInvalidValue;
}

// occ as for the face kernel; fused: form the corrected gradients in the
// volume kernel (Gm unused) instead of reading them.
template <class R, class MM>
hipError_t volume_mfma_dispatch(int cfg, bool jvp, const double* U, const double* V, const R* Gm, const R* H,
                                double* out, double shift, const MTablesT<R>& mt, const Mesh& m, const Phys& ph,
                                int occ, bool fused, hipStream_t s, const R* Hm, const double* Vn) {
  if (!Hm) Hm = H;
  if (!Vn) Vn = V;
  int nb = 0, nq = 0, kl = 0, o = 0;
#define X(id, nb_, nq_, kl_)                                 \
  if (cfg == id) {                                           \
    nb = nb_;                                                \
    nq = nq_;                                                \
    kl = kl_;                                                \
    o = occ ? occ : volume_occupancy<R, nb_>();              \
  }
  DG_MFMA_CONFIGS(X)
#undef X
  if (nb == 0 || mt.kl != kl) return hipErrorInvalidValue;
  if (o == 1)
    return fused ? volume_launch<R, MM, 1, true>(nb, nq, kl, jvp, U, V, Vn, Gm, H, Hm, out, shift, mt, m, ph, s)
                 : volume_launch<R, MM, 1, false>(nb, nq, kl, jvp, U, V, Vn, Gm, H, Hm, out, shift, mt, m, ph, s);
  if (o == 2)
    return fused ? volume_launch<R, MM, 2, true>(nb, nq, kl, jvp, U, V, Vn, Gm, H, Hm, out, shift, mt, m, ph, s)
                 : volume_launch<R, MM, 2, false>(nb, nq, kl, jvp, U, V, Vn, Gm, H, Hm, out, shift, mt, m, ph, s);
  return hipErrorInvalidValue;
}

template <class R, class MM>
hipError_t grad_mfma_dispatch(int cfg, bool jvp, const double* U, const double* V, R* Gm, const MTablesT<R>& mt,
                              const Mesh& m, hipStream_t s, const double* Vn) {
#define X(id, nb_, nq_, kl_)                                                                \
  case id: {                                                                                \
    dim3 grid((unsigned)((m.ne + 15) / 16), 3, jvp ? 2 : 1);                                \
    k_grad_mfma<R, nb_, MM><<<grid, 64, 0, s>>>(U, V, Vn ? Vn : V, Gm, mt.lA, m);               \
    return hipGetLastError();                                                               \
  }
  switch (cfg) { DG_MFMA_CONFIGS(X) }
#undef X
  return hipErrorInvalidValue;
}

}  // namespace dgk
