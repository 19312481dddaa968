// Element-wise block Jacobi (EWBJ, Sec. 2.3: LU factorisation of the
// diagonal blocks of the global operator G = shift*I + J).
//
// Setup: the diagonal block D_K = shift*I + dR_K/dU_K is probed column by
// column with the exact Jacobian-vector product, one colour class of
// elements at a time (no two elements of a class are face neighbours, so the
// product restricted to K only sees K's own perturbation).  Each block is then
// inverted in place by Gauss-Jordan elimination with partial (row) pivoting
// and stored explicitly (column-major with a padded column stride ld =
// block_ld(m), a multiple of 8 elements so every column starts on a 16-byte
// boundary: A[j*ld + i] = entry (i, j)), in FP64, FP32 or BF16 (FP32
// elimination rounded on store), so the apply is a batched matrix-vector
// product bound by HBM, read with 16-byte loads (FP32 accumulation for
// FP32/BF16).
#include "dg_internal.h"

namespace dgk {

#define DEVI __device__ __forceinline__

namespace {

__global__ void k_probe(double* __restrict__ P, const int* __restrict__ color, int col, int l, int nb, int nv,
                        int64_t ne) {
  const int64_t n = (int64_t)nv * nb * ne;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i % ne;
    const int r = (int)(i / ne);
    P[i] = (r == l && (col < 0 || color[e] == col)) ? 1.0 : 0.0;
  }
}

// D[e][l][r] = Jv[r*ne + e] for every element of colour `col`, every element
// if col < 0 (Jv already includes shift*P);
// block e starts at e*m*ld, column l at l*ld
__global__ void k_extract(const double* __restrict__ Jv, const int* __restrict__ color, int col, int l, int m,
                          int ld, int64_t ne, double* __restrict__ D) {
  const int64_t n = (int64_t)m * ne;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i % ne;
    const int r = (int)(i / ne);
    if (col < 0 || color[e] == col) D[((size_t)e * m + l) * ld + r] = Jv[i];
  }
}

// Storage conversions: FP64/FP32 pass through; BF16 = round-to-nearest-even
// of the FP32 value (upper 16 bits), kept as raw bits.
struct bf16_t {
  unsigned short bits;
};
__device__ __forceinline__ void store_as(double& o, double v) { o = v; }
__device__ __forceinline__ void store_as(float& o, float v) { o = v; }
__device__ __forceinline__ void store_as(bf16_t& o, float v) {
  unsigned int u = __float_as_uint(v);
  if ((u & 0x7f800000u) == 0x7f800000u) {  // Inf / NaN: truncate, keep NaN quiet
    o.bits = (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    return;
  }
  u += 0x7fffu + ((u >> 16) & 1u);
  o.bits = (unsigned short)(u >> 16);
}
__device__ __forceinline__ double load_as(const double& v) { return v; }
__device__ __forceinline__ float load_as(const float& v) { return v; }
__device__ __forceinline__ float load_as(const bf16_t& v) { return __uint_as_float(((unsigned int)v.bits) << 16); }

// Gauss-Jordan inversion with partial (row) pivoting, one m x m block per
// workgroup (m <= 256), thread i owning row i.  Columns j < nl of row i are
// at A[j*lda + i] in LDS, columns nl <= j < nl + NREG in the thread's
// registers rr.  Per
// pivot step: a wave-level max reduction of |A[i][k]| over i >= k (ties: the
// smallest row), the scaled pivot row and the old row k through LDS (double
// buffered, so two barriers per step), and a rank-1 update of each thread's
// own row.  The row interchanges are undone at the end as column
// interchanges within each row.
DEVI double fma_s(double a, double b, double c) { return fma(a, b, c); }
DEVI float fma_s(float a, float b, float c) { return fmaf(a, b, c); }

template <class S, int NREG>
DEVI S gj_get(const S* Ai, int lda, int nl, const S (&rr)[NREG > 0 ? NREG : 1], int j) {
  if (j < nl) return Ai[(size_t)j * lda];
  S v = S(0);
#pragma unroll
  for (int jj = 0; jj < NREG; ++jj) v = (jj == j - nl) ? rr[jj] : v;
  return v;
}
template <class S, int NREG>
DEVI void gj_set(S* Ai, int lda, int nl, S (&rr)[NREG > 0 ? NREG : 1], int j, S v) {
  if (j < nl) {
    Ai[(size_t)j * lda] = v;
    return;
  }
#pragma unroll
  for (int jj = 0; jj < NREG; ++jj) rr[jj] = (jj == j - nl) ? v : rr[jj];
}

template <class S, int NREG>
DEVI void gauss_jordan_rows(S* A, int m, int lda, int nl, S (&rr)[NREG > 0 ? NREG : 1], S (*rk2)[256],
                            S (*ro2)[256], double (*wv)[4], int (*wi)[4], S (*wp)[4], int* ipiv, int* bad) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool own = tid < m;
  S* Ai = A + tid;
  for (int k = 0; k < m; ++k) {
    const int par = k & 1;
    // pivot: max |A[i][k]| over i >= k (ties: the smallest i), with its value
    double best = -1.0;
    int bi = 0x7fffffff;
    S pv = S(0);
    if (own && tid >= k) {
      pv = gj_get<S, NREG>(Ai, lda, nl, rr, k);
      const double a = fabs((double)pv);
      best = (a != a) ? 1e308 : a;
      bi = tid;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      const S op = __shfl_xor(pv, off);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
        pv = op;
      }
    }
    if (lane == 0) {
      wv[par][wave] = best;
      wi[par][wave] = bi;
      wp[par][wave] = pv;
    }
    __syncthreads();
    best = wv[par][0];
    bi = wi[par][0];
    pv = wp[par][0];
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      const double ob = wv[par][w];
      const int oi = wi[par][w];
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
        pv = wp[par][w];
      }
    }
    const int piv = bi;
    if (tid == 0) {
      ipiv[k] = piv;
      if (!(pv != S(0) && (double)pv - (double)pv == 0.0)) *bad = 1;
    }
    const S pinv = (pv != S(0)) ? S(1) / pv : S(0);
    S* rk = rk2[par];
    S* ro = ro2[par];
    // Row interchange and scaled pivot row, one column per thread: rk = row
    // piv * pinv (entry k: pinv); row piv <- row k.  Register columns go
    // through rk / ro from the threads that own rows piv and k.
    if (tid < nl) {
      const S apv = A[(size_t)tid * lda + piv];
      const S ak = A[(size_t)tid * lda + k];
      rk[tid] = (tid == k) ? pinv : apv * pinv;
      A[(size_t)tid * lda + piv] = ak;
    }
    if (NREG > 0 && tid == piv) {
#pragma unroll
      for (int jj = 0; jj < NREG; ++jj) rk[nl + jj] = (nl + jj == k) ? pinv : rr[jj] * pinv;
    }
    if (NREG > 0 && tid == k) {
#pragma unroll
      for (int jj = 0; jj < NREG; ++jj) ro[nl + jj] = rr[jj];
    }
    __syncthreads();
    if (own) {
      if (NREG > 0 && tid == piv && piv != k) {
#pragma unroll
        for (int jj = 0; jj < NREG; ++jj) rr[jj] = ro[nl + jj];
      }
      // row k becomes the scaled pivot row (zero row, multiplier -1); every
      // other row i: A[i][j] -= A[i][k] rk[j], then A[i][k] = -A[i][k] pinv.
      // A multiplier rather than a select keeps the loads unconditional.
      const bool rowk = (tid == k);
      const S c = rowk ? S(-1) : gj_get<S, NREG>(Ai, lda, nl, rr, k);
      const S keep = rowk ? S(0) : S(1);
      int j = 0;
      for (; j + 8 <= nl; j += 8) {  // 8 loads issued before the 8 stores
        S a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = Ai[(size_t)(j + u) * lda];
#pragma unroll
        for (int u = 0; u < 8; ++u) Ai[(size_t)(j + u) * lda] = fma_s(-c, rk[j + u], a[u] * keep);
      }
      for (; j < nl; ++j) Ai[(size_t)j * lda] = fma_s(-c, rk[j], Ai[(size_t)j * lda] * keep);
#pragma unroll
      for (int jj = 0; jj < NREG; ++jj) rr[jj] = fma_s(-c, rk[nl + jj], rr[jj] * keep);
      gj_set<S, NREG>(Ai, lda, nl, rr, k, -c * rk[k]);
    }
  }
  __syncthreads();  // ipiv complete
  if (own)
    for (int k = m - 1; k >= 0; --k) {
      const int p = ipiv[k];
      if (p != k) {
        const S a = gj_get<S, NREG>(Ai, lda, nl, rr, k);
        const S b = gj_get<S, NREG>(Ai, lda, nl, rr, p);
        gj_set<S, NREG>(Ai, lda, nl, rr, k, b);
        gj_set<S, NREG>(Ai, lda, nl, rr, p, a);
      }
    }
}

// One block per workgroup.  Input blocks D (FP64, column stride ldd, block
// stride m*ldd); columns j < nl are copied to LDS as type S (stride m), the
// remaining m - nl <= NREG columns to registers, and the inverse is written to
// `out` (storage O, column stride ldo, block stride m*ldo, padding rows zero).
// Each thread reads and writes only its own row, so out may be D itself when
// ldo = ldd.
template <class S, class O, int NREG>
__global__ __launch_bounds__(256, 1) void k_invert(const double* __restrict__ D, int ldd, O* __restrict__ out,
                                                   int ldo, int m, int nl, int* __restrict__ info) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ S rk2[2][256], ro2[2][256];
  __shared__ double wv[2][4];
  __shared__ int wi[2][4], ipiv[256], bad;
  __shared__ S wp[2][4];
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  const double* Dg = D + (size_t)blockIdx.x * m * ldd;
  S* A = reinterpret_cast<S*>(smem);
  const int lda = m;
  if (tid < m)
    for (int j = 0; j < nl; ++j) A[(size_t)j * lda + tid] = (S)Dg[(size_t)j * ldd + tid];
  S rr[NREG > 0 ? NREG : 1];
#pragma unroll
  for (int jj = 0; jj < (NREG > 0 ? NREG : 1); ++jj)
    rr[jj] = (NREG > 0 && tid < m && nl + jj < m) ? (S)Dg[(size_t)(nl + jj) * ldd + tid] : S(0);
  __syncthreads();
  gauss_jordan_rows<S, NREG>(A, m, lda, nl, rr, rk2, ro2, wv, wi, wp, ipiv, &bad);
  O* Ob = out + (size_t)blockIdx.x * m * ldo;
  if (tid < ldo) {
    for (int j = 0; j < nl; ++j) store_as(Ob[(size_t)j * ldo + tid], tid < m ? A[(size_t)j * lda + tid] : S(0));
#pragma unroll
    for (int jj = 0; jj < NREG; ++jj)
      if (nl + jj < m) store_as(Ob[(size_t)(nl + jj) * ldo + tid], tid < m ? rr[jj] : S(0));
  }
  __syncthreads();
  if (tid == 0 && bad) info[0] = 1;
}

// z_K = Dinv_K r_K.  16-byte loads along the (padded) columns: T threads per
// element, a thread owns VEC consecutive rows of one column set (columns cs,
// cs + C, ..., C = T / (ld / VEC) column sets), the C column sets' partial
// sums are added in a fixed order; EPW elements per workgroup.  ACC is the
// accumulation type (FP64 for FP64 factors, FP32 for FP32/BF16).
template <class S> struct Vec16;
template <> struct Vec16<double> {
  static constexpr int n = 2;
  using T = double2;
  static DEVI void get(const T& v, double* o) { o[0] = v.x; o[1] = v.y; }
};
template <> struct Vec16<float> {
  static constexpr int n = 4;
  using T = float4;
  static DEVI void get(const T& v, float* o) { o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w; }
};
template <> struct Vec16<bf16_t> {
  static constexpr int n = 8;
  using T = uint4;
  static DEVI void get(const T& v, float* o) {
    const unsigned int w[4] = {v.x, v.y, v.z, v.w};
    for (int q = 0; q < 4; ++q) {
      o[2 * q] = __uint_as_float(w[q] << 16);
      o[2 * q + 1] = __uint_as_float(w[q] & 0xffff0000u);
    }
  }
};

template <class VT>
DEVI VT nt_load(const void* p) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  const u4 w = __builtin_nontemporal_load(reinterpret_cast<const u4*>(p));
  VT out;
  __builtin_memcpy(&out, &w, sizeof(out));
  return out;
}

template <class S, class ACC, int T, int EPW>
__global__ __launch_bounds__(T * EPW) void k_apply(const S* __restrict__ Dinv, int m, int ld, int64_t ne,
                                                   const double* __restrict__ r, double* __restrict__ z) {
  using V = Vec16<S>;
  constexpr int VEC = V::n;
  extern __shared__ __align__(16) unsigned char smem[];
  const int G = ld / VEC, C = T / G;
  const int sub = threadIdx.x / T, t = threadIdx.x - sub * T;
  const int64_t e = (int64_t)blockIdx.x * EPW + sub;
  const bool live = e < ne;
  double* rk = reinterpret_cast<double*>(smem) + (size_t)sub * (m + C * ld);  // [m]
  double* part = rk + m;                                                       // [C][ld]
  if (live)
    for (int j = t; j < m; j += T) rk[j] = r[(size_t)j * ne + e];
  __syncthreads();
  if (live && t < G * C) {
    const int rg = t % G, cs = t / G;
    ACC acc[VEC];
#pragma unroll
    for (int q = 0; q < VEC; ++q) acc[q] = 0;
    const S* A = Dinv + (size_t)e * m * ld + rg * VEC;
    for (int j = cs; j < m; j += C) {
      const typename V::T v = nt_load<typename V::T>(A + (size_t)j * ld);
      ACC x[VEC];
      V::get(v, x);
      const ACC rj = (ACC)rk[j];
#pragma unroll
      for (int q = 0; q < VEC; ++q) acc[q] += x[q] * rj;
    }
#pragma unroll
    for (int q = 0; q < VEC; ++q) part[cs * ld + rg * VEC + q] = (double)acc[q];
  }
  __syncthreads();
  if (live)
    for (int i = t; i < m; i += T) {
      double s = 0.0;
      for (int cs = 0; cs < C; ++cs) s += part[cs * ld + i];
      z[(size_t)i * ne + e] = s;
    }
}

// LDS of one register-resident inversion (buffers double buffered by step
// parity) and the per-thread context of a step.
template <class S>
struct GjShared {
  S prow[2][256];     // scaled pivot row (zero beyond the block's columns)
  S colk[2][256];     // multipliers A[i][k]
  double redv[2][16];  // per-wave pivot candidates: |value|, row, value
  int redi[2][16];
  S redp[2][16];
  int pivrow[256], kinv[256];
  int bad;
};
struct GjThread {
  int m, R, lane, wave, sl, i;
  bool own;
};

// Step k = sk * CW + KK (KK a compile-time column of the thread's registers).
template <class S, int CW, int KK>
DEVI void gj_regs_step(S (&a)[CW], bool& used, int sk, const GjThread& t, GjShared<S>& sh) {
  const int k = sk * CW + KK;
  if (k >= t.m) return;  // uniform
  const int par = k & 1;
  // pivot candidates: the threads of slice sk hold column k
  double best = -1.0;
  int bi = 0x7fffffff;
  S pv = S(0);
  if (t.sl == sk && t.own && !used) {
    pv = a[KK];
    const double v = fabs((double)pv);
    best = (v != v) ? 1e308 : v;
    bi = t.i;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off);
    const int oi = __shfl_xor(bi, off);
    const S op = __shfl_xor(pv, off);
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
      pv = op;
    }
  }
  if (t.lane == 0) {
    sh.redv[par][t.wave] = best;
    sh.redi[par][t.wave] = bi;
    sh.redp[par][t.wave] = pv;
  }
  __syncthreads();
  const int w0 = sk * t.R / 64;
  best = sh.redv[par][w0];
  bi = sh.redi[par][w0];
  pv = sh.redp[par][w0];
  for (int w = w0 + 1; w < w0 + t.R / 64; ++w) {
    const double ob = sh.redv[par][w];
    const int oi = sh.redi[par][w];
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
      pv = sh.redp[par][w];
    }
  }
  const int p = bi;
  const bool okp = pv != S(0) && (double)pv - (double)pv == 0.0;
  const S pinv = okp ? S(1) / pv : S(0);
  if (t.i == p) {  // columns >= m of the last slice hold zeros (a stays 0 there)
#pragma unroll
    for (int jj = 0; jj < CW; ++jj) sh.prow[par][t.sl * CW + jj] = (t.sl == sk && jj == KK) ? pinv : a[jj] * pinv;
  }
  if (t.sl == sk && t.own) sh.colk[par][t.i] = a[KK];
  if (threadIdx.x == 0) {
    sh.pivrow[k] = p < t.m ? p : 0;
    if (p < t.m) sh.kinv[p] = k;
    if (!okp) sh.bad = 1;
  }
  __syncthreads();
  if (t.own) {
    // row p becomes the scaled pivot row (multiplier -1, old value dropped);
    // every other row i: A[i][j] -= A[i][k] prow[j], and column k holds
    // -A[i][k] / A[p][k]
    // FP32: branch-free over the thread's columns (padding columns stay 0 =
    // fma(-c, 0, 0)), the pivot-row reads issued together.  FP64: one column
    // at a time behind its bounds test, which keeps the pivot-row values from
    // being hoisted next to the 35 register-resident doubles (measured at
    // P4: 43 ms against 76 ms with the hoisted reads spilling)
    const bool rowp = t.i == p;
    const S c = rowp ? S(-1) : sh.colk[par][t.i];
    const S* pr = &sh.prow[par][t.sl * CW];
#pragma unroll
    for (int jj = 0; jj < CW; ++jj) {
      const bool drop = rowp || (t.sl == sk && jj == KK);
      if constexpr (sizeof(S) == 8) {
        if (t.sl * CW + jj < t.m) a[jj] = fma_s(-c, pr[jj], drop ? S(0) : a[jj]);
      } else {
        a[jj] = fma_s(-c, pr[jj], drop ? S(0) : a[jj]);
      }
    }
    used = used || rowp;
  }
}

// The CW steps of one column slice, unrolled by template recursion (the
// loop unroller refuses bodies this large, and a runtime column index would
// move the register array to scratch).
template <class S, int CW, int KK>
struct GjSteps {
  static DEVI void run(S (&a)[CW], bool& used, int sk, const GjThread& t, GjShared<S>& sh) {
    gj_regs_step<S, CW, KK>(a, used, sk, t, sh);
    GjSteps<S, CW, KK + 1>::run(a, used, sk, t, sh);
  }
};
template <class S, int CW>
struct GjSteps<S, CW, CW> {
  static DEVI void run(S (&)[CW], bool&, int, const GjThread&, GjShared<S>&) {}
};

// Register-resident Gauss-Jordan for the larger blocks (64 < m <= 175): one
// block per workgroup of NS * R threads (R = m rounded up to 64, NS =
// ceil(m / CW) column slices), thread (s, i) holding row i's columns
// s*CW .. s*CW + CW - 1 in registers, so every step updates the whole block
// with CW fused multiply-adds per thread and LDS carries only the pivot row
// and the multipliers.  Partial pivoting without row interchanges: step k
// takes, among the rows not yet used as pivot rows, the one with the largest
// |A[i][k]| (ties: the smallest row index), p_k; row p_k is scaled by
// 1/A[p_k][k] and subtracted from every other row, and column k (which would
// become the unit vector e_{p_k}) stores the new column p_k of the
// accumulated inverse instead.  At the end the stored array S satisfies
// inv(A)[k][p_j] = S[p_k][j], which the write-out applies.  Two barriers per
// step.  D and out may be the same array (every load precedes every store).
// The inverse is stored as S, or (S = float, out_bf16) rounded to BF16.
template <class S, int CW>
__global__ __launch_bounds__(1024) void k_invert_regs(const double* D, int ldd, void* out, int out_bf16, int ldo,
                                                      int m, int* __restrict__ info) {
  __shared__ GjShared<S> sh;
  GjThread t;
  t.m = m;
  t.R = (m + 63) & ~63;
  const int NS = (m + CW - 1) / CW;
  const int tid = threadIdx.x;
  t.lane = tid & 63;
  t.wave = tid >> 6;
  t.sl = tid / t.R;
  t.i = tid - t.sl * t.R;
  t.own = t.i < m;
  const double* Dg = D + (size_t)blockIdx.x * m * ldd;
  S a[CW];
#pragma unroll
  for (int jj = 0; jj < CW; ++jj) {
    const int j = t.sl * CW + jj;
    a[jj] = (t.own && j < m) ? (S)Dg[(size_t)j * ldd + t.i] : S(0);
  }
  if (tid == 0) sh.bad = 0;
  if (tid < 256) sh.kinv[tid] = tid < m ? tid : 0;  // every row is a pivot row once; a safe start
  bool used = false;
  __syncthreads();  // every load of the block precedes every store (out may be D)
  for (int sk = 0; sk < NS; ++sk) GjSteps<S, CW, 0>::run(a, used, sk, t, sh);
  __syncthreads();  // pivrow / kinv complete
  const size_t ob = (size_t)blockIdx.x * m * ldo;
  auto put = [&](size_t idx, S v) {
    if constexpr (sizeof(S) == 4) {
      if (out_bf16) {
        store_as(static_cast<bf16_t*>(out)[ob + idx], v);
        return;
      }
    }
    static_cast<S*>(out)[ob + idx] = v;
  };
  if (t.own) {
    const int row = sh.kinv[t.i];
#pragma unroll
    for (int jj = 0; jj < CW; ++jj) {
      const int j = t.sl * CW + jj;
      if (j < m) put((size_t)sh.pivrow[j] * ldo + row, a[jj]);
    }
  } else if (t.i < ldo) {  // padding rows of this slice's columns
#pragma unroll
    for (int jj = 0; jj < CW; ++jj) {
      const int j = t.sl * CW + jj;
      if (j < m) put((size_t)j * ldo + t.i, S(0));
    }
  }
  if (tid == 0 && sh.bad) info[0] = 1;
}

// Small blocks (m <= 64): one wave per element (WPG per workgroup), lane i
// owns row i and walks the columns (column-major storage: consecutive lanes
// read consecutive entries); r_K sits in the wave's slice of LDS.
template <class S, class ACC, int WPG>
__global__ __launch_bounds__(64 * WPG) void k_apply_small(const S* __restrict__ Dinv, int m, int ld, int64_t ne,
                                                          const double* __restrict__ r, double* __restrict__ z) {
  __shared__ double rs[WPG][64];
  const int wv = threadIdx.x >> 6, i = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * WPG + wv;
  const bool live = e < ne && i < m;
  if (live) rs[wv][i] = r[(size_t)i * ne + e];
  __syncthreads();
  if (!live) return;
  const S* A = Dinv + (size_t)e * m * ld + i;
  ACC acc = 0;
#pragma unroll 8
  for (int j = 0; j < m; ++j) acc += (ACC)load_as(A[(size_t)j * ld]) * (ACC)rs[wv][j];
  z[(size_t)i * ne + e] = (double)acc;
}

unsigned grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (unsigned)g;
}

// ---------------------------------------------------------------- block ILU(0)
// Block ILU(0) of a level operator stored block-sparse (B[s][K], s = 0 the
// element's own block, s = 1..nf its face neighbours, column-major m x m),
// in the multicolour order of the face-neighbour graph: colours in order, and
// within a colour no two elements couple.  On a lattice no two neighbours of
// an element are neighbours of each other, so the only entries that the
// elimination changes inside the pattern are the diagonal blocks:
//   D'_K = D_K - sum_{J ~ K, colour(J) < colour(K)} A_KJ D'_J^{-1} A_JK,
// with A_KJ the sum of K's blocks that point to J (a face neighbour reached
// through two faces, or the element itself through a periodic face of a
// one-element direction, are summed; self couplings belong to D_K).
// One workgroup per element of colour q; D'_K^{-1} (FP64) is written to Dinv.
__global__ __launch_bounds__(256, 1) void k_ilu_factor(const double* __restrict__ B, const int64_t* __restrict__ nbr,
                                                       const int* __restrict__ color, int q, int nf, int m,
                                                       int64_t ne, double* __restrict__ Dinv, int* __restrict__ info) {
  const int64_t K = blockIdx.x;
  if (color[K] != q) return;  // uniform in the workgroup
  extern __shared__ __align__(16) unsigned char smem[];
  double* Dp = reinterpret_cast<double*>(smem);
  double* T1 = Dp + m * m;  // A_JK
  double* T2 = T1 + m * m;  // A_KJ
  double* X = T2 + m * m;   // D'_J^{-1} A_JK
  __shared__ double rk2[2][256], ro2[2][256];
  __shared__ double wv[2][4], wp[2][4];
  __shared__ int wi[2][4], ipiv[256], bad;
  const int tid = threadIdx.x;
  const int mm = m * m;
  if (tid == 0) bad = 0;
  for (int i = tid; i < mm; i += 256) {
    double v = B[(size_t)K * mm + i];
    for (int t = 1; t <= nf; ++t)
      if (nbr[(size_t)(t - 1) * ne + K] == K) v += B[((size_t)t * ne + K) * mm + i];
    Dp[i] = v;
  }
  for (int t = 1; t <= nf; ++t) {
    const int64_t J = nbr[(size_t)(t - 1) * ne + K];
    if (J == K || color[J] >= q) continue;
    bool dup = false;
    for (int t0 = 1; t0 < t; ++t0) dup = dup || nbr[(size_t)(t0 - 1) * ne + K] == J;
    if (dup) continue;
    __syncthreads();  // previous products done with T1, T2, X
    for (int i = tid; i < mm; i += 256) {
      double a = 0.0, b = 0.0;
      for (int u = 1; u <= nf; ++u) {
        if (nbr[(size_t)(u - 1) * ne + J] == K) a += B[((size_t)u * ne + J) * mm + i];
        if (nbr[(size_t)(u - 1) * ne + K] == J) b += B[((size_t)u * ne + K) * mm + i];
      }
      T1[i] = a;
      T2[i] = b;
    }
    __syncthreads();
    const double* DJ = Dinv + (size_t)J * mm;
    for (int i = tid; i < mm; i += 256) {  // X(r, c) = sum_k D'_J^{-1}(r, k) A_JK(k, c)
      const int r = i % m, cc = i / m;
      double s = 0.0;
      for (int k = 0; k < m; ++k) s = fma(DJ[(size_t)k * m + r], T1[cc * m + k], s);
      X[i] = s;
    }
    __syncthreads();
    for (int i = tid; i < mm; i += 256) {  // D' -= A_KJ X
      const int r = i % m, cc = i / m;
      double s = 0.0;
      for (int k = 0; k < m; ++k) s = fma(T2[k * m + r], X[cc * m + k], s);
      Dp[i] -= s;
    }
  }
  __syncthreads();
  double rr[1] = {0.0};
  gauss_jordan_rows<double, 0>(Dp, m, m, m, rr, rk2, ro2, wv, wi, wp, ipiv, &bad);
  __syncthreads();
  for (int i = tid; i < mm; i += 256) Dinv[(size_t)K * mm + i] = Dp[i];
  if (tid == 0 && bad) info[0] = 1;
}

// One sweep over the elements of colour q (one wave per element, thread =
// row).  Forward: z_K = D'_K^{-1} (r_K - sum_{earlier colours} A_K,t z_J);
// backward: z_K -= D'_K^{-1} sum_{later colours} A_K,t z_J.
__global__ __launch_bounds__(64) void k_ilu_sweep(const double* __restrict__ B, const int64_t* __restrict__ nbr,
                                                  const int* __restrict__ color, int q, int forward, int nf, int m,
                                                  int64_t ne, const double* __restrict__ Dinv,
                                                  const double* __restrict__ r, double* __restrict__ z) {
  const int64_t K = blockIdx.x;
  if (color[K] != q) return;
  __shared__ double y[64];
  const int row = threadIdx.x;
  const int mm = m * m;
  double acc = (forward && row < m) ? r[(size_t)row * ne + K] : 0.0;
  for (int t = 1; t <= nf; ++t) {
    const int64_t J = nbr[(size_t)(t - 1) * ne + K];
    if (J == K) continue;
    const int cj = color[J];
    if (forward ? cj >= q : cj <= q) continue;
    if (row < m) {
      const double* BK = B + ((size_t)t * ne + K) * mm;
      for (int j = 0; j < m; ++j) acc = fma(-BK[(size_t)j * m + row], z[(size_t)j * ne + J], acc);
    }
  }
  y[row] = acc;
  __syncthreads();
  if (row < m) {
    const double* DK = Dinv + (size_t)K * mm;
    double s = 0.0;
    for (int j = 0; j < m; ++j) s = fma(DK[(size_t)j * m + row], y[j], s);
    if (forward)
      z[(size_t)row * ne + K] = s;
    else
      z[(size_t)row * ne + K] += s;
  }
}

}  // namespace

hipError_t launch_probe_vector(double* P, const int* color, int col, int l, int nb, int nv, int64_t ne,
                               hipStream_t s) {
  k_probe<<<grid_for((int64_t)nv * nb * ne), 256, 0, s>>>(P, color, col, l, nb, nv, ne);
  return hipGetLastError();
}

hipError_t launch_extract_column(const double* Jv, const int* color, int col, int l, int m, int64_t ne,
                                 double /*shift*/, double* D, hipStream_t s) {
  k_extract<<<grid_for((int64_t)m * ne), 256, 0, s>>>(Jv, color, col, l, m, block_ld(m), ne, D);
  return hipGetLastError();
}

static constexpr size_t kMaxLds = 160 * 1024;

namespace {

// Column-slice width of the register-resident kernel for blocks of 65 to 175
// rows (0: the LDS kernel): 16 or 35, the smaller with ceil(m / CW) *
// roundup(m, 64) <= 1024 threads.
int regs_width(int m) {
  if (m <= 64 || m > 175) return 0;
  const int R = (m + 63) & ~63;
  for (int cw : {16, 35})
    if ((m + cw - 1) / cw * R <= 1024) return cw;
  return 0;
}

template <class S>
hipError_t invert_regs(double* D64, int ldd, void* out, int out_bf16, int ldo, int m, int64_t ne, int* info,
                       hipStream_t s) {
  const int cw = regs_width(m);
  const unsigned threads = (unsigned)((m + cw - 1) / cw * ((m + 63) & ~63));
  if (cw == 16)
    k_invert_regs<S, 16><<<(unsigned)ne, threads, 0, s>>>(D64, ldd, out, out_bf16, ldo, m, info);
  else if (cw == 35)
    k_invert_regs<S, 35><<<(unsigned)ne, threads, 0, s>>>(D64, ldd, out, out_bf16, ldo, m, info);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_block_invert(int storage, double* D64, int ldd, void* Dout, int m, int64_t ne, int* info,
                              hipStream_t s) {
  if (m < 1 || m > 256) return hipErrorInvalidValue;
  const int ldo = block_ld(m);
  if (regs_width(m) > 0) {  // register-resident Gauss-Jordan
    if (storage == DG_FP64) return invert_regs<double>(D64, ldd, Dout, 0, ldo, m, ne, info, s);
    if (storage == DG_FP32) return invert_regs<float>(D64, ldd, Dout, 0, ldo, m, ne, info, s);
    if (storage == DG_BF16) return invert_regs<float>(D64, ldd, Dout, 1, ldo, m, ne, info, s);
    return hipErrorInvalidValue;
  }
  constexpr int kRegCols = 72;  // FP64 columns kept in registers when the block does not fit LDS
  // static LDS: pivot rows (2 x 2 x 256 entries), reductions, pivots
  auto fixed = [](size_t es) { return (4 * 256 + 8) * es + 2 * 4 * (sizeof(double) + sizeof(int)) + 257 * sizeof(int) + 64; };
  if (storage == DG_FP64) {
    double* O = static_cast<double*>(Dout);
    const size_t all = (size_t)m * m * sizeof(double);
    if (all + fixed(8) <= kMaxLds) {
      hipFuncSetAttribute((const void*)k_invert<double, double, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)all);
      k_invert<double, double, 0><<<(unsigned)ne, 256, all, s>>>(D64, ldd, O, ldo, m, m, info);
    } else if (m > kRegCols && (size_t)(m - kRegCols) * m * sizeof(double) + fixed(8) <= kMaxLds) {
      const size_t part = (size_t)(m - kRegCols) * m * sizeof(double);
      hipFuncSetAttribute((const void*)k_invert<double, double, kRegCols>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)part);
      k_invert<double, double, kRegCols><<<(unsigned)ne, 256, part, s>>>(D64, ldd, O, ldo, m, m - kRegCols, info);
    } else {
      return hipErrorInvalidValue;  // FP64 blocks above m = 189 do not fit LDS + registers
    }
    return hipGetLastError();
  }
  if (storage == DG_FP32 || storage == DG_BF16) {
    // FP32 Gauss-Jordan in LDS; BF16 storage rounds the FP32 inverse
    const size_t all = (size_t)m * m * sizeof(float);
    if (all + fixed(4) > kMaxLds) return hipErrorInvalidValue;
    if (storage == DG_FP32) {
      hipFuncSetAttribute((const void*)k_invert<float, float, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)all);
      k_invert<float, float, 0><<<(unsigned)ne, 256, all, s>>>(D64, ldd, static_cast<float*>(Dout), ldo, m, m, info);
    } else {
      hipFuncSetAttribute((const void*)k_invert<float, bf16_t, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)all);
      k_invert<float, bf16_t, 0><<<(unsigned)ne, 256, all, s>>>(D64, ldd, static_cast<bf16_t*>(Dout), ldo, m, m, info);
    }
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

hipError_t launch_ilu_factor(const double* B, const int64_t* nbr, const int* color, int ncolor, int nf, int m,
                             int64_t ne, double* Dinv, int* info, hipStream_t s) {
  if (m < 1 || m > 64 || ncolor < 1 || ne < 1) return hipErrorInvalidValue;
  const size_t lds = (size_t)4 * m * m * sizeof(double);
  hipFuncSetAttribute((const void*)k_ilu_factor, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  for (int q = 0; q < ncolor; ++q)
    k_ilu_factor<<<(unsigned)ne, 256, lds, s>>>(B, nbr, color, q, nf, m, ne, Dinv, info);
  return hipGetLastError();
}

hipError_t launch_ilu_apply(const double* B, const int64_t* nbr, const int* color, int ncolor, int nf, int m,
                            int64_t ne, const double* Dinv, const double* r, double* z, hipStream_t s) {
  if (m < 1 || m > 64 || ncolor < 1 || ne < 1 || r == z) return hipErrorInvalidValue;
  for (int q = 0; q < ncolor; ++q)
    k_ilu_sweep<<<(unsigned)ne, 64, 0, s>>>(B, nbr, color, q, 1, nf, m, ne, Dinv, r, z);
  for (int q = ncolor - 1; q >= 0; --q)
    k_ilu_sweep<<<(unsigned)ne, 64, 0, s>>>(B, nbr, color, q, 0, nf, m, ne, Dinv, r, z);
  return hipGetLastError();
}

namespace {

template <class S, class ACC, int WPG>
hipError_t apply_small(const void* Dinv, int m, int64_t ne, const double* r, double* z, hipStream_t s) {
  const unsigned grid = (unsigned)((ne + WPG - 1) / WPG);
  k_apply_small<S, ACC, WPG><<<grid, 64 * WPG, 0, s>>>(static_cast<const S*>(Dinv), m, block_ld(m), ne, r, z);
  return hipGetLastError();
}

template <class S, class ACC, int T, int EPW>
hipError_t apply_vec(const void* Dinv, int m, int64_t ne, const double* r, double* z, hipStream_t s) {
  const int ld = block_ld(m), G = ld / Vec16<S>::n;
  const size_t lds = (size_t)EPW * (m + (T / G) * ld) * sizeof(double);
  const unsigned grid = (unsigned)((ne + EPW - 1) / EPW);
  k_apply<S, ACC, T, EPW><<<grid, T * EPW, lds, s>>>(static_cast<const S*>(Dinv), m, ld, ne, r, z);
  return hipGetLastError();
}

template <class S, class ACC>
hipError_t apply_shape(const ApplyShape& sh, const void* Dinv, int m, int64_t ne, const double* r, double* z,
                       hipStream_t s) {
  if (sh.kind == kApplyRow) {
    switch (sh.epw) {
      case 1: return apply_small<S, ACC, 1>(Dinv, m, ne, r, z, s);
      case 2: return apply_small<S, ACC, 2>(Dinv, m, ne, r, z, s);
      case 4: return apply_small<S, ACC, 4>(Dinv, m, ne, r, z, s);
      case 8: return apply_small<S, ACC, 8>(Dinv, m, ne, r, z, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (sh.kind != kApplyVec) return hipErrorInvalidValue;
  if (sh.threads == 64) {
    switch (sh.epw) {
      case 1: return apply_vec<S, ACC, 64, 1>(Dinv, m, ne, r, z, s);
      case 2: return apply_vec<S, ACC, 64, 2>(Dinv, m, ne, r, z, s);
      case 4: return apply_vec<S, ACC, 64, 4>(Dinv, m, ne, r, z, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (sh.epw != 1) return hipErrorInvalidValue;
  switch (sh.threads) {
    case 128: return apply_vec<S, ACC, 128, 1>(Dinv, m, ne, r, z, s);
    case 256: return apply_vec<S, ACC, 256, 1>(Dinv, m, ne, r, z, s);
    case 512: return apply_vec<S, ACC, 512, 1>(Dinv, m, ne, r, z, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool apply_shape_fits(const ApplyShape& sh, int m, int storage) {
  if (m < 1 || m > 256 || (storage != DG_FP64 && storage != DG_FP32 && storage != DG_BF16)) return false;
  if (sh.kind == kApplyDefault) return true;
  const bool e1248 = sh.epw == 1 || sh.epw == 2 || sh.epw == 4 || sh.epw == 8;
  if (sh.kind == kApplyRow) return m <= 64 && sh.threads == 64 && e1248;
  if (sh.kind != kApplyVec) return false;
  if (sh.threads == 64) {
    if (sh.epw != 1 && sh.epw != 2 && sh.epw != 4) return false;
  } else if (sh.threads == 128 || sh.threads == 256 || sh.threads == 512) {
    if (sh.epw != 1) return false;
  } else {
    return false;
  }
  const int vec = storage == DG_FP64 ? 2 : (storage == DG_FP32 ? 4 : 8);
  const int ld = block_ld(m), G = ld / vec;
  if (G > sh.threads) return false;  // every thread group needs one column set at least
  return (size_t)sh.epw * (m + (sh.threads / G) * ld) * sizeof(double) <= 65536;
}

ApplyShape default_apply_shape(int m) {
  ApplyShape sh;
  if (m <= 64) {
    sh.kind = kApplyRow;
    sh.threads = 64;
    sh.epw = 4;
  } else {
    sh.kind = kApplyVec;
    sh.threads = 256;
    sh.epw = 1;
  }
  return sh;
}

hipError_t launch_block_apply(int storage, const void* Dinv, int m, int64_t ne, const double* r, double* z,
                              hipStream_t s, const ApplyShape* shape) {
  const ApplyShape sh = (shape && shape->kind) ? *shape : default_apply_shape(m);
  if (!apply_shape_fits(sh, m, storage)) return hipErrorInvalidValue;
  if (storage == DG_FP64) return apply_shape<double, double>(sh, Dinv, m, ne, r, z, s);
  if (storage == DG_FP32) return apply_shape<float, float>(sh, Dinv, m, ne, r, z, s);
  if (storage == DG_BF16) return apply_shape<bf16_t, float>(sh, Dinv, m, ne, r, z, s);
  return hipErrorInvalidValue;
}

}  // namespace dgk
