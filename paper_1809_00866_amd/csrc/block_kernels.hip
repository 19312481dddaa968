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
    P[i] = (r == l && color[e] == col) ? 1.0 : 0.0;
  }
}

// D[e][l][r] = Jv[r*ne + e] for every element of colour `col` (Jv already includes shift*P);
// block e starts at e*m*ld, column l at l*ld
__global__ void k_extract(const double* __restrict__ Jv, const int* __restrict__ color, int col, int l, int m,
                          int ld, int64_t ne, double* __restrict__ D) {
  const int64_t n = (int64_t)m * ne;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i % ne;
    const int r = (int)(i / ne);
    if (color[e] == col) D[((size_t)e * m + l) * ld + r] = Jv[i];
  }
}

// In-place Gauss-Jordan inversion with row pivoting of one m x m column-major
// block per workgroup.  S is the arithmetic/storage type of the working copy
// A (LDS when it fits, else the block's own global storage).
template <class S>
__device__ void gauss_jordan(S* A, int m, int lda, S* colk, S* rowk, int* ipiv, double* rv, int* ri, int* bad) {
  const int tid = threadIdx.x;
  for (int k = 0; k < m; ++k) {
    // pivot: max |A[i][k]|, i >= k; ties keep the smallest row index
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < m; i += 256) {
      const double a = fabs((double)A[(size_t)k * lda + i]);
      if (a > best || (a != a)) {
        best = (a != a) ? 1e308 : a;
        bi = i;
      }
    }
    rv[tid] = best;
    ri[tid] = bi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) {
        const double o = rv[tid + s];
        const int oi = ri[tid + s];
        if (o > rv[tid] || (o == rv[tid] && oi < ri[tid])) {
          rv[tid] = o;
          ri[tid] = oi;
        }
      }
      __syncthreads();
    }
    const int piv = ri[0];
    if (tid == 0) ipiv[k] = piv;
    // swap rows k and piv
    if (piv != k)
      for (int j = tid; j < m; j += 256) {
        const S t = A[(size_t)j * lda + k];
        A[(size_t)j * lda + k] = A[(size_t)j * lda + piv];
        A[(size_t)j * lda + piv] = t;
      }
    __syncthreads();
    const S pv = A[(size_t)k * lda + k];
    if (tid == 0 && !(pv != (S)0 && (double)pv - (double)pv == 0.0)) *bad = 1;
    const S pinv = (pv != (S)0) ? (S)1 / pv : (S)0;
    // scaled pivot row (entry k becomes pinv) and the old column k
    for (int j = tid; j < m; j += 256) rowk[j] = (j == k) ? pinv : A[(size_t)j * lda + k] * pinv;
    for (int i = tid; i < m; i += 256) colk[i] = A[(size_t)k * lda + i];
    __syncthreads();
    for (size_t idx = tid; idx < (size_t)m * m; idx += 256) {
      const int i = (int)(idx % m), j = (int)(idx / m);
      S* a = &A[(size_t)j * lda + i];
      if (i == k) {
        *a = rowk[j];
      } else {
        const S base = (j == k) ? (S)0 : *a;
        *a = base - colk[i] * rowk[j];
      }
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last first
  for (int k = m - 1; k >= 0; --k) {
    const int p = ipiv[k];
    if (p != k)
      for (int i = tid; i < m; i += 256) {
        const S t = A[(size_t)k * lda + i];
        A[(size_t)k * lda + i] = A[(size_t)p * lda + i];
        A[(size_t)p * lda + i] = t;
      }
    __syncthreads();
  }
}

// FP64 working copy in global memory (in place, column stride ld).
__global__ __launch_bounds__(256) void k_invert_global64(double* __restrict__ D, int m, int ld,
                                                         int* __restrict__ info) {
  __shared__ double colk[256], rowk[256], rv[256];
  __shared__ int ipiv[256], ri[256], bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  double* A = D + (size_t)blockIdx.x * m * ld;
  gauss_jordan<double>(A, m, ld, colk, rowk, ipiv, rv, ri, &bad);
  if (threadIdx.x == 0 && bad) info[0] = 1;
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

// LDS working copy of type S (compact, stride m); input blocks of column
// stride ldd, result written to `out` (storage type O, column stride ldo,
// padding rows zero).
template <class S, class O = S>
__global__ __launch_bounds__(256) void k_invert_lds(const double* __restrict__ D, int ldd, O* __restrict__ out,
                                                    int ldo, int m, int* __restrict__ info) {
  extern __shared__ __align__(16) unsigned char smem[];
  S* A = reinterpret_cast<S*>(smem);
  __shared__ S colk[256], rowk[256];
  __shared__ double rv[256];
  __shared__ int ipiv[256], ri[256], bad;
  if (threadIdx.x == 0) bad = 0;
  const double* Dg = D + (size_t)blockIdx.x * m * ldd;
  for (size_t i = threadIdx.x; i < (size_t)m * m; i += 256) A[i] = (S)Dg[(i / m) * ldd + i % m];
  __syncthreads();
  gauss_jordan<S>(A, m, m, colk, rowk, ipiv, rv, ri, &bad);
  O* Ob = out + (size_t)blockIdx.x * m * ldo;
  for (size_t i = threadIdx.x; i < (size_t)m * ldo; i += 256) {
    const int r = (int)(i % ldo), j = (int)(i / ldo);
    store_as(Ob[i], r < m ? A[(size_t)j * m + r] : S(0));
  }
  if (threadIdx.x == 0 && bad) info[0] = 1;
}

// z_K = Dinv_K r_K.  16-byte loads along the (padded) columns: a thread owns
// VEC consecutive rows of one column set (columns cs, cs + C, ...), the C
// column sets' partial sums are added in a fixed order.  ACC is the
// accumulation type (FP64 for FP64 factors, FP32 for FP32/BF16).
constexpr int kApplyThreads = 256;
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

template <class S, class ACC>
__global__ __launch_bounds__(kApplyThreads) void k_apply(const S* __restrict__ Dinv, int m, int ld, int64_t ne,
                                                         const double* __restrict__ r, double* __restrict__ z) {
  using V = Vec16<S>;
  constexpr int VEC = V::n;
  extern __shared__ __align__(16) unsigned char smem[];
  double* rk = reinterpret_cast<double*>(smem);  // [m]
  double* part = rk + m;                         // [C][ld]
  const int G = ld / VEC, C = kApplyThreads / G;
  const int64_t e = blockIdx.x;
  for (int j = threadIdx.x; j < m; j += kApplyThreads) rk[j] = r[(size_t)j * ne + e];
  __syncthreads();
  const int t = threadIdx.x;
  if (t < G * C) {
    const int rg = t % G, cs = t / G;
    ACC acc[VEC];
#pragma unroll
    for (int q = 0; q < VEC; ++q) acc[q] = 0;
    const S* A = Dinv + (size_t)e * m * ld + rg * VEC;
    for (int j = cs; j < m; j += C) {
      const typename V::T v = *reinterpret_cast<const typename V::T*>(A + (size_t)j * ld);
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
  for (int i = threadIdx.x; i < m; i += kApplyThreads) {
    double s = 0.0;
    for (int cs = 0; cs < C; ++cs) s += part[cs * ld + i];
    z[(size_t)i * ne + e] = s;
  }
}

unsigned grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (unsigned)g;
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

hipError_t launch_block_invert(int storage, double* D64, int ldd, void* Dout, int m, int64_t ne, int* info,
                              hipStream_t s) {
  if (m > 256) return hipErrorInvalidValue;
  const int ldo = block_ld(m);
  // static LDS of the kernels: pivot row/column, reduction scratch
  const size_t static_lds = 2 * 256 * sizeof(double) + 256 * sizeof(double) + 2 * 256 * sizeof(int) + 64;
  if (storage == DG_FP64) {
    const size_t need = (size_t)m * m * sizeof(double);
    if (need + static_lds <= kMaxLds) {
      hipFuncSetAttribute((const void*)k_invert_lds<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
      k_invert_lds<double><<<(unsigned)ne, 256, need, s>>>(D64, ldd, static_cast<double*>(Dout), ldo, m, info);
    } else {
      if (Dout != D64 || ldd != ldo) return hipErrorInvalidValue;
      k_invert_global64<<<(unsigned)ne, 256, 0, s>>>(D64, m, ldd, info);
    }
    return hipGetLastError();
  }
  if (storage == DG_FP32 || storage == DG_BF16) {
    // FP32 Gauss-Jordan in LDS; BF16 storage rounds the FP32 inverse
    const size_t need = (size_t)m * m * sizeof(float);
    if (need + static_lds > kMaxLds) return hipErrorInvalidValue;
    if (storage == DG_FP32) {
      hipFuncSetAttribute((const void*)k_invert_lds<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need);
      k_invert_lds<float><<<(unsigned)ne, 256, need, s>>>(D64, ldd, static_cast<float*>(Dout), ldo, m, info);
    } else {
      hipFuncSetAttribute((const void*)k_invert_lds<float, bf16_t>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)need);
      k_invert_lds<float, bf16_t><<<(unsigned)ne, 256, need, s>>>(D64, ldd, static_cast<bf16_t*>(Dout), ldo, m, info);
    }
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

hipError_t launch_block_apply(int storage, const void* Dinv, int m, int64_t ne, const double* r, double* z,
                              hipStream_t s) {
  if (m < 1 || m > 256) return hipErrorInvalidValue;
  const int ld = block_ld(m);
  constexpr int T = kApplyThreads;
  auto lds = [&](int vec) { return (size_t)(m + (T / (ld / vec)) * ld) * sizeof(double); };
  if (storage == DG_FP64)
    k_apply<double, double><<<(unsigned)ne, T, lds(2), s>>>(static_cast<const double*>(Dinv), m, ld, ne, r, z);
  else if (storage == DG_FP32)
    k_apply<float, float><<<(unsigned)ne, T, lds(4), s>>>(static_cast<const float*>(Dinv), m, ld, ne, r, z);
  else if (storage == DG_BF16)
    k_apply<bf16_t, float><<<(unsigned)ne, T, lds(8), s>>>(static_cast<const bf16_t*>(Dinv), m, ld, ne, r, z);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace dgk
