// FP64 vector kernels for the Krylov solver (Arnoldi with classical
// Gram-Schmidt and one re-orthogonalisation, Sec. 2.5) and the
// finite-difference Jacobian-vector product of eqs. (matrix-free)/(epsdef).
// Reductions are deterministic: every block writes one partial per output,
// a second one-block kernel sums the partials in a fixed order.
#include "dg_internal.h"

namespace dgk {

namespace {

// Sum over a 256-thread workgroup: wave shuffles, then the four wave sums
// through LDS (sh needs 4 entries); every thread gets the result.
__device__ __forceinline__ double block_sum256(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_dot_partials(const double* __restrict__ x, const double* __restrict__ y,
                                                       int64_t n, double* __restrict__ partial) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) a += x[i] * y[i];
  a = block_sum256(a, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = a;
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partial, int np,
                                                       double* __restrict__ out, int sqrt_flag) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) a += partial[i];
  a = block_sum256(a, sh);
  if (threadIdx.x == 0) out[0] = sqrt_flag ? sqrt(a) : a;
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                        double* __restrict__ z) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    z[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

// z = x + (dscale[0] * c) * y
__global__ void k_axpy_dev(int64_t n, const double* __restrict__ x, const double* __restrict__ dscale, double c,
                           const double* __restrict__ y, double* __restrict__ z) {
  const double s = dscale[0] * c;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    z[i] = x[i] + s * y[i];
}

// out = shift*v + (rp - r0) * dinv[0]
__global__ void k_fd_combine(int64_t n, int64_t nm, const double* __restrict__ rp, const double* __restrict__ r0,
                             const double* __restrict__ dinv, const double* __restrict__ v, double shift,
                             double* __restrict__ out) {
  const double s = dinv[0];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (i < nm ? shift * v[i] : 0.0) + (s == 0.0 ? 0.0 : (rp[i] - r0[i]) * s);
}

// y = x / dnorm[0] (0 if the norm is 0)
__global__ void k_scale_dev(int64_t n, const double* __restrict__ x, const double* __restrict__ dnorm,
                            double* __restrict__ y) {
  const double nr = dnorm[0];
  const double s = nr > 0.0 ? 1.0 / nr : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i] * s;
}

constexpr int kMaxK = 64;

// partial[j][blk] = sum over the block's range of V_j[i] * w[i], j < k
// Partial dot products of w with V_j0 .. V_j0+G-1 per pass: every w value is
// read once per G basis vectors; VEC loads two consecutive entries at a time
// (n even).  The per-block sums go through wave shuffles and one LDS step.
template <int G, bool VEC>
__global__ __launch_bounds__(256) void k_mdot(const double* __restrict__ V, int k, int64_t n,
                                               const double* __restrict__ w, double* __restrict__ partial) {
  __shared__ double sh[4][G];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int j0 = 0; j0 < k; j0 += G) {
    double a[G];
#pragma unroll
    for (int jj = 0; jj < G; ++jj) a[jj] = 0.0;
    const int jn = min(G, k - j0);
    if constexpr (VEC) {
      const int64_t n2 = n / 2;
      const double2* w2 = reinterpret_cast<const double2*>(w);
      for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n2; i += stride) {
        const double2 wi = w2[i];
#pragma unroll
        for (int jj = 0; jj < G; ++jj)
          if (jj < jn) {
            const double2 v = reinterpret_cast<const double2*>(V + (size_t)(j0 + jj) * n)[i];
            a[jj] += v.x * wi.x + v.y * wi.y;
          }
      }
    } else {
      for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const double wi = w[i];
#pragma unroll
        for (int jj = 0; jj < G; ++jj)
          if (jj < jn) a[jj] += V[(size_t)(j0 + jj) * n + i] * wi;
      }
    }
#pragma unroll
    for (int jj = 0; jj < G; ++jj) {
      double v = a[jj];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      a[jj] = v;
    }
    if (lane == 0)
#pragma unroll
      for (int jj = 0; jj < G; ++jj) sh[wv][jj] = a[jj];
    __syncthreads();
    if ((int)threadIdx.x < jn) {
      const int t = threadIdx.x;
      partial[(size_t)(j0 + t) * gridDim.x + blockIdx.x] = (sh[0][t] + sh[1][t]) + (sh[2][t] + sh[3][t]);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_msum(const double* __restrict__ partial, int np, double* __restrict__ h) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) a += partial[(size_t)blockIdx.x * np + i];
  a = block_sum256(a, sh);
  if (threadIdx.x == 0) h[blockIdx.x] = a;
}

// w -= sum_j h[j] V_j   (sign = -1)  or  x += sum_j h[j] V_j (sign = +1)
__global__ __launch_bounds__(256) void k_mupdate(const double* __restrict__ V, int k, int64_t n,
                                                  const double* __restrict__ h, double* __restrict__ w, double sign) {
  __shared__ double hs[kMaxK];
  if ((int)threadIdx.x < k) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double a = 0.0;
    for (int j = 0; j < k; ++j) a += hs[j] * V[(size_t)j * n + i];
    w[i] += sign * a;
  }
}

__global__ void k_fill(double* __restrict__ x, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

__global__ void k_nonfinite(const double* __restrict__ x, int64_t n, int* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = x[i];
    bad |= !(v - v == 0.0);
  }
  if (bad) flag[0] = 1;  // benign race: every writer stores 1
}

// d[2] = eps*sqrt(1 + ||w||)/||v|| and d[3] = 1/d[2] from d[0] = ||w||, d[1] = ||v||
// (eq. epsdef); both 0 when ||v|| = 0.
__global__ void k_fd_delta(double* d, double eps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double nw = d[0], nv = d[1];
    const double delta = nv > 0.0 ? eps * sqrt(1.0 + nw) / nv : 0.0;
    d[2] = delta;
    d[3] = delta > 0.0 ? 1.0 / delta : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_max_partials(const double* __restrict__ partial, int np,
                                                       double* __restrict__ out) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) {
    const double v = partial[i];
    a = (v > a || v != v) ? v : a;
  }
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double o = sh[threadIdx.x + s];
      sh[threadIdx.x] = (o > sh[threadIdx.x] || o != o) ? o : sh[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

unsigned grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_dot_partials(const double* x, const double* y, int64_t n, double* partial, hipStream_t s) {
  k_dot_partials<<<kRedBlocks, 256, 0, s>>>(x, y, n, partial);
  return hipGetLastError();
}
hipError_t launch_sum_partials(const double* partial, int np, double* out, int sqrt_flag, hipStream_t s) {
  k_sum_partials<<<1, 256, 0, s>>>(partial, np, out, sqrt_flag);
  return hipGetLastError();
}
hipError_t launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* z, hipStream_t s) {
  k_axpby<<<grid_for(n), 256, 0, s>>>(n, a, x, b, y, z);
  return hipGetLastError();
}
hipError_t launch_axpy_dev(int64_t n, const double* x, const double* dscale, double c, const double* y, double* z,
                           hipStream_t s) {
  k_axpy_dev<<<grid_for(n), 256, 0, s>>>(n, x, dscale, c, y, z);
  return hipGetLastError();
}
hipError_t launch_fd_combine(int64_t n, int64_t nm, const double* rp, const double* r0, const double* dinv,
                             const double* v, double shift, double* out, hipStream_t s) {
  k_fd_combine<<<grid_for(n), 256, 0, s>>>(n, nm, rp, r0, dinv, v, shift, out);
  return hipGetLastError();
}
hipError_t launch_scale_dev(int64_t n, const double* x, const double* dnorm, double* y, hipStream_t s) {
  k_scale_dev<<<grid_for(n), 256, 0, s>>>(n, x, dnorm, y);
  return hipGetLastError();
}
hipError_t launch_mdot(const double* V, int k, int64_t n, const double* w, double* partial, hipStream_t s) {
  if (k > kMaxK) return hipErrorInvalidValue;
  if (n % 2 == 0)
    k_mdot<16, true><<<kRedBlocks, 256, 0, s>>>(V, k, n, w, partial);
  else
    k_mdot<16, false><<<kRedBlocks, 256, 0, s>>>(V, k, n, w, partial);
  return hipGetLastError();
}
hipError_t launch_msum(const double* partial, int k, double* h, hipStream_t s) {
  k_msum<<<k, 256, 0, s>>>(partial, kRedBlocks, h);
  return hipGetLastError();
}
hipError_t launch_mupdate(const double* V, int k, int64_t n, const double* h, double* w, hipStream_t s) {
  if (k > kMaxK) return hipErrorInvalidValue;
  k_mupdate<<<grid_for(n), 256, 0, s>>>(V, k, n, h, w, -1.0);
  return hipGetLastError();
}
hipError_t launch_mupdate_add(const double* Z, int k, int64_t n, const double* y, double* x, hipStream_t s) {
  if (k > kMaxK) return hipErrorInvalidValue;
  k_mupdate<<<grid_for(n), 256, 0, s>>>(Z, k, n, y, x, 1.0);
  return hipGetLastError();
}
hipError_t launch_fd_delta(double* d, double eps, hipStream_t s) {
  k_fd_delta<<<1, 64, 0, s>>>(d, eps);
  return hipGetLastError();
}
hipError_t launch_max_partials(const double* partial, int np, double* out, hipStream_t s) {
  k_max_partials<<<1, 256, 0, s>>>(partial, np, out);
  return hipGetLastError();
}
hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s) {
  k_fill<<<grid_for(n), 256, 0, s>>>(x, n, v);
  return hipGetLastError();
}
hipError_t launch_nonfinite_check(const double* x, int64_t n, int* flag, hipStream_t s) {
  k_nonfinite<<<grid_for(n), 256, 0, s>>>(x, n, flag);
  return hipGetLastError();
}

}  // namespace dgk
