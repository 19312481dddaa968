// Learned element-local preconditioner: feature assembly, BF16 MFMA GEMMs
// with FP32 accumulation and fused epilogues, loss, bias gradients, Adam.
//
// The flexible outer solver (Sec. 2.5) tolerates a preconditioner that
// changes between applications; the network maps the normalised residual of
// an element and the mean states of its face neighbours to the normalised
// correction of that element (z_K = s_K * MLP(x_K), s_K = ||r_K|| + 1e-300).
//
// MFMA BF16 16x16x32 lane layout (gfx950, checked with an in-bounds probe):
// lane l supplies A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16],
// j = 0..7, and receives D[4 (l / 16) + r][l % 16], r = 0..3.
#include "dg_internal.h"

namespace dgk {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float v) {
  unsigned int u = __float_as_uint(v);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

unsigned grid_for(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

// mref[c] = sqrt(sum_K mean_c(K)^2 / ne) from ss[c] = sum_K U[c,0,K]^2 (mean = U_c0 / sqrt|K|)
__global__ void k_mlp_mref(const double* __restrict__ ss, int nv, int64_t ne, double inv_vol, double* __restrict__ mref) {
  const int c = threadIdx.x;
  if (c < nv) mref[c] = sqrt(ss[c] * inv_vol / (double)ne) + 1e-300;
}

// Features of element K (FP32 row of X, width ldx >= n_in, zero padding),
// optional normalised targets T[K][j] = z_K,j / s_K and scales s_K.
__global__ void k_mlp_features(const double* __restrict__ w, const double* __restrict__ r,
                               const double* __restrict__ z, const int64_t* __restrict__ nbr,
                               const double* __restrict__ mref, int nv, int nb, int nf, int64_t ne, double inv_sqrt_vol,
                               float* __restrict__ X, int ldx, float* __restrict__ T, double* __restrict__ s_out) {
  const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= ne) return;
  const int m = nv * nb;
  double ss = 0.0;
  for (int j = 0; j < m; ++j) {
    const double v = r[(int64_t)j * ne + K];
    ss += v * v;
  }
  const double s = sqrt(ss) + 1e-300;
  const double inv = 1.0 / s;
  float* x = X + K * ldx;
  for (int j = 0; j < m; ++j) x[j] = (float)(r[(int64_t)j * ne + K] * inv);
  for (int f = 0; f < nf; ++f) {
    const int64_t J = nbr[(int64_t)f * ne + K];
    for (int c = 0; c < nv; ++c) x[m + f * nv + c] = (float)(w[(int64_t)(c * nb) * ne + J] * inv_sqrt_vol / mref[c]);
  }
  for (int j = m + nf * nv; j < ldx; ++j) x[j] = 0.0f;
  if (T)
    for (int j = 0; j < m; ++j) T[K * m + j] = (float)(z[(int64_t)j * ne + K] * inv);
  if (s_out) s_out[K] = s;
}

// Xb[b][k] = bf16(X[row_b][k]) for k < n_in, 0 for n_in <= k < ldb and for rows b >= B (up to Bp)
__global__ void k_mlp_pack_rows(const float* __restrict__ X, int ldx, int n_in, const int64_t* __restrict__ rows,
                                int64_t B, int64_t Bp, unsigned short* __restrict__ Xb, int ldb) {
  const int64_t n = Bp * ldb;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / ldb;
    const int k = (int)(i - b * ldb);
    float v = 0.0f;
    if (b < B && k < n_in) {
      const int64_t src = rows ? rows[b] : b;
      v = X[src * ldx + k];
    }
    Xb[i] = f2bf(v);
  }
}

// C = A(MxK) * B(KxN), BF16 operands, FP32 accumulation; K % 32 == 0.
// A(m,k) = A[m*lda + k] (AT = false) or A[k*lda + m] (AT = true);
// B(k,n) = B[n*ldb + k] (BT = true) or B[k*ldb + n] (BT = false).
// Workgroup = 4 waves = 64x64 tile, each wave 32x32 = 2x2 MFMA tiles.
// Epilogues: 0 FP32 out (+bias), 1 BF16 relu(acc + bias), 2 BF16 acc masked by aux > 0.
template <bool AT, bool BT, int EPI>
__global__ __launch_bounds__(256) void k_gemm_bf16(int64_t M, int N, int64_t K, const unsigned short* __restrict__ A,
                                                   int64_t lda, const unsigned short* __restrict__ B, int64_t ldb,
                                                   void* __restrict__ out, int64_t ldo, const float* __restrict__ bias,
                                                   const unsigned short* __restrict__ aux) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t m0 = (int64_t)blockIdx.y * 64 + (wv >> 1) * 32;
  const int n0 = blockIdx.x * 64 + (wv & 1) * 32;
  const int lr = lane & 15, lk = (lane >> 4) * 8;
  f32x4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t k0 = 0; k0 < K; k0 += 32) {
    bf16x8 fa[2], fb[2];
    for (int t = 0; t < 2; ++t) {
      const int64_t m = m0 + t * 16 + lr;
      const int n = n0 + t * 16 + lr;
      for (int j = 0; j < 8; ++j) {
        const int64_t k = k0 + lk + j;
        unsigned short va = 0, vb = 0;
        if (m < M) va = AT ? A[k * lda + m] : A[m * lda + k];
        if (n < N) vb = BT ? B[(int64_t)n * ldb + k] : B[k * ldb + n];
        fa[t][j] = __builtin_bit_cast(__bf16, va);
        fb[t][j] = __builtin_bit_cast(__bf16, vb);
      }
    }
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + a * 16 + (lane >> 4) * 4 + r;
        const int n = n0 + b * 16 + lr;
        if (m >= M || n >= N) continue;
        float v = acc[a][b][r];
        if (EPI == 0) {
          static_cast<float*>(out)[m * ldo + n] = v + (bias ? bias[n] : 0.0f);
        } else if (EPI == 1) {
          v += bias[n];
          static_cast<unsigned short*>(out)[m * ldo + n] = f2bf(v > 0.0f ? v : 0.0f);
        } else {
          const float g = bf2f(aux[m * ldo + n]);
          static_cast<unsigned short*>(out)[m * ldo + n] = f2bf(g > 0.0f ? v : 0.0f);
        }
      }
}

// dY[b][j] = bf16(2 (Y - T) / (B n_out)) for j < n_out (0 up to ldd and for b >= B), loss partials
__global__ __launch_bounds__(256) void k_mlp_loss(const float* __restrict__ Y, int ldy, const float* __restrict__ T,
                                                  const int64_t* __restrict__ rows, int n_out, int64_t B, int64_t Bp,
                                                  unsigned short* __restrict__ dY, int ldd, double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  const double scale = 2.0 / ((double)B * n_out);
  const int64_t n = Bp * ldd;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int64_t b = i / ldd;
    const int j = (int)(i - b * ldd);
    float g = 0.0f;
    if (b < B && j < n_out) {
      const int64_t src = rows ? rows[b] : b;
      const double e = (double)Y[b * ldy + j] - (double)T[src * n_out + j];
      acc += e * e;
      g = (float)(scale * e);
    }
    dY[i] = f2bf(g);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_mlp_loss_final(const double* __restrict__ part, int np, double denom,
                                                        float* __restrict__ loss) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) a += part[i];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)(sh[0] / denom);
}

// g[n] = sum_b D[b][n] (FP32 accumulation over the batch), n < N
__global__ void k_colsum_bf16(const unsigned short* __restrict__ D, int ldd, int64_t B, int N, float* __restrict__ g) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float a = 0.0f;
  for (int64_t b = 0; b < B; ++b) a += bf2f(D[b * ldd + n]);
  g[n] = a;
}

// Adam on the flat FP32 parameters
__global__ void k_adam(int64_t n, float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// Row-major FP32 [rows][cols] block of the flat parameters -> padded BF16 [prow][pcol] (zeros outside)
__global__ void k_pack_weight(const float* __restrict__ W, int rows, int cols, unsigned short* __restrict__ Wb,
                              int prow, int pcol) {
  const int64_t n = (int64_t)prow * pcol;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / pcol), c = (int)(i - (int64_t)r * pcol);
    Wb[i] = (r < rows && c < cols) ? f2bf(W[(int64_t)r * cols + c]) : (unsigned short)0;
  }
}

__global__ void k_pack_bias(const float* __restrict__ b, int n, float* __restrict__ bp, int np) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) bp[i] = i < n ? b[i] : 0.0f;
}

// z[j*ne + K] = s_K * Y[K][j]
// z = s_K Y (add = 0) or z += s_K Y (add = 1; the learned correction on top
// of the block-Jacobi vector already in z)
__global__ void k_mlp_scatter(const float* __restrict__ Y, int ldy, const double* __restrict__ s, int m, int64_t ne,
                              double* __restrict__ z, int add) {
  const int64_t n = (int64_t)m * ne;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t K = i % ne;
    const int j = (int)(i / ne);
    const double y = s[K] * (double)Y[K * ldy + j];
    z[i] = add ? z[i] + y : y;
  }
}

}  // namespace

hipError_t launch_mlp_mref(const double* ss, int nv, int64_t ne, double inv_vol, double* mref, hipStream_t s) {
  k_mlp_mref<<<1, 64, 0, s>>>(ss, nv, ne, inv_vol, mref);
  return hipGetLastError();
}

hipError_t launch_mlp_features(const double* w, const double* r, const double* z, const int64_t* nbr,
                               const double* mref, int nv, int nb, int nf, int64_t ne, double inv_sqrt_vol, float* X,
                               int ldx, float* T, double* s_out, hipStream_t s) {
  k_mlp_features<<<(unsigned)((ne + 127) / 128), 128, 0, s>>>(w, r, z, nbr, mref, nv, nb, nf, ne, inv_sqrt_vol, X, ldx,
                                                               T, s_out);
  return hipGetLastError();
}

hipError_t launch_mlp_pack_rows(const float* X, int ldx, int n_in, const int64_t* rows, int64_t B, int64_t Bp,
                                unsigned short* Xb, int ldb, hipStream_t s) {
  k_mlp_pack_rows<<<grid_for(Bp * ldb), 256, 0, s>>>(X, ldx, n_in, rows, B, Bp, Xb, ldb);
  return hipGetLastError();
}

hipError_t launch_gemm_bf16(bool at, bool bt, int epi, int64_t M, int N, int64_t K, const unsigned short* A,
                            int64_t lda, const unsigned short* B, int64_t ldb, void* out, int64_t ldo,
                            const float* bias, const unsigned short* aux, hipStream_t s) {
  if (K % 32 != 0 || M < 0 || N < 0) return hipErrorInvalidValue;
  if (M == 0 || N == 0) return hipSuccess;
  const dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
#define DG_GEMM(AT_, BT_, E_)                                                                                     \
  if (at == AT_ && bt == BT_ && epi == E_) {                                                                      \
    k_gemm_bf16<AT_, BT_, E_><<<grid, 256, 0, s>>>(M, N, K, A, lda, B, ldb, out, ldo, bias, aux);                 \
    return hipGetLastError();                                                                                     \
  }
  DG_GEMM(false, true, 0)
  DG_GEMM(false, true, 1)
  DG_GEMM(false, false, 2)
  DG_GEMM(true, false, 0)
#undef DG_GEMM
  return hipErrorInvalidValue;
}

hipError_t launch_mlp_loss(const float* Y, int ldy, const float* T, const int64_t* rows, int n_out, int64_t B,
                           int64_t Bp, unsigned short* dY, int ldd, double* part, int npart, float* loss,
                           hipStream_t s) {
  k_mlp_loss<<<npart, 256, 0, s>>>(Y, ldy, T, rows, n_out, B, Bp, dY, ldd, part);
  k_mlp_loss_final<<<1, 256, 0, s>>>(part, npart, (double)B * n_out, loss);
  return hipGetLastError();
}

hipError_t launch_colsum_bf16(const unsigned short* D, int ldd, int64_t B, int N, float* g, hipStream_t s) {
  k_colsum_bf16<<<(unsigned)((N + 127) / 128), 128, 0, s>>>(D, ldd, B, N, g);
  return hipGetLastError();
}

hipError_t launch_adam(int64_t n, float* th, float* m, float* v, const float* g, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s) {
  k_adam<<<grid_for(n), 256, 0, s>>>(n, th, m, v, g, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_pack_weight(const float* W, int rows, int cols, unsigned short* Wb, int prow, int pcol,
                              hipStream_t s) {
  k_pack_weight<<<grid_for((int64_t)prow * pcol), 256, 0, s>>>(W, rows, cols, Wb, prow, pcol);
  return hipGetLastError();
}

hipError_t launch_pack_bias(const float* b, int n, float* bp, int np, hipStream_t s) {
  k_pack_bias<<<(unsigned)((np + 255) / 256), 256, 0, s>>>(b, n, bp, np);
  return hipGetLastError();
}

hipError_t launch_mlp_scatter(const float* Y, int ldy, const double* sc, int m, int64_t ne, double* z, int add,
                              hipStream_t s) {
  k_mlp_scatter<<<grid_for((int64_t)m * ne), 256, 0, s>>>(Y, ldy, sc, m, ne, z, add);
  return hipGetLastError();
}

}  // namespace dgk
