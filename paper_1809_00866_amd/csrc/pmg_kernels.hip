// Kernels of the p-multigrid preconditioner (Sec. 2.4): mode truncation and
// zero-padding between levels, the inherited coarse operators of eq. GalProj
// stored block-sparse, and the device-side bookkeeping of the fixed-count
// GMRES smoothers.
//
// Level vectors use the DOF layout of the library with the level's own mode
// count: idx(e, c, b) = (c*Nb_l + b)*ne + e.  With the hierarchical
// orthonormal basis the first Nb_l modes of the fine basis span the level's
// space, so restriction keeps them and prolongation pads with zeros.
//
// Coarse operator storage (BSR, one block row per element): slot 0 holds the
// diagonal block, slot 1 + f the coupling to the face neighbour f (order
// -x,+x,-y,+y,-z,+z); blocks are m x m column-major, laid out [slot][e][m*m],
// so slot 0 is the contiguous stack of diagonal blocks the block-Jacobi
// inversion reads.
#include <algorithm>

#include "dg_internal.h"

namespace dgk {

namespace {

__global__ void k_restrict(const double* __restrict__ f, int nbf, double* __restrict__ cv, int nbc, int nv,
                           int64_t ne) {
  const int64_t n = (int64_t)nv * nbc * ne;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i % ne;
    const int r = (int)(i / ne);
    const int c = r / nbc, b = r % nbc;
    cv[i] = f[((int64_t)c * nbf + b) * ne + e];
  }
}

// f += pad(cv) on the modes the coarse level has
__global__ void k_prolong_add(const double* __restrict__ cv, int nbc, double* __restrict__ f, int nbf, int nv,
                              int64_t ne) {
  const int64_t n = (int64_t)nv * nbc * ne;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i % ne;
    const int r = (int)(i / ne);
    const int c = r / nbc, b = r % nbc;
    f[((int64_t)c * nbf + b) * ne + e] += cv[i];
  }
}

// Slot of element K whose element carries colour `col` (the first such slot;
// later slots naming the same element keep zero blocks), or -1.
__device__ __forceinline__ int colour_slot(const int* color, const int64_t* nbr, int nf, int64_t ne, int64_t K,
                                           int col) {
  if (color[K] == col) return 0;
  for (int f = 0; f < nf; ++f) {
    const int64_t J = nbr[(int64_t)f * ne + K];
    if (color[J] != col) continue;
    bool dup = (J == K);
    for (int g = 0; g < f && !dup; ++g) dup = (nbr[(int64_t)g * ne + K] == J);
    return dup ? -1 : 1 + f;
  }
  return -1;
}

// Column l (coarse local index c*nbc + b) of the block of row K in the slot of
// the perturbed element: B[slot][K][l*m + r] = (G_0 P)_{K, r} for coarse rows r.
__global__ void k_extract_bsr(const double* __restrict__ Jv, const int* __restrict__ color, int col, int l,
                              const int64_t* __restrict__ nbr, int nf, int nbf, int nbc, int nv, int64_t ne,
                              double* __restrict__ B) {
  const int m = nv * nbc;
  const int64_t n = (int64_t)m * ne;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t K = i % ne;
    const int r = (int)(i / ne);
    const int s = colour_slot(color, nbr, nf, ne, K, col);
    if (s < 0) continue;
    const int c = r / nbc, b = r % nbc;
    B[((int64_t)s * ne + K) * m * m + (int64_t)l * m + r] = Jv[((int64_t)c * nbf + b) * ne + K];
  }
}

// Leading sub-blocks: B2[s][K](r2, j2) = B1[s][K](r1, j1), r = c*nb + b with b < nb2.
__global__ void k_truncate_bsr(const double* __restrict__ B1, int nb1, double* __restrict__ B2, int nb2, int nv,
                               int nslot, int64_t ne) {
  const int m1 = nv * nb1, m2 = nv * nb2;
  const int64_t n = (int64_t)nslot * ne * m2 * m2;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = i / ((int64_t)m2 * m2);
    const int q = (int)(i % ((int64_t)m2 * m2));
    const int j2 = q / m2, r2 = q % m2;
    const int j1 = (j2 / nb2) * nb1 + j2 % nb2, r1 = (r2 / nb2) * nb1 + r2 % nb2;
    B2[i] = B1[blk * m1 * m1 + (int64_t)j1 * m1 + r1];
  }
}

// y_K = sum_s B[s][K] x_{elem(K, s)}.  A row of the level operator is
// summed by CS threads (column slices: columns c, c+CS, c+2CS, ... of the
// (2d+1)*m gathered x values), each owning RPT consecutive rows (one vector
// load per column), and the CS partial sums are added in a fixed order.  The
// result depends on CS (summation order) but not on the workgroup size BS,
// which only sets how many element rows (BS / (CS m / RPT)) share a
// workgroup; the autotuner picks (BS, RPT, CS) per level.  The blocks are
// stored in S (FP64, or an FP32 copy for the reduced-precision smoothers);
// the sums are FP64.
template <class S, int RPT>
struct RowVec;  // RPT consecutive entries of a column, one load
template <>
struct RowVec<double, 1> {
  static __device__ __forceinline__ void ld(const double* p, double* o) { o[0] = p[0]; }
};
template <>
struct RowVec<double, 2> {
  static __device__ __forceinline__ void ld(const double* p, double* o) {
    const double2 v = *reinterpret_cast<const double2*>(p);
    o[0] = v.x;
    o[1] = v.y;
  }
};
template <>
struct RowVec<float, 1> {
  static __device__ __forceinline__ void ld(const float* p, double* o) { o[0] = p[0]; }
};
template <>
struct RowVec<float, 2> {
  static __device__ __forceinline__ void ld(const float* p, double* o) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    o[0] = v.x;
    o[1] = v.y;
  }
};
template <>
struct RowVec<float, 4> {
  static __device__ __forceinline__ void ld(const float* p, double* o) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
};

// part[element][slice][row] holds the slices' partial sums.
template <int BS, class S, int RPT, int CS>
__global__ __launch_bounds__(BS) void k_bsr_apply(const S* __restrict__ B, const int64_t* __restrict__ nbr,
                                                  int nf, int m, int R, int64_t ne, const double* __restrict__ x,
                                                  double* __restrict__ y) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int mr = m / RPT;          // row groups
  const int tpr = CS * mr;         // threads per element row; R element rows per workgroup
  const int ncol = (nf + 1) * m;
  double* xs = reinterpret_cast<double*>(smem);  // [R][ncol]
  double* part = xs + R * ncol;                  // [R][CS][m]
  const int64_t K0 = (int64_t)blockIdx.x * R;
  for (int t = threadIdx.x; t < R * ncol; t += BS) {
    const int rr = t / ncol, q = t - rr * ncol;
    const int64_t K = K0 + rr;
    if (K < ne) {
      const int s = q / m, j = q - s * m;
      const int64_t E = s == 0 ? K : nbr[(int64_t)(s - 1) * ne + K];
      xs[t] = x[(int64_t)j * ne + E];
    }
  }
  __syncthreads();
  const int rr = threadIdx.x / tpr, q = threadIdx.x - rr * tpr;
  const int cc = q / mr, ig = q - cc * mr;
  const int64_t K = K0 + rr;
  double a[RPT];
#pragma unroll
  for (int u = 0; u < RPT; ++u) a[u] = 0.0;
  if (rr < R && K < ne) {
    const double* xr = xs + rr * ncol;
#pragma unroll 8
    for (int col = cc; col < ncol; col += CS) {
      const int s = col / m, j = col - s * m;
      double v[RPT];
      RowVec<S, RPT>::ld(B + ((int64_t)s * ne + K) * m * m + (int64_t)j * m + ig * RPT, v);
      const double xc = xr[col];
#pragma unroll
      for (int u = 0; u < RPT; ++u) a[u] += v[u] * xc;
    }
  }
  if (rr < R)
#pragma unroll
    for (int u = 0; u < RPT; ++u) part[(rr * CS + cc) * m + ig * RPT + u] = a[u];
  __syncthreads();
  for (int t = threadIdx.x; t < R * m; t += BS) {
    const int r2 = t / m, i2 = t - r2 * m;
    const int64_t K2 = K0 + r2;
    const double* p = part + r2 * CS * m + i2;
    double acc = p[0];
#pragma unroll
    for (int k = 1; k < CS; ++k) acc += p[k * m];
    if (K2 < ne) y[(int64_t)i2 * ne + K2] = acc;
  }
}

// --- fixed-count GMRES bookkeeping (one thread; column j of the Hessenberg
// matrix, already orthogonalised, arrives in h1 + h2; ||w|| from partials) ---

__global__ void k_gmres_init(double* __restrict__ sc, int m) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double* gv = sc + kScG;
  for (int i = 0; i <= m; ++i) gv[i] = 0.0;
  gv[0] = sc[kScBeta];
  sc[kScFlag] = 0.0;
}

// ||w|| after orthogonalisation from the partial sums of w.w (one workgroup
// of 256 threads), then the Givens update of column j (thread 0).
__global__ __launch_bounds__(256) void k_norm_gmres_step(const double* __restrict__ partial, int np,
                                                         double* __restrict__ sc, int j, int m) {
  __shared__ double wsum[4];
  double a = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) a += partial[i];
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x != 0) return;
  sc[kScHn] = sqrt((wsum[0] + wsum[1]) + (wsum[2] + wsum[3]));
  double* R = sc + kScR + (int64_t)j * (m + 1);  // column j, rows 0..j+1
  double* cs = sc + kScCs;
  double* sn = sc + kScSn;
  double* gv = sc + kScG;
  const double w0 = sqrt(sc[kScH1 + j + 1]), hn = sc[kScHn];  // |w| before orthogonalisation
  for (int i = 0; i <= j; ++i) R[i] = sc[kScH1 + i] + sc[kScH2 + i];
  R[j + 1] = hn;
  // happy breakdown (or a zero column after one): later Krylov vectors are 0
  const bool brk = sc[kScFlag] != 0.0 || !(hn > 1e-14 * w0);
  sc[kScFlag] = brk ? 1.0 : 0.0;
  sc[kScInv] = brk ? 0.0 : 1.0 / hn;
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * R[i] + sn[i] * R[i + 1];
    R[i + 1] = -sn[i] * R[i] + cs[i] * R[i + 1];
    R[i] = t;
  }
  const double den = hypot(R[j], R[j + 1]);
  cs[j] = den > 0.0 ? R[j] / den : 1.0;
  sn[j] = den > 0.0 ? R[j + 1] / den : 0.0;
  R[j] = den;
  R[j + 1] = 0.0;
  gv[j + 1] = -sn[j] * gv[j];
  gv[j] = cs[j] * gv[j];
}

// y = R^-1 g (upper triangular, columns with a zero pivot give y = 0)
__global__ void k_gmres_backsolve(double* __restrict__ sc, int m) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double* R = sc + kScR;
  const double* gv = sc + kScG;
  double* y = sc + kScY;
  for (int i = m - 1; i >= 0; --i) {
    double a = gv[i];
    for (int l = i + 1; l < m; ++l) a -= R[(int64_t)l * (m + 1) + i] * y[l];
    const double d = R[(int64_t)i * (m + 1) + i];
    y[i] = d != 0.0 ? a / d : 0.0;
  }
}

// x *= s[0]
__global__ void k_scale_by(int64_t n, double* __restrict__ x, const double* __restrict__ s) {
  const double a = s[0];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] *= a;
}

unsigned grid_for(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

hipError_t launch_restrict(const double* f, int nbf, double* cv, int nbc, int nv, int64_t ne, hipStream_t s) {
  k_restrict<<<grid_for((int64_t)nv * nbc * ne), 256, 0, s>>>(f, nbf, cv, nbc, nv, ne);
  return hipGetLastError();
}

hipError_t launch_prolong_add(const double* cv, int nbc, double* f, int nbf, int nv, int64_t ne, hipStream_t s) {
  k_prolong_add<<<grid_for((int64_t)nv * nbc * ne), 256, 0, s>>>(cv, nbc, f, nbf, nv, ne);
  return hipGetLastError();
}

hipError_t launch_extract_bsr(const double* Jv, const int* color, int col, int l, const int64_t* nbr, int nf,
                              int nbf, int nbc, int nv, int64_t ne, double* B, hipStream_t s) {
  k_extract_bsr<<<grid_for((int64_t)nv * nbc * ne), 256, 0, s>>>(Jv, color, col, l, nbr, nf, nbf, nbc, nv, ne, B);
  return hipGetLastError();
}

hipError_t launch_truncate_bsr(const double* B1, int nb1, double* B2, int nb2, int nv, int nslot, int64_t ne,
                               hipStream_t s) {
  const int64_t m2 = (int64_t)nv * nb2;
  k_truncate_bsr<<<grid_for((int64_t)nslot * ne * m2 * m2), 256, 0, s>>>(B1, nb1, B2, nb2, nv, nslot, ne);
  return hipGetLastError();
}

namespace {

template <class S, int RPT, int CS>
hipError_t bsr_apply_shape(int bs, const S* B, const int64_t* nbr, int nf, int m, int64_t ne, const double* x,
                           double* y, hipStream_t s) {
  // element rows per workgroup: as many as the threads allow, within 64 KB of
  // LDS (at least one: bsr_shape_fits)
  const size_t per = ((size_t)(nf + 1) * m + (size_t)CS * m) * sizeof(double);
  const int R = std::min<int>(bs / (CS * (m / RPT)), (int)(65536 / per));
  const unsigned grid = (unsigned)((ne + R - 1) / R);
  const size_t lds = (size_t)R * per;
  switch (bs) {
    case 256: k_bsr_apply<256, S, RPT, CS><<<grid, 256, lds, s>>>(B, nbr, nf, m, R, ne, x, y); break;
    case 512: k_bsr_apply<512, S, RPT, CS><<<grid, 512, lds, s>>>(B, nbr, nf, m, R, ne, x, y); break;
    case 1024: k_bsr_apply<1024, S, RPT, CS><<<grid, 1024, lds, s>>>(B, nbr, nf, m, R, ne, x, y); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class S, int RPT>
hipError_t bsr_apply_rpt(const BsrShape& sh, const S* B, const int64_t* nbr, int nf, int m, int64_t ne,
                         const double* x, double* y, hipStream_t s) {
  switch (sh.cs) {
    case 1: return bsr_apply_shape<S, RPT, 1>(sh.bs, B, nbr, nf, m, ne, x, y, s);
    case 2: return bsr_apply_shape<S, RPT, 2>(sh.bs, B, nbr, nf, m, ne, x, y, s);
    case 4: return bsr_apply_shape<S, RPT, 4>(sh.bs, B, nbr, nf, m, ne, x, y, s);
    case 8: return bsr_apply_shape<S, RPT, 8>(sh.bs, B, nbr, nf, m, ne, x, y, s);
    default: return hipErrorInvalidValue;
  }
}

template <class S>
hipError_t bsr_apply(const BsrShape& sh, const S* B, const int64_t* nbr, int nf, int m, int64_t ne,
                     const double* x, double* y, hipStream_t s) {
  if (ne < 1 || !bsr_shape_fits(sh, m, sizeof(S), nf)) return hipErrorInvalidValue;
  const int rpt = sh.rpt ? sh.rpt : bsr_widest_rpt(m, sizeof(S));
  switch (rpt) {
    case 1: return bsr_apply_rpt<S, 1>(sh, B, nbr, nf, m, ne, x, y, s);
    case 2: return bsr_apply_rpt<S, 2>(sh, B, nbr, nf, m, ne, x, y, s);
    case 4:
      if constexpr (sizeof(S) == 4) return bsr_apply_rpt<S, 4>(sh, B, nbr, nf, m, ne, x, y, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

__global__ void k_to_f32(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

}  // namespace

bool bsr_shape_fits(const BsrShape& sh, int m, size_t elem, int nf) {
  if (m < 1 || nf < 0 || (elem != 4 && elem != 8)) return false;
  if (sh.bs != 256 && sh.bs != 512 && sh.bs != 1024) return false;
  if (sh.cs != 1 && sh.cs != 2 && sh.cs != 4 && sh.cs != 8) return false;
  const int rpt = sh.rpt ? sh.rpt : bsr_widest_rpt(m, elem);
  if (rpt != 1 && rpt != 2 && !(rpt == 4 && elem == 4)) return false;
  if (m % rpt != 0) return false;
  const size_t per = ((size_t)(nf + 1) * m + (size_t)sh.cs * m) * sizeof(double);
  return sh.bs >= sh.cs * (m / rpt) && per <= 65536;
}

hipError_t launch_bsr_apply(const BsrShape& sh, const double* B, const int64_t* nbr, int nf, int m, int64_t ne,
                            const double* x, double* y, hipStream_t s) {
  return bsr_apply<double>(sh, B, nbr, nf, m, ne, x, y, s);
}

hipError_t launch_bsr_apply_f32(const BsrShape& sh, const float* B, const int64_t* nbr, int nf, int m, int64_t ne,
                                const double* x, double* y, hipStream_t s) {
  return bsr_apply<float>(sh, B, nbr, nf, m, ne, x, y, s);
}

hipError_t launch_to_f32(const double* x, float* y, int64_t n, hipStream_t s) {
  k_to_f32<<<grid_for(n), 256, 0, s>>>(x, y, n);
  return hipGetLastError();
}

hipError_t launch_gmres_init(double* sc, int m, hipStream_t s) {
  k_gmres_init<<<1, 64, 0, s>>>(sc, m);
  return hipGetLastError();
}

hipError_t launch_norm_gmres_step(const double* partial, int np, double* sc, int j, int m, hipStream_t s) {
  k_norm_gmres_step<<<1, 256, 0, s>>>(partial, np, sc, j, m);
  return hipGetLastError();
}

hipError_t launch_gmres_backsolve(double* sc, int m, hipStream_t s) {
  k_gmres_backsolve<<<1, 64, 0, s>>>(sc, m);
  return hipGetLastError();
}

hipError_t launch_scale_by(int64_t n, double* x, const double* sc, hipStream_t s) {
  k_scale_by<<<grid_for(n), 256, 0, s>>>(n, x, sc);
  return hipGetLastError();
}

}  // namespace dgk
